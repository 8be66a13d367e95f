#!/usr/bin/env python3
"""Benchmark of the ensemble-PCG hot path on one MI355X.

Workload: -div(a(x) K(y) grad u) = 1 on a 512 x 512 interior grid (262,144
unknowns), nine-point scheme, FP64, d = 4 parameters (anisotropy, angle, two
a(x) modes, amp 0.4); samples are the nodes of an adaptive piecewise-linear
sparse grid, levels 1-5, 1024-sample budget, refined on G(y) = ||u||^2;
ensembles of S = 32 grouped by the sparse-grid surrogate of iteration counts;
Jacobi-PCG, rtol 1e-8.  One step = the whole adaptive pass: per level,
grouping, ensemble assembly, ensemble PCG solves, G(y), refinement.

Prints one JSON line.  `value` is sample-solves/s of the whole pass (real
samples / wall time of the step, inputs generated on the device).
`roofline` is for the dominant kernel, the fused direction-update + SpMV
kernel, timed live with HIP events on the solver's stream, beside two
streaming references measured in the same run (the STREAM triad and the
kernel's own mix of eight reads and three writes) and the same kernel's
rate at 1024^2, where no cache holds its working set.  `cpu_baseline` is
the oracle on the benchmark's first 32 samples in solve order (found by the
oracle itself, before the GPU run), with the GPU's time on the ensembles
holding the same samples beside it.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_GRID = 512
D = 4
AMP = 0.4
RTOL = 1e-8
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per member-row.  The fused kernel reads five matrix
# values (C, E, N, NE, NW; the other four are the neighbours' by symmetry),
# r, p_old, x and writes p, q, x: 11 FP64 words (15 with --full-stencil,
# which reads all nine).  A Jacobi-PCG iteration adds the update kernel's
# 4 words.  A Jacobi-Chebyshev-4 iteration is 37 words (53 with nine): the
# fused PCG step (11), the residual update fused with the first Chebyshev
# step (reads r, q, diagonal and four more matrix values, writes r, z: 9),
# the second step (five matrix values, z_1, r; writes z_2: 8; the increment
# is formed from the iterates, not stored) and the last (five matrix
# values, z_2, r, z_1; writes z_3: 9).
FULL_STENCIL = False
FUSED_BYTES = 11 * 8
ITER_BYTES = 15 * 8
CHEB_ITER_BYTES = 37 * 8


def set_byte_model(full: bool) -> None:
    global FULL_STENCIL, FUSED_BYTES, ITER_BYTES, CHEB_ITER_BYTES
    FULL_STENCIL = full
    extra = 4 if full else 0
    FUSED_BYTES = (11 + extra) * 8
    ITER_BYTES = (15 + extra) * 8
    CHEB_ITER_BYTES = (37 + 4 * extra) * 8


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "stencil_pcg_512x512_S32_traffic.json")


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "common.h", "device.h"):
        with open(os.path.join(ROOT, "paper_1705_02003_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(S: int):
    """HBM bytes per launch of the fused kernel from the committed counter
    record, or None if it was taken on other kernel source or another width."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if S != 32 or rec.get("source_sha256_16") != kernel_source_hash():
        return None
    if bool(rec.get("full_stencil", False)) != FULL_STENCIL:
        return None
    return rec.get("traffic_bytes_per_launch")


# ------------------------------------------------------------ CPU baseline
def _oracle_one(y):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        import numpy as np
        from oracle import pcg, problem
        A, b, diag = problem.assemble(np.asarray(y), N_GRID, 0, AMP)
        t = time.perf_counter()
        x, I, st, _ = pcg.pcg(A, b, diag, RTOL, 20000)
        return time.perf_counter() - t, int(I), int(st), float(x @ x)


def run_order(res):
    """Ids of the run's real samples in the order the GPU solved them: level
    by level, ensemble by ensemble (level 1 in generation order, later levels
    in the surrogate's ascending predicted-iteration order), each sample once."""
    out, seen, off = [], set(), 0
    for lvl in res.levels:
        for g in lvl.groups:
            for i in g:
                k = off + int(i)
                if k not in seen:
                    seen.add(k)
                    out.append(k)
        off += lvl.n_samples
    return out


def cpu_baseline(procs: int, count: int, S: int):
    """The oracle (per-sample FP64 Jacobi-PCG, one process per core, BLAS on
    one thread) on the benchmark's first `count` samples in solve order,
    found by the oracle itself before the GPU is touched (forked workers):
    the level-1 grid is solved, the oracle's refinement of it on G = ||u||^2
    gives level 2, and the oracle's surrogate of the level-1 counts orders
    level 2 into ensembles of S; the first samples of that order follow."""
    import numpy as np
    from oracle import sparse_grid as sg
    ctx = mp.get_context("fork")          # no GPU state exists yet in this process
    lvl1 = sg.full_grid(D, 1)
    t0 = time.perf_counter()
    with ctx.Pool(procs) as pool:
        out1 = pool.map(_oracle_one, [list(sg.coords(nd)) for nd in lvl1])
        print(f"[bench] oracle: level 1 ({len(lvl1)} samples) in {time.perf_counter() - t0:.1f} s",
              flush=True)
        lvl2 = sg.refine(lvl1, [o[3] for o in out1], 1, 1e-3, 1024)
        groups, _ = sg.group_samples(lvl1, [float(o[1]) for o in out1],
                                     np.array([sg.coords(nd) for nd in lvl2]), S)
        order = []
        for g in groups:
            for i in g:
                if i not in order:
                    order.append(i)
        more = [lvl2[i] for i in order[:max(0, count - len(lvl1))]]
        out2 = pool.map(_oracle_one, [list(sg.coords(nd)) for nd in more])
    wall = time.perf_counter() - t0
    out = out1 + out2
    ys = np.array([sg.coords(nd) for nd in lvl1 + more])
    its = [o[1] for o in out]
    solve_s = sum(o[0] for o in out)
    return {
        "value": round(len(ys) / wall, 4),
        "unit": "sample-solves/s",
        "cores": procs,
        "kind": "oracle",
        "ms_per_iteration": round(1e3 * solve_s / sum(its), 3),
        "sample": (f"the benchmark's first {len(ys)} samples in its solve order (the level-1 grid, "
                   f"then level-2 nodes in surrogate order, both derived by the oracle), FP64 "
                   f"scipy Jacobi-PCG solves on {procs} processes at {N_GRID}x{N_GRID}, rtol {RTOL}; "
                   f"iterations {min(its)}-{max(its)}; wall {wall:.1f} s"),
    }, ys


def gpu_same_samples(res, ids, S, opts):
    """GPU time of the ensembles that hold the given samples, solved as the
    run solved them (assembly included): the GPU side of the CPU baseline's
    comparison on the same samples."""
    import torch
    from paper_1705_02003_amd import ensemble as E
    want = set(ids)
    prob = E.Problem(N_GRID, D, 0, AMP)
    ws = E.workspace(prob, S, opts)
    jobs, off = [], 0
    for lvl in res.levels:
        for g in lvl.groups:
            ks = [off + int(i) for i in g]
            if want & set(ks):
                jobs.append(ks)
        off += lvl.n_samples
    covered = len(set(k for ks in jobs for k in ks))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for ks in jobs:
        V, b = E.assemble(prob, res.y[ks])
        E.solve(prob, V, b, opts, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    return {"value": round(covered / dt, 3), "unit": "sample-solves/s", "ensembles": len(jobs),
            "samples_solved": covered, "seconds": round(dt, 3)}


# ------------------------------------------------------------ GPU parts
def s1_comparison(res, S, opts, n_groups=2):
    """Solve the samples of the last level's first ensembles alone (S = 1) and
    as the S-wide ensembles they belong to; same samples, same GPU."""
    import numpy as np
    import torch
    from paper_1705_02003_amd import ensemble as E
    lvl = res.levels[-1]
    offset = sum(r.n_samples for r in res.levels[:-1])
    groups = lvl.groups[:n_groups]
    ys = res.y[offset:offset + lvl.n_samples]
    prob = E.Problem(N_GRID, D, 0, AMP)
    ws1 = E.workspace(prob, 1, opts)
    wsS = E.workspace(prob, S, opts)
    ids = sorted(set(int(i) for g in groups for i in g))

    def run_S():
        for g in groups:
            V, b = E.assemble(prob, torch.tensor(ys[g], dtype=torch.float64, device="cuda"))
            E.solve(prob, V, b, opts, ws=wsS)

    def run_1():
        its = []
        for i in ids:
            V, b = E.assemble(prob, torch.tensor(ys[i:i + 1], dtype=torch.float64, device="cuda"))
            its.append(E.solve(prob, V, b, opts, ws=ws1).iters[0])
        return its

    run_1()                                   # warm the S = 1 path
    torch.cuda.synchronize()
    t = time.perf_counter()
    run_S()
    torch.cuda.synchronize()
    tS = time.perf_counter() - t
    t = time.perf_counter()
    its1 = run_1()
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t
    return {"samples": len(ids), "S": S, "seconds_S": round(tS, 4), "seconds_S1": round(t1, 4),
            "sample_solves_per_s_S": round(len(ids) / tS, 3),
            "sample_solves_per_s_S1": round(len(ids) / t1, 3),
            "speedup_vs_S1": round(t1 / tS, 3),
            "iters_S1": [int(min(its1)), int(max(its1))]}


def measure_streams(gib: float = 1.0, reps: int = 5) -> dict:
    """Achievable HBM bandwidth: the library's STREAM triad (c = a + s b) and
    the solver step's mix of eight reads and three writes (ens_stream_mix),
    on arrays of `gib` GiB each, carved from one buffer and offset by 4 KiB
    (as the solver's matrix slots and vectors are); best of `reps` launches."""
    import torch
    from paper_1705_02003_amd import ensemble as E
    n = int(gib * (1 << 30)) // 8
    stride = ((n + 31) // 32) * 32 + 512
    buf = torch.empty(14 * stride, dtype=torch.float64, device="cuda")
    buf.fill_(1.0)
    src, dst = buf[:8 * stride], buf[8 * stride:]

    def best(fn):
        fn()
        torch.cuda.synchronize()
        out = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            dt = e0.elapsed_time(e1) * 1e-3
            out = dt if out is None else min(out, dt)
        return out

    a, b, c = buf[:n], buf[stride:stride + n], buf[2 * stride:2 * stride + n]
    t_triad = best(lambda: E.stream_triad(a, b, c, 0.5))
    t_mix = best(lambda: E.stream_mix(src, dst, stride, n, 8, 3))
    del buf
    torch.cuda.empty_cache()
    return {"triad_GBs": round(3 * n * 8 / t_triad / 1e9, 1),
            "mix_8r3w_GBs": round(11 * n * 8 / t_mix / 1e9, 1),
            "array_GiB": gib, "offset_bytes": (stride - n) * 8,
            "kernels": "ens_stream_triad, ens_stream_mix(8 reads, 3 writes)"}


def measure_triad(gib: int = 4, reps: int = 5) -> dict:
    """The triad alone (kept for --mode kernel): see measure_streams."""
    r = measure_streams(gib, reps)
    return {"GBs": r["triad_GBs"], "array_GiB": gib, "kernel": "ens_stream_triad"}


def fused_kernel_rate(n: int, S: int, iters: int = 40) -> dict:
    """The fused Jacobi step (direction update + nine-point product) on an
    n x n grid at width S with the benchmark's coefficient model, timed with
    HIP events over a fixed-iteration solve: at 1024^2 and S = 32 its working
    set (about 3.8 GB) is far beyond the 256 MB Infinity Cache, so this rate
    is an HBM rate."""
    import torch
    import workloads
    from paper_1705_02003_amd import ensemble as E
    prob = E.Problem(n, D, 0, AMP)
    V, b = E.assemble(prob, workloads.uniform_samples(1, S, D))
    opts = E.SolverOptions(rtol=0.0, max_iter=iters, time_spmv=True, full_stencil=FULL_STENCIL)
    ws = E.workspace(prob, S, opts)
    E.solve(prob, V, b, opts, ws=ws)
    r = E.solve(prob, V, b, opts, ws=ws)
    us = 1e3 * r.stats["spmv_ms"] / max(1, r.stats["spmv_timed"])
    gbs = prob.rows * S * FUSED_BYTES / (us * 1e-6) / 1e9
    del V, b, ws
    torch.cuda.empty_cache()
    return {"grid": f"{n}x{n}", "S": S, "avg_launch_us": round(us, 2), "achieved": round(gbs, 1),
            "frac": round(gbs / HBM_PEAK_GBS, 4), "timed_launches": r.stats["spmv_timed"]}


def device_info() -> dict:
    import subprocess
    import torch
    props = torch.cuda.get_device_properties(0)
    info = {"name": torch.cuda.get_device_name(0), "arch": getattr(props, "gcnArchName", ""),
            "compute_units": props.multi_processor_count,
            "memory_GiB": round(props.total_memory / 2**30, 1)}
    try:
        out = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True,
                             timeout=20).stdout
        clocks = [l.strip() for l in out.splitlines() if "sclk" in l or "mclk" in l]
        info["clocks"] = clocks[:4]
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def su_mode(args) -> int:
    """Perfect grouping (the MI355X analogue of the paper's Fig. 1): S copies
    of one sample y = (-1, 0, 0, 0) (isotropic, a = 1) at 512x512, Jacobi-PCG,
    rtol 1e-8, for S = 1, 2, ..., 64.  SU(S) = S t(1) / t(S), t the median of
    three solves (assembly excluded).  At S = 1 the working set (~30 MB)
    fits the 256 MB Infinity Cache, so its bandwidth is not an HBM figure."""
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    y0 = np.array([-1.0, 0.0, 0.0, 0.0])
    rows = su_rows(None, None, (1, 2, 4, 8, 16, 32, 64), y0, verbose=True)
    print(json.dumps({"mode": "su", "workload": "identical-samples-512x512", "y": y0.tolist(),
                      "rows": rows}), flush=True)
    return 0


def su_rows(prob, opts, S_list, y0, verbose=False) -> list:
    """Median solve time of S identical samples y0 for each S in S_list (the
    first entry must be 1) and SU(S) = S t(1) / t(S); prob / opts default to
    the benchmark's 512^2 problem and Jacobi at rtol 1e-8."""
    import numpy as np
    import torch
    import workloads
    from paper_1705_02003_amd import ensemble as E
    prob = prob or E.Problem(N_GRID, D, 0, AMP)
    opts = opts or E.SolverOptions(rtol=RTOL, full_stencil=FULL_STENCIL)
    # Jacobi iteration bytes per member-row (3-D: 26 words, 39 with all 27 values)
    it_bytes = ITER_BYTES if prob.dim == 2 else (39 if FULL_STENCIL else 26) * 8
    rows, t1 = [], None
    for S in S_list:
        y = torch.tensor(workloads.identical_samples(y0, S), dtype=torch.float64, device="cuda")
        V, b = E.assemble(prob, y)
        ws = E.workspace(prob, S, opts)
        E.solve(prob, V, b, opts, ws=ws)
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = E.solve(prob, V, b, opts, ws=ws)
            ts.append(time.perf_counter() - t)
        t = float(np.median(ts))
        t1 = t if S == 1 else t1
        rows.append({"S": S, "seconds": round(t, 5), "iters": int(r.ens_iters),
                     "sample_solves_per_s": round(S / t, 2), "SU": round(S * t1 / t, 3),
                     "iteration_alg_GBs": round(r.ens_iters * prob.rows * S * it_bytes / t / 1e9, 1)})
        if verbose:
            print(json.dumps(rows[-1]), flush=True)
        del V, b, ws
    return rows


def table_mode(args) -> int:
    """The MI355X analogue of the paper's Tables 2-3 (Section 4) on the
    benchmark's adaptive sample set: for each S and the groupings "its"
    (ascending true counts, hypothetical), "sur" (surrogate), "par"
    (parameter-based) and "nat" (generation order), the per-level cost ratios
    R_l, the total R, the measured speed-up (time of every linear solve done
    alone, S = 1, over the time of the ensemble solves; the assemblies'
    device time excluded from both) and the predicted speed-up SU(S) / R from
    the identical-sample curve.  Also the quantity of interest E[G^] after
    each level.

    --dim 3: the same for the paper's own 3-D test problem (32^3 trilinear
    cells, d = 4, the paper's Test 1 settings: tau 1e-3, at most 2000 samples,
    up to 8 levels, solver tolerance 1e-7), SU(S) from S copies of y = 0;
    with --test 2 the paper's Test 2 (a_hat(y) in {1, 100, 10} banded by
    |y|, the same settings; Table 3's analogue); --precond picks the
    preconditioner (Jacobi by default; multigrid is the paper's kind)."""
    import numpy as np
    import torch
    import workloads
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq
    torch.cuda.set_device(0)
    S_list = tuple(int(v) for v in args.S_list.split(","))
    if args.dim == 3:
        w = workloads.FE3D_32 if args.test == 1 else workloads.FE3D_32_TEST2
        prob = E.Problem(w.n, w.d, w.eps_model, dim=3)
        opts = E.SolverOptions(precond=args.precond, rtol=w.rtol, max_iter=w.max_iter,
                               full_stencil=FULL_STENCIL)
        res = uq.adaptive(prob, args.S, budget=2000, max_level=8, tau_rel=1e-3,
                          strategy="surrogate", opts=opts, perm_seed=1)
        y0, workload = np.zeros(w.d), "adaptive-sg-" + w.name
    else:
        prob = E.Problem(N_GRID, D, 0, AMP)
        opts = E.SolverOptions(rtol=RTOL, max_iter=20000, full_stencil=FULL_STENCIL)
        res = uq.adaptive(prob, args.S, budget=args.budget, max_level=5, tau_rel=1e-3,
                          strategy="surrogate", opts=opts, perm_seed=1)
        y0, workload = np.array([-1.0, 0.0, 0.0, 0.0]), "adaptive-sg-512x512-d4"
    print(f"[bench] adaptive run: levels {[l.n_samples for l in res.levels]}, "
          f"E[G] by level {[l.qoi_mean for l in res.levels]}", flush=True)
    # SU at every width the varying-width grouping may choose from (any S
    # from 1 to 64 runs; these 15 cover the curve), the fixed widths included
    curve = su_rows(prob, opts, (1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 32, 40, 48, 56, 64), y0)
    su = {r["S"]: r["SU"] for r in curve}
    print(f"[bench] SU(S): {su}", flush=True)
    # seconds per ensemble iteration at each width, from the same curve
    widths = [r["S"] for r in curve]
    iter_s = [r["seconds"] / r["iters"] for r in curve]
    seq = uq.time_groupings(prob, res, 1, opts, strategies=("natural",))["natural"]
    print(f"[bench] every sample alone: {seq}", flush=True)
    rows = []
    names = (("its", "its"), ("surrogate", "sur"), ("param", "par"), ("natural", "nat"))
    for S in S_list:
        costs = uq.grouping_costs(res, S)
        times = uq.time_groupings(prob, res, S, opts, strategies=("surrogate", "param", "natural"))
        for key, name in names:
            t = times.get(key)
            row = {"I": name, "S": S, "R_levels": costs[key]["R_levels"],
                   "R": round(costs[key]["R"], 3),
                   "speedup": round(seq["solve_seconds"] / t["solve_seconds"], 2) if t else None,
                   "predicted": round(su[S] / costs[key]["R"], 2),
                   "solve_seconds": t["solve_seconds"] if t else None}
            rows.append(row)
            print(json.dumps(row), flush=True)
    # ensembles of varying width (Section 5): least predicted time per level
    per = uq.variable_groups(res, widths, iter_s)
    vc = uq.variable_costs(res, per)
    t = uq.time_groupings(prob, res, 64, opts, strategies=("variable",),
                          extra={"variable": per})["variable"]
    its = res.iters
    pred_t = iter_s[0] * float(its.sum())
    var_t = sum(sum(iter_s[widths.index(len(g))] * int(it[np.asarray(g)].max()) for g in gs)
                for gs, it in zip(per, (r.iters for r in res.levels)))
    row = {"I": "var", "S": "1-64", "R_levels": vc["R_levels"], "R": round(vc["R"], 3),
           "speedup": round(seq["solve_seconds"] / t["solve_seconds"], 2),
           "predicted": round(pred_t / var_t, 2), "solve_seconds": t["solve_seconds"],
           "widths": vc["widths"]}
    rows.append(row)
    print(json.dumps(row), flush=True)
    print(json.dumps({"mode": "table", "workload": workload,
                      "samples": len(res.y), "levels": [l.n_samples for l in res.levels],
                      "qoi_mean_levels": [l.qoi_mean for l in res.levels],
                      "SU": su, "sequential": seq, "rows": rows}), flush=True)
    return 0


def grouping_mode(args) -> int:
    """GPU time of each grouping strategy on the samples of one adaptive run
    of the benchmark workload (the surrogate run itself is untimed here)."""
    import torch
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq
    torch.cuda.set_device(0)
    prob = E.Problem(N_GRID, D, 0, AMP)
    opts = E.SolverOptions(rtol=RTOL, max_iter=20000, full_stencil=FULL_STENCIL)
    res = uq.adaptive(prob, args.S, budget=args.budget, max_level=5, tau_rel=1e-3,
                      strategy="surrogate", opts=opts, perm_seed=1)
    print(f"[bench] adaptive run: {len(res.y)} samples", flush=True)
    out = {"mode": "grouping", "workload": "adaptive-sg-512x512-d4", "samples": len(res.y)}
    for S in (args.S, 16) if args.S != 16 else (16,):
        costs = uq.grouping_costs(res, S)
        times = uq.time_groupings(prob, res, S, opts)
        out[f"S{S}"] = {k: {**times[k], "R": round(costs[k]["R"], 4)} for k in times}
        print(json.dumps({f"S{S}": out[f"S{S}"]}), flush=True)
    print(json.dumps(out), flush=True)
    return 0


def kernel_mode(args) -> int:
    """One S-wide ensemble solved for a fixed number of iterations (rtol 0) in
    the default launch configuration, then a plain 1 GiB device-to-device
    copy whose counter readings calibrate FETCH_SIZE / WRITE_SIZE.  Jacobi:
    the benchmark's coefficient model on the --grid (default 512^2) grid;
    --precond chebyshev: the Chebyshev workload's (d = 8, eps down to 1e-3),
    degree 4.  Prints one JSON line with the measured times."""
    import torch
    import workloads
    from paper_1705_02003_amd import ensemble as E
    if args.precond == "multigrid":
        print("--mode kernel runs the 2-D model: --precond jacobi or chebyshev", file=sys.stderr)
        return 2
    torch.cuda.set_device(0)
    n = args.grid
    if args.precond == "chebyshev":
        w = workloads.CHEB_1024
        prob = E.Problem(n, w.d, w.eps_model, w.amp)
        y = workloads.uniform_samples(w.seed, args.S, w.d)
        words = CHEB_ITER_BYTES // 8
    else:
        prob = E.Problem(n, D, 0, AMP)
        y = workloads.uniform_samples(1, args.S, D)
        words = ITER_BYTES // 8
    V, b = E.assemble(prob, y)
    opts = E.SolverOptions(precond=args.precond, rtol=0.0, max_iter=args.iters, time_spmv=True,
                           full_stencil=FULL_STENCIL)
    ws = E.workspace(prob, args.S, opts)
    E.solve(prob, V, b, opts, ws=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = E.solve(prob, V, b, opts, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    # achievable bandwidth: a plain device copy and the library's streams
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_bytes = src.numel() * 8
    copy_gbs = 2 * copy_bytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    streams = measure_streams()
    us = 1e3 * r.stats["spmv_ms"] / max(1, r.stats["spmv_timed"])
    rows = prob.rows * args.S
    print(json.dumps({"mode": "kernel", "grid": f"{n}x{n}", "precond": args.precond, "S": args.S,
                      "iterations": args.iters,
                      "fused_avg_us": round(us, 2),
                      "fused_alg_GBs": round(rows * FUSED_BYTES / (us * 1e-6) / 1e9, 1),
                      "iteration_us": round(1e6 * dt / args.iters, 2),
                      "iteration_words_per_member_row": words,
                      "iteration_alg_GBs": round(rows * words * 8 * args.iters / dt / 1e9, 1),
                      "fused_alg_bytes": rows * FUSED_BYTES,
                      "copy_bytes_each_way": copy_bytes,
                      "stream_copy_GBs": round(copy_gbs, 1), **streams,
                      "tile_lines": r.stats["tile_lines"], "groups": r.stats["spmv_groups"]}),
          flush=True)
    return 0


def adjoint_mode(args) -> int:
    """Differentiation workload: 512x512, d = 6, 512 uniform samples (seed 4)
    in ensembles of S; forward ensemble PCG + QoI, then the adjoint ensemble
    PCG + dQ/dy kernel through EnsembleQoI.  The first ensemble's gradient is
    checked against central differences (h = 1e-6, forward solves at rtol
    1e-13, all members perturbed at once)."""
    import numpy as np
    import torch
    import workloads
    from paper_1705_02003_amd import autograd as A
    from paper_1705_02003_amd import ensemble as E
    torch.cuda.set_device(0)
    w = workloads.ADJOINT_512
    prob = E.Problem(w.n, w.d, w.eps_model, w.amp)
    ys = workloads.uniform_samples(w.seed, w.n_samples, w.d)
    S = args.S
    n_ens = args.ensembles or (w.n_samples // S)
    opts = E.SolverOptions(rtol=w.rtol)
    fwd = bwd = 0.0
    grads, fits, bits = [], [], []
    for k in range(n_ens):
        y = torch.tensor(ys[k * S:(k + 1) * S], dtype=torch.float64, device="cuda",
                         requires_grad=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        Q = A.EnsembleQoI.apply(y, prob, opts)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Q.sum().backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fwd += t1 - t
        bwd += t2 - t1
        grads.append(y.grad.cpu().numpy())
        print(f"[bench] adjoint ensemble {k}: forward {t1 - t:.2f} s, backward {t2 - t1:.2f} s",
              flush=True)
    y0 = torch.tensor(ys[:S], dtype=torch.float64, device="cuda")
    fd = A.central_difference(prob, y0, 1e-6, E.SolverOptions(rtol=1e-13))
    scale = np.maximum(np.abs(fd), 1e-2 * np.abs(fd).max(axis=1, keepdims=True))
    errs = {}
    for rtol, g0 in ((w.rtol, grads[0]), (1e-10, None)):
        if g0 is None:
            yt = y0.clone().requires_grad_(True)
            A.EnsembleQoI.apply(yt, prob, E.SolverOptions(rtol=rtol)).sum().backward()
            g0 = yt.grad.cpu().numpy()
        errs[f"{rtol:g}"] = {"componentwise": float(np.max(np.abs(g0 - fd) / scale)),
                             "normwise": float(np.max(np.abs(g0 - fd)) / np.abs(fd).max())}
    out = {"mode": "adjoint", "workload": w.name, "S": S, "ensembles": n_ens,
           "samples": n_ens * S, "forward_s": round(fwd, 3), "backward_s": round(bwd, 3),
           "sample_gradients_per_s": round(n_ens * S / (fwd + bwd), 3),
           "fd_check": {"h": 1e-6, "fd_rtol": 1e-13, "max_rel_err_by_solve_rtol": errs,
                        "componentwise": "|g - fd| / max(|fd|, 1e-2 max_j |fd_j|)",
                        "normwise": "max |g - fd| / max |fd| (per member row)"}}
    print(json.dumps(out), flush=True)
    return 0


def cheb_mode(args) -> int:
    """1024x1024, d = 8, degree-4 Jacobi-Chebyshev: the full level-2 sparse
    grid (145 nodes) is solved to build the iteration surrogate, the 4096
    uniform samples (seed 2) are ordered by it into ensembles of S, and
    ensembles spread evenly over that order are solved."""
    import numpy as np
    import torch
    import workloads
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq
    torch.cuda.set_device(0)
    w = workloads.CHEB_1024
    prob = E.Problem(w.n, w.d, w.eps_model, w.amp)
    ys = workloads.uniform_samples(w.seed, w.n_samples, w.d)
    S = args.S
    ng = (w.n_samples + S - 1) // S
    k = ng if args.all_ensembles else (args.ensembles or 4)
    sel = sorted(set(int(v) for v in np.linspace(0, ng - 1, k).round()))
    opts = E.SolverOptions(precond="chebyshev", rtol=w.rtol, max_iter=w.max_iter, time_spmv=True,
                           full_stencil=FULL_STENCIL)
    def progress(done, total):
        if done % 8 == 0 or done == total:
            print(f"[bench] {done}/{total} ensembles solved", flush=True)

    res = uq.nonadaptive(prob, S, ys, 2, opts, solve_groups=sel, progress=progress)
    solved = [i for g in res.groups[sel] for i in g]
    real = sorted(set(solved))
    its = res.iters[real]
    us = 1e3 * res.spmv_ms / max(1, res.spmv_launches)
    rows = prob.rows * S
    out = {"mode": "cheb", "workload": w.name, "S": S, "ensembles_solved": sel,
           "samples_solved": len(real), "train_samples": len(res.train_iters),
           "train_seconds": round(res.train_seconds, 2), "solve_seconds": round(res.solve_seconds, 2),
           "sample_solves_per_s": round(len(real) / res.solve_seconds, 3),
           "iters_train": [int(res.train_iters.min()), int(res.train_iters.max())],
           "iters_solved": [int(its.min()), int(its.max())], "ens_iters": res.ens_iters,
           "R_solved": round(S * sum(res.ens_iters) / float(its.sum()), 4),
           "fused_avg_us": round(us, 2),
           "fused_alg_GBs": round(rows * FUSED_BYTES / (us * 1e-6) / 1e9, 1),
           "iteration_alg_GBs": round(sum(res.ens_iters) * rows * CHEB_ITER_BYTES / res.solve_seconds / 1e9, 1)}
    if len(real) == w.n_samples:
        out["grouping"] = grouping_costs(res, prob, ys, S, w.seed)
        out["grouping_note"] = GROUPING_NOTE
    print(json.dumps(out), flush=True)
    return 0


GROUPING_NOTE = ("seconds measured for the surrogate grouping (the solved one); for the others "
                 "Sum K_e times the measured seconds per ensemble iteration")


def grouping_costs(res, prob, ys, S: int, seed: int) -> dict:
    """Every sample of a non-adaptive run solved: the cost of other
    groupings of the same samples follows from the recorded counts (a
    member's count does not depend on its companions), eqs. (Rl), (R); their
    time is predicted from the measured time per ensemble iteration."""
    import numpy as np
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import grouping as G
    M = len(ys)
    its_all = res.iters
    per_iter = res.solve_seconds / float(sum(res.ens_iters))
    hind = E.param_indicator_samples(prob, ys)
    orders = {"surrogate": None,
              "random": list(np.random.default_rng(seed).permutation(M)),
              "natural": list(range(M)),
              "param": sorted(range(M), key=lambda i: (hind[i], i)),
              "its": sorted(range(M), key=lambda i: (its_all[i], i))}
    table = {}
    for name, order in orders.items():
        groups = res.groups if name == "surrogate" else G.chunk(order, S)
        tot = G.ensemble_iteration_total(groups, its_all)
        table[name] = {"sum_ensemble_iters": tot, "R": round(G.cost_ratio(groups, its_all, S), 4),
                       "seconds": round(res.solve_seconds, 3) if name == "surrogate"
                       else round(tot * per_iter, 3)}
    return table


def fe3d_mode(args) -> int:
    """The paper's 3-D test problem: 32^3 trilinear cells, d = 4 KL terms,
    rtol 1e-7.  The level-2 sparse grid (41 nodes) is solved to build the
    iteration surrogate, the 512 uniform samples (seed 5) are ordered by it
    into ensembles of S and every ensemble is solved, with Jacobi, with
    degree-4 Jacobi-Chebyshev and with the multigrid V-cycle (--precs picks
    a subset), --streams ensembles at a time (default 2) on separate HIP
    streams; the first ensemble's samples are also solved one at a time
    (S = 1).  --test 2 takes the paper's Test 2 coefficient.  At this size
    an ensemble's matrix (27 x 8 B per member-row, 206 MB at S = 32) fits
    the 256 MB Infinity Cache, so the product kernel's rate is partly a
    cache rate."""
    import numpy as np
    import torch
    import workloads
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq
    torch.cuda.set_device(0)
    w = workloads.FE3D_32_TEST2 if args.test == 2 else workloads.FE3D_32
    prob = E.Problem(w.n, w.d, w.eps_model, dim=3)
    ys = workloads.uniform_samples(w.seed, w.n_samples, w.d)
    S = args.S
    # bytes per member-row: direction kernel (r, diagonal, p_old, x in;
    # p, x out) + product (27 matrix values, p in; q out) = 35 words; the
    # update adds r, q, diagonal in and r out
    # (by default the product reads 14 matrix values per row and takes the
    # other 13 from the neighbours' rows by symmetry: 22 and 26 words)
    step_bytes, iter_bytes = (35 * 8, 39 * 8) if FULL_STENCIL else (22 * 8, 26 * 8)
    K = args.streams or 2
    out = {"mode": "fe3d", "workload": w.name, "grid": f"{w.n + 1}^3 cells", "S": S,
           "samples": w.n_samples, "rtol": w.rtol, "full_stencil": FULL_STENCIL,
           "step_bytes_per_member_row": step_bytes, "streams": K}
    precs = [p for p in args.precs.split(",") if p] if args.precs else ["jacobi", "chebyshev", "multigrid"]
    for pre in precs:
        opts = E.SolverOptions(precond=pre, rtol=w.rtol, max_iter=w.max_iter, time_spmv=True,
                               full_stencil=FULL_STENCIL)
        uq.nonadaptive(prob, S, ys[:S], 1, opts, solve_groups=[0], streams=K)       # warm-up
        res = uq.nonadaptive(prob, S, ys, 2, opts, streams=K)
        its = res.iters
        us = 1e3 * res.spmv_ms / max(1, res.spmv_launches)
        rows = prob.rows * S
        r = {"sample_solves_per_s": round(len(ys) / res.solve_seconds, 2),
             "solve_seconds": round(res.solve_seconds, 3),
             "iters": [int(its.min()), int(its.max())], "sum_ens_iters": int(sum(res.ens_iters)),
             "R": round(S * sum(res.ens_iters) / float(its.sum()), 4),
             "grouping": {k: v["R"] for k, v in grouping_costs(res, prob, ys, S, w.seed).items()}}
        if K == 1:
            # (with concurrent ensembles the timed launches overlap others' work)
            r["step_avg_us"] = round(us, 2)
            r["step_alg_GBs"] = round(rows * step_bytes / (us * 1e-6) / 1e9, 1)
        if pre == "jacobi":
            r["iteration_alg_GBs"] = round(sum(res.ens_iters) * rows * iter_bytes
                                           / res.solve_seconds / 1e9, 1)
            # the first ensemble's samples one at a time
            g0 = [int(i) for i in res.groups[0]]
            ws1 = E.workspace(prob, 1, opts)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for i in g0:
                V, b = E.assemble(prob, torch.tensor(ys[i:i + 1], dtype=torch.float64,
                                                     device="cuda"))
                E.solve(prob, V, b, opts, ws=ws1)
            torch.cuda.synchronize()
            t1 = time.perf_counter() - t
            wsS = E.workspace(prob, S, opts)
            torch.cuda.synchronize()
            t = time.perf_counter()
            V, b = E.assemble(prob, torch.tensor(ys[g0], dtype=torch.float64, device="cuda"))
            E.solve(prob, V, b, opts, ws=wsS)
            torch.cuda.synchronize()
            tS = time.perf_counter() - t
            r["first_ensemble_S1_seconds"] = round(t1, 4)
            r["first_ensemble_S_seconds"] = round(tS, 4)
            r["speedup_vs_S1"] = round(t1 / tS, 2)
        out[pre] = r
        print(json.dumps({pre: r}), flush=True)
    print(json.dumps(out), flush=True)
    return 0


def batch_mode(args) -> int:
    """64 ensembles, widths drawn from {4..64}, grids from {256, 512, 1024}^2,
    d = 8 coefficient model (seed 3), Jacobi-PCG rtol 1e-8, solved together by
    the graph-replayed batched solver, smallest first in waves of the
    autotuner's size (--wave-gb sets it, -1 one batch).  Launch shapes
    (member tile width, tile height) and the wave size come from the
    autotuner (untimed).  Reports total sample-solves/s, p50 / p99 of the
    per-ensemble retirement latency, and the same ensembles solved one after
    another in the same run."""
    import numpy as np
    import torch
    import workloads
    from paper_1705_02003_amd import autotune
    from paper_1705_02003_amd import ensemble as E
    torch.cuda.set_device(0)
    w = workloads.BATCHED
    draw = workloads.batched_draw(w.seed)
    k = args.ensembles or len(draw.widths)
    widths, grids, samples = draw.widths[:k], draw.grids[:k], draw.samples[:k]
    t0 = time.perf_counter()
    shapes = {key: autotune.tune(*key) for key in sorted(set(zip(grids, widths)))}
    # smallest-first waves by default, of the autotuner's size; --wave-gb
    # sets it, --wave-gb -1 solves every ensemble in one batch
    if args.wave_gb > 0:
        wave_bytes, wave_src = args.wave_gb * 1e9, "option"
    elif args.wave_gb < 0:
        wave_bytes, wave_src = None, "one batch"
    else:
        wave_bytes, wave_src = autotune.tune_wave()["wave_bytes"], "autotuned"
    tune_s = time.perf_counter() - t0
    print(f"[bench] autotuned {len(shapes)} (n, S) shapes and the wave size "
          f"({wave_bytes and round(wave_bytes / 1e9, 3)} GB per CG step, {wave_src}) in "
          f"{tune_s:.1f} s", flush=True)
    # device bytes an ensemble keeps resident: matrix (9 slots), b, x and its
    # Jacobi workspace (5 vectors); if the draw does not fit in 80 % of HBM,
    # it is assembled and solved in residency waves, in draw order
    def resident(S, n):
        prob = E.Problem(n, w.d, w.eps_model, w.amp)
        return 8 * (9 + 2) * E.matrix_slot_stride(prob, S) + E.workspace_bytes(prob, S)
    cap = args.resident_gb * 2**30 if args.resident_gb > 0 else \
        0.8 * torch.cuda.get_device_properties(0).total_memory
    need = [resident(S, n) for S, n in zip(widths, grids)]
    residency, cur, tot = [], [], 0
    for i, nb in enumerate(need):
        if cur and tot + nb > cap:
            residency.append(cur)
            cur, tot = [], 0
        cur.append(i)
        tot += nb
    residency.append(cur)
    print(f"[bench] draw needs {sum(need) / 2**30:.1f} GiB resident: "
          f"{len(residency)} residency wave(s)", flush=True)
    opts = E.SolverOptions(rtol=w.rtol, max_iter=w.max_iter, full_stencil=FULL_STENCIL)
    items, res, dt = [None] * k, [None] * k, 0.0
    for wave in residency:
        for i in wave:
            S, n, y = widths[i], grids[i], samples[i]
            prob = E.Problem(n, w.d, w.eps_model, w.amp)
            V, b = E.assemble(prob, torch.tensor(y, dtype=torch.float64, device="cuda"))
            sh = shapes[(n, S)]
            items[i] = {"prob": prob, "V": V, "b": b, "tile_lines": sh["tile_lines"],
                        "member_tile": sh["member_tile"]}
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = E.batch_solve([items[i] for i in wave], opts, max_wave_bytes=wave_bytes)
        torch.cuda.synchronize()
        for i, r in zip(wave, out):
            res[i] = r._replace(seconds=dt + r.seconds)
        dt += time.perf_counter() - t
        print(f"[bench] batch: {len(wave)} ensembles solved, {dt:.2f} s so far", flush=True)
        if len(residency) > 1:
            for i in wave:
                items[i] = {"prob": items[i]["prob"], "b_shape": tuple(items[i]["b"].shape)}
            torch.cuda.empty_cache()
    lat = np.array([r.seconds for r in res])
    n_samples = int(sum(widths))
    rows = sum(r.ens_iters * E.Problem(n, w.d).rows * S for r, S, n in zip(res, widths, grids))
    out = {"mode": "batch", "workload": w.name, "ensembles": k, "samples": n_samples,
           "wave_gb": wave_bytes and round(wave_bytes / 1e9, 4), "wave_size": wave_src,
           "resident_GiB": round(sum(need) / 2**30, 1),
           "residency_waves": len(residency),
           "seconds": round(dt, 3), "sample_solves_per_s": round(n_samples / dt, 3),
           "latency_p50_s": round(float(np.percentile(lat, 50)), 4),
           "latency_p99_s": round(float(np.percentile(lat, 99)), 4),
           "latency_max_s": round(float(lat.max()), 4),
           "ensemble_iters": [int(r.ens_iters) for r in res],
           "iteration_alg_GBs": round(rows * ITER_BYTES / dt / 1e9, 1),
           "all_converged": bool(all(np.all(r.status == 0) for r in res)),
           "shapes": {f"{n}x{S}": [v["member_tile"], v["tile_lines"]] for (n, S), v in shapes.items()}}
    if not args.no_sequential and len(residency) == 1:
        torch.cuda.synchronize()
        t = time.perf_counter()
        for j, it in enumerate(items):
            E.solve(it["prob"], it["V"], it["b"],
                    E.SolverOptions(rtol=w.rtol, max_iter=w.max_iter, full_stencil=FULL_STENCIL,
                                    tile_lines=it["tile_lines"],
                                    member_tile=it["member_tile"]))
            if j % 16 == 15:
                print(f"[bench] sequential: {j + 1} ensembles, {time.perf_counter() - t:.2f} s",
                      flush=True)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t
        out["sequential_seconds"] = round(ts, 3)
        out["batch_speedup_vs_sequential"] = round(ts / dt, 3)
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--S", type=int, default=32)
    ap.add_argument("--budget", type=int, default=1024)
    ap.add_argument("--cpu-procs", type=int, default=0, help="0: min(16, cpu count)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=32,
                    help="samples the oracle solves for the CPU baseline (the run's first ones; "
                         "about 30 s on 16 cores at 32)")
    ap.add_argument("--no-s1", action="store_true")
    ap.add_argument("--mode", choices=["full", "kernel", "adjoint", "cheb", "batch", "su", "grouping",
                                       "table", "fe3d"],
                    default="full",
                    help="kernel: a fixed-iteration solve of one ensemble plus a 1 GiB "
                         "copy, for hardware-counter runs")
    ap.add_argument("--iters", type=int, default=100, help="iterations in --mode kernel")
    ap.add_argument("--grid", type=int, default=N_GRID, help="grid size n in --mode kernel")
    ap.add_argument("--precond", choices=["jacobi", "chebyshev", "multigrid"], default="jacobi",
                    help="preconditioner in --mode kernel (jacobi, chebyshev) and --mode table --dim 3")
    ap.add_argument("--S-list", default="4,8,16,32,64", help="ensemble widths in --mode table")
    ap.add_argument("--resident-gb", type=float, default=0.0,
                    help="--mode batch: device memory the draw may keep resident (0: 80 %% of HBM)")
    ap.add_argument("--wave-gb", type=float, default=0.0,
                    help="--mode batch: smallest-first waves of at most this many GB per CG "
                         "iteration (0: the autotuner's size; -1: all ensembles in one batch)")
    ap.add_argument("--streams", type=int, default=0,
                    help="ensembles solved at a time on separate HIP streams (0: 2 in --mode fe3d, "
                         "else 1)")
    ap.add_argument("--dim", type=int, default=2, choices=(2, 3),
                    help="--mode table: the 2-D benchmark problem or the 3-D test problem")
    ap.add_argument("--precs", default="",
                    help="comma-separated preconditioners of --mode fe3d (default jacobi,chebyshev,multigrid)")
    ap.add_argument("--test", type=int, default=1, choices=(1, 2),
                    help="--mode table --dim 3 and --mode fe3d: the paper's Test 1 (a_hat = 1) "
                         "or Test 2 (a_hat banded by |y|)")
    ap.add_argument("--full-stencil", action="store_true",
                    help="read all nine matrix values per row (no symmetric reuse)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="--mode batch: skip solving the ensembles one after another")
    ap.add_argument("--ensembles", type=int, default=0,
                    help="ensembles to solve in --mode adjoint / cheb (0: the mode's default)")
    ap.add_argument("--all-ensembles", action="store_true",
                    help="--mode cheb: solve every ensemble (all 4096 samples) and compare groupings")
    args = ap.parse_args()
    set_byte_model(args.full_stencil)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the ensemble solver runs on a single "
              "MI355X (ensembles are independent; see the design notes for how the "
              "path would shard). Run with --gpus 1.", file=sys.stderr)
        return 2

    if args.mode == "kernel":
        return kernel_mode(args)
    if args.mode == "adjoint":
        return adjoint_mode(args)
    if args.mode == "cheb":
        return cheb_mode(args)
    if args.mode == "batch":
        return batch_mode(args)
    if args.mode == "su":
        return su_mode(args)
    if args.mode == "grouping":
        return grouping_mode(args)
    if args.mode == "table":
        return table_mode(args)
    if args.mode == "fe3d":
        return fe3d_mode(args)

    cpu, cpu_ys = None, None
    if not args.no_cpu_baseline:
        procs = args.cpu_procs or min(16, os.cpu_count() or 1)
        cpu, cpu_ys = cpu_baseline(procs, args.cpu_samples, args.S)
        print(f"[bench] cpu baseline: {cpu['value']} sample-solves/s on {procs} cores", flush=True)

    import numpy as np
    import torch
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    prob = E.Problem(N_GRID, D, 0, AMP)
    opts = E.SolverOptions(rtol=RTOL, max_iter=20000, time_spmv=True, full_stencil=FULL_STENCIL)

    def step():
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = uq.adaptive(prob, args.S, budget=args.budget, max_level=5, tau_rel=1e-3,
                        strategy="surrogate", opts=opts, perm_seed=1)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    for w in range(args.warmup):
        r, dt = step()
        print(f"[bench] warmup {w}: {len(r.y)} samples in {dt:.2f} s", flush=True)
    times, spmv_ms, spmv_rows, launches, res = [], 0.0, 0.0, 0, None
    for k in range(args.steps):
        res, dt = step()
        times.append(dt)
        spmv_ms += res.spmv_ms
        spmv_rows += res.spmv_member_rows
        launches += res.spmv_launches
        print(f"[bench] step {k}: {len(res.y)} samples, {res.total_ensemble_iters} ensemble "
              f"iterations in {dt:.2f} s", flush=True)
    total = sum(times)
    n_samples = len(res.y)
    value = n_samples * args.steps / total

    achieved = (spmv_rows * FUSED_BYTES / 1e9) / (spmv_ms / 1e3) if spmv_ms > 0 else None
    solve_s = sum(l.solve_seconds for l in res.levels)
    member_iter_rows = res.total_ensemble_iters * args.S * prob.rows
    useful_rows = int(res.iters.sum()) * prob.rows
    costs = uq.grouping_costs(res, args.S)
    costs16 = uq.grouping_costs(res, 16) if args.S != 16 else None
    asm_s = res.assemble_ms / 1e3

    # the GPU on the ensembles holding the oracle's samples
    if cpu is not None:
        pos = {tuple(y): k for k, y in enumerate(res.y)}
        ids = [pos[tuple(y)] for y in cpu_ys if tuple(y) in pos]
        cpu["same_samples_as_gpu_run_start"] = sorted(ids) == sorted(run_order(res)[:len(cpu_ys)])
        cpu["gpu_same_samples"] = gpu_same_samples(res, ids, args.S, opts)
        print(f"[bench] GPU on the oracle's samples: {cpu['gpu_same_samples']['value']} "
              f"sample-solves/s", flush=True)

    out = {
        "metric": "sample-solves/s + HBM GB/s, ensemble PCG S=32 vs S=1, 512² grid, rtol 1e-8",
        "value": round(value, 3),
        "unit": "sample-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "adaptive-sg-512x512-d4", "grid": f"{N_GRID}x{N_GRID}",
                   "samples": n_samples, "S": args.S, "precond": "jacobi", "rtol": RTOL,
                   "grouping": "surrogate", "levels": [l.n_samples for l in res.levels]},
        "roofline": {"bound": "hbm",
                     "achieved": round(achieved, 1) if achieved else None,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                     "traffic": measured_traffic(args.S),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "stencil_kernel<2, M_PCG_J> (fused direction update + SpMV)",
                     "bytes_per_member_row": FUSED_BYTES,
                     "bytes_note": ("the method's own reads: five stored matrix values per row "
                                    "(the other four are the neighbours' by symmetry), r, p_old, "
                                    "x; writes p, q, x"),
                     "timed_launches": launches,
                     "avg_launch_us": round(1e3 * spmv_ms / max(1, launches), 2)},
        "gbps_iteration_alg": round(member_iter_rows * ITER_BYTES / solve_s / 1e9, 1),
        "gbps_iteration_useful": round(useful_rows * ITER_BYTES / solve_s / 1e9, 1),
        "ensemble_iterations": res.total_ensemble_iters,
        "sample_solves_per_s_without_assembly": round(n_samples / (times[-1] - asm_s), 3),
        "assembly_seconds": round(asm_s, 3),
        "qoi_mean_levels": [l.qoi_mean for l in res.levels],
        "grouping": costs,
        "grouping_S16": costs16,
        "cpu_baseline": cpu,
    }
    if not args.no_s1:
        out["s1_comparison"] = s1_comparison(res, args.S, E.SolverOptions(rtol=RTOL))
    traffic = out["roofline"]["traffic"]
    if traffic and spmv_ms > 0:
        # measured HBM bytes per launch over the same launches' average time
        out["roofline"]["measured_GBs"] = round(traffic / 1e9 / (spmv_ms / launches / 1e3), 1)
    if achieved and not FULL_STENCIL:
        # the nine-stored-values byte count of a plain (non-symmetric) read:
        # 15 words; it exceeds 8 TB/s at this kernel's time, which shows the
        # kernel does not move those bytes
        a9 = achieved * 15 / 11
        out["roofline"]["nine_value_model"] = {
            "bytes_per_member_row": 120, "achieved": round(a9, 1),
            "frac": round(a9 / HBM_PEAK_GBS, 4)}
    streams = measure_streams()
    out["roofline"]["stream_triad_GBs"] = streams["triad_GBs"]
    out["roofline"]["stream_mix_8r3w_GBs"] = streams["mix_8r3w_GBs"]
    if achieved:
        out["roofline"]["frac_of_stream_triad"] = round(achieved / streams["triad_GBs"], 4)
        out["roofline"]["frac_of_stream_mix"] = round(achieved / streams["mix_8r3w_GBs"], 4)
    # At 512^2 the benchmark's vectors (67 MB each) partly stay in the 256 MB
    # Infinity Cache between kernels, so the figure above is L2-miss
    # bandwidth (HBM plus Infinity Cache); the same kernel at 1024^2 has a
    # working set far beyond that cache: an HBM-only rate.
    out["roofline"]["memory"] = "L2 misses: HBM + Infinity Cache"
    out["roofline"]["hbm_only_1024"] = fused_kernel_rate(1024, args.S)
    out["device"] = device_info()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
