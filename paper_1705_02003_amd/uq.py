"""Adaptive sparse-grid sampling with surrogate-grouped ensemble solves.

Paper, Section 3.1 ("The algorithm", flow chart of Fig. 2): starting from an
initial sparse grid grouped in generation order, repeat
  1. solve the level's samples in ensembles, record G(y) and I(y);
  2. build the surrogates G^ and I^ from every sample so far;
  3. use G^ to select the next level's samples (classic refinement);
  4. use I^ to group them into ensembles of S,
until no sample is selected, the level cap is reached, or the budget is
spent.  The output of interest is G(y) = ||u(y)||_2^2 (Section 4); after each
level the quantity of interest E[G] is the mean of the interpolant G^
(Section 2.1).

Grouping strategies: "surrogate" (the paper's), "natural" (generation
order), "random" (one seeded permutation per level).  The ideal grouping by
true iteration counts ("its") is computed after the fact from the recorded
counts; each member's count does not depend on its ensemble companions
(per-member arithmetic, deterministic reductions), so the cost of any other
grouping of the same samples follows exactly from the recorded counts.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import ensemble as E
from . import grouping as G


@dataclass
class LevelRecord:
    level: int
    n_samples: int
    groups: np.ndarray          # (K_l, S) indices into this level's samples (a list of
                                # id arrays of varying width with strategy "variable")
    ens_iters: List[int]        # K_e per ensemble
    iters: np.ndarray           # per real sample
    qoi: np.ndarray             # G(y) per real sample
    pred: np.ndarray            # I^(y) used for grouping (0 on the first level)
    solve_seconds: float
    qoi_mean: float = 0.0       # E[G^] over every sample up to this level


@dataclass
class UQResult:
    level: np.ndarray = None    # (M, d) node levels, generation order
    index: np.ndarray = None
    y: np.ndarray = None        # (M, d)
    iters: np.ndarray = None    # (M,)
    qoi: np.ndarray = None      # (M,)
    levels: List[LevelRecord] = field(default_factory=list)
    spmv_ms: float = 0.0
    spmv_launches: int = 0
    spmv_member_rows: float = 0.0   # sum over timed launches of N_r * S
    assemble_ms: float = 0.0        # device time of the ensemble assemblies
    hind: np.ndarray = None         # parameter-based indicator H(y) per sample (Section 3.2)

    @property
    def qoi_mean(self) -> float:
        """The quantity of interest E[G(y)], y uniform on [-1, 1]^d, from the
        sparse-grid interpolant of every computed G (Section 2.1)."""
        return self.levels[-1].qoi_mean if self.levels else 0.0

    @property
    def total_ensemble_iters(self) -> int:
        return int(sum(sum(r.ens_iters) for r in self.levels))


class _Workspaces:
    """Solver workspaces by ensemble width (and by worker, for concurrent
    solves), allocated on first use; one HIP stream per extra worker."""

    def __init__(self, prob, opts, device):
        self.prob, self.opts, self.device, self.by_width, self.streams = prob, opts, device, {}, {}

    def __call__(self, S: int, worker: int = 0):
        if (S, worker) not in self.by_width:
            self.by_width[(S, worker)] = E.workspace(self.prob, S, self.opts, self.device)
        return self.by_width[(S, worker)]

    def stream(self, worker: int):
        if worker not in self.streams:
            self.streams[worker] = torch.cuda.Stream(device=self.device)
        return self.streams[worker]


def _solve_groups(prob, y_level, groups, opts, wss, device, spmv_acc, streams: int = 1,
                  progress=None):
    """Solve each group (an id array; its length is the ensemble width) and
    record per-sample counts and G(y) = ||u||^2.  With streams = K > 1, K
    host threads solve the groups round-robin, each on its own HIP stream
    with its own workspace: small ensembles leave most of the GPU idle
    between kernels, and concurrent ensembles fill it (each ensemble's
    arithmetic is unchanged).  ens_iters stays in group order."""
    K = min(max(1, streams), len(groups))
    if K > 1:
        torch.cuda.synchronize(device)
        accs = [[0.0, 0, 0.0, 0.0] for _ in range(K)]

        def work(k):
            with torch.cuda.stream(wss.stream(k)):
                out = _solve_serial(prob, y_level, groups[k::K], opts,
                                    lambda S: wss(S, k), device, accs[k])
            wss.stream(k).synchronize()
            return out

        with ThreadPoolExecutor(K) as ex:
            parts = list(ex.map(work, range(K)))
        iters = np.full(len(y_level), -1, np.int64)
        qoi = np.zeros(len(y_level))
        ens_iters = [0] * len(groups)
        for k, (it, q, ei) in enumerate(parts):
            done = it >= 0
            iters[done], qoi[done] = it[done], q[done]
            ens_iters[k::K] = ei
        for acc in accs:
            for i in range(4):
                spmv_acc[i] += acc[i]
        return iters, qoi, ens_iters
    return _solve_serial(prob, y_level, groups, opts, wss, device, spmv_acc, progress)


def _solve_serial(prob, y_level, groups, opts, wss, device, spmv_acc, progress=None):
    iters = np.full(len(y_level), -1, np.int64)
    qoi = np.zeros(len(y_level))
    ens_iters = []
    for g in groups:
        g = np.asarray(g)
        S = len(g)
        ws = wss(S)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        V, b = E.assemble(prob, y_level[g], device=device)
        e1.record()
        res = E.solve(prob, V, b, opts, ws=ws)     # blocks: both events have completed
        spmv_acc[3] += e0.elapsed_time(e1)
        if np.any(res.status != 0):
            raise RuntimeError(f"ensemble did not converge: status {res.status.tolist()}")
        gval = E.member_dot(res.x, res.x, ws=ws)
        ens_iters.append(res.ens_iters)
        for s, idx in enumerate(g):
            if iters[idx] < 0:
                iters[idx] = int(res.iters[s])
                qoi[idx] = gval[s]
        st = res.stats
        spmv_acc[0] += st["spmv_ms"]
        spmv_acc[1] += st["spmv_timed"]
        spmv_acc[2] += st["spmv_timed"] * prob.rows * S
        if progress is not None:
            progress(len(ens_iters), len(groups))
    return iters, qoi, ens_iters


def adaptive(prob: E.Problem, S: int, budget: int = 1024, max_level: int = 5,
             tau_rel: float = 1e-3, strategy: str = "surrogate",
             opts: Optional[E.SolverOptions] = None, perm_seed: int = 1,
             device="cuda", widths=None, iter_seconds=None, streams: int = 1) -> UQResult:
    """Run the adaptive loop; every sample is solved on the GPU in ensembles
    of S, or, with strategy "variable", in ensembles of the given ``widths``
    chosen by least predicted time (``iter_seconds`` per ensemble iteration
    at each width; the surrogate predicts the counts, all counts are taken
    equal on the first level).  ``streams`` > 1 solves that many ensembles
    at a time on separate HIP streams."""
    opts = opts or E.SolverOptions()
    rng = np.random.default_rng(perm_seed)
    wss = _Workspaces(prob, opts, device)
    lv, ix = G.initial_grid(prob.d)
    out = UQResult(level=np.zeros((0, prob.d), np.int32), index=np.zeros((0, prob.d), np.int32),
                   y=np.zeros((0, prob.d)), iters=np.zeros(0, np.int64), qoi=np.zeros(0),
                   hind=np.zeros(0))
    spmv_acc = [0.0, 0, 0.0, 0.0]
    level = 1
    while True:
        y_level = G.coords(lv, ix)
        hind = E.param_indicator_samples(prob, y_level, device)
        if strategy == "param":
            # Section 3.2: ascending H, ties in generation order, on every level
            groups = G.chunk(sorted(range(len(y_level)), key=lambda i: (hind[i], i)), S)
            pred = np.zeros(len(y_level))
        elif strategy != "variable" and (level == 1 or strategy == "natural"):
            groups = G.chunk(list(range(len(y_level))), S)
            pred = np.zeros(len(y_level))
        elif strategy == "surrogate":
            groups, pred = G.group_samples(out.level, out.index, out.iters, y_level, S)
        elif strategy == "random":
            groups = G.chunk(list(rng.permutation(len(y_level))), S)
            pred = np.zeros(len(y_level))
        elif strategy == "variable":
            if level == 1:
                pred = np.ones(len(y_level))
            else:
                _, pred = G.group_samples(out.level, out.index, out.iters, y_level, 1)
            groups, _ = G.group_variable(pred, widths, iter_seconds)
        else:
            raise ValueError(strategy)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, qoi, ens_iters = _solve_groups(prob, y_level, groups, opts, wss, device, spmv_acc,
                                              streams)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.level = np.vstack([out.level, lv])
        out.index = np.vstack([out.index, ix])
        out.y = np.vstack([out.y, y_level])
        out.iters = np.concatenate([out.iters, iters])
        out.qoi = np.concatenate([out.qoi, qoi])
        out.hind = np.concatenate([out.hind, hind])
        mean = G.expectation(out.level, out.index, out.qoi)
        out.levels.append(LevelRecord(level, len(y_level), groups, ens_iters, iters, qoi, pred, dt,
                                      mean))
        if level >= max_level or len(out.y) >= budget:
            break
        lv, ix = G.refine(out.level, out.index, out.qoi, level, tau_rel, budget)
        if len(lv) == 0:
            break
        level += 1
    out.spmv_ms, out.spmv_launches, out.spmv_member_rows = spmv_acc[0], int(spmv_acc[1]), spmv_acc[2]
    out.assemble_ms = spmv_acc[3]
    return out


def strategy_groups(res: UQResult, S: int, perm_seed: int = 1) -> dict:
    """Per-level ensembles of S for each grouping strategy applied to the
    samples of an adaptive run (S may differ from the run's width: the
    surrogate grouping is then recomputed from the same data).  Strategies:
    "surrogate" (Section 3.1), "natural" (generation order), "random" (one
    seeded permutation per level), "param" (Section 3.2: ascending
    H(y) = max_x lambda_max / lambda_min of the diffusion tensor, from the
    library, ties in generation order; for the 2-D model H = 1 / eps(y_1))
    and "its" (ascending true counts, the ideal).  On the first level
    "surrogate" and "random" use generation order: there is nothing to go on
    yet."""
    rng = np.random.default_rng(perm_seed)
    per = {"surrogate": [], "natural": [], "random": [], "param": [], "its": []}
    start = 0
    for r in res.levels:
        its = r.iters
        m = len(its)
        y = res.y[start:start + m]
        nat = G.chunk(list(range(m)), S)
        per["natural"].append(nat)
        per["random"].append(G.chunk(list(rng.permutation(m)), S) if r.level > 1 else nat)
        hv = res.hind[start:start + m]
        per["param"].append(G.chunk(sorted(range(m), key=lambda i: (hv[i], i)), S))
        per["its"].append(G.chunk(sorted(range(m), key=lambda i: (its[i], i)), S))
        if r.level == 1:
            sur = nat
        elif isinstance(r.groups, np.ndarray) and r.groups.shape[1] == S:
            sur = r.groups
        else:
            sur, _ = G.group_samples(res.level[:start], res.index[:start], res.iters[:start], y, S)
        per["surrogate"].append(sur)
        start += m
    return per


def variable_groups(res: UQResult, widths, iter_seconds) -> list:
    """Per-level ensembles of varying width for the samples of an adaptive
    run (Section 5): least predicted time with the surrogate of the earlier
    levels' counts (equal counts assumed on the first level)."""
    per, start = [], 0
    for r in res.levels:
        m = r.n_samples
        if r.level == 1:
            pred = np.ones(m)
        else:
            _, pred = G.group_samples(res.level[:start], res.index[:start], res.iters[:start],
                                      res.y[start:start + m], 1)
        groups, _ = G.group_variable(pred, widths, iter_seconds)
        per.append(groups)
        start += m
    return per


def variable_costs(res: UQResult, per: list) -> dict:
    """R (widths weighted) of per-level ensembles of varying width, and the
    widths used."""
    lst = list(zip(per, (r.iters for r in res.levels)))
    num = sum(sum(len(g) * int(it[np.asarray(g)].max()) for g in gs) for gs, it in lst)
    den = sum(int(it.sum()) for _, it in lst)
    widths = sorted({len(g) for gs in per for g in gs})
    return {"R": num / den, "R_levels": [round(G.cost_ratio_variable(gs, it), 4) for gs, it in lst],
            "widths": {int(w): sum(1 for gs in per for g in gs if len(g) == w) for w in widths}}


def grouping_costs(res: UQResult, S: int, perm_seed: int = 1) -> dict:
    """Total ensemble iterations and R (eqs. (Rl), (R)) of each grouping
    strategy on the same samples.  Each member's count does not depend on
    its companions, so these follow exactly from the recorded counts."""
    out = {}
    for k, groups in strategy_groups(res, S, perm_seed).items():
        lst = list(zip(groups, (r.iters for r in res.levels)))
        num = sum(G.ensemble_iteration_total(g, it) for g, it in lst)
        den = sum(int(it.sum()) for _, it in lst)
        out[k] = {"sum_ensemble_iters": int(num), "R": S * num / den,
                  "R_levels": [round(G.cost_ratio(g, it, S), 4) for g, it in lst]}
    return out


def time_groupings(prob: E.Problem, res: UQResult, S: int, opts: Optional[E.SolverOptions] = None,
                   strategies=("natural", "random", "param", "its", "surrogate"),
                   perm_seed: int = 1, device="cuda", extra: Optional[dict] = None,
                   streams: int = 1) -> dict:
    """Wall seconds to solve every sample of an adaptive run grouped by each
    strategy, assembly included ("seconds") and without the assemblies'
    device time ("solve_seconds"), and the ensemble iterations it took.
    ``extra`` adds strategies given as per-level group lists."""
    opts = opts or E.SolverOptions()
    wss = _Workspaces(prob, opts, device)
    per = strategy_groups(res, S, perm_seed)
    if extra:
        per.update(extra)
    out = {}
    for k in strategies:
        acc = [0.0, 0, 0.0, 0.0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        total, start = 0, 0
        for r, groups in zip(res.levels, per[k]):
            y = res.y[start:start + r.n_samples]
            _, _, ens_iters = _solve_groups(prob, y, groups, opts, wss, device, acc, streams)
            total += sum(ens_iters)
            start += r.n_samples
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[k] = {"seconds": round(dt, 3), "solve_seconds": round(dt - acc[3] * 1e-3, 3),
                  "sum_ensemble_iters": int(total)}
    return out


@dataclass
class NonAdaptiveResult:
    train_iters: np.ndarray       # iteration counts at the training grid nodes
    groups: np.ndarray            # (K, S) indices into the samples
    pred: np.ndarray              # surrogate prediction per sample
    iters: np.ndarray             # per sample (solved ensembles only; -1 otherwise)
    ens_iters: List[int]
    solve_seconds: float
    train_seconds: float
    spmv_ms: float = 0.0
    spmv_launches: int = 0
    spmv_member_rows: float = 0.0


def nonadaptive(prob: E.Problem, S: int, y: np.ndarray, train_level: int,
                opts: Optional[E.SolverOptions] = None, solve_groups: Optional[List[int]] = None,
                device="cuda", streams: int = 1, progress=None) -> NonAdaptiveResult:
    """Surrogate grouping without adaptivity (paper, Section 5: pre-select
    samples, evaluate them, build the iteration surrogate, group the rest).

    The training set is the full sparse grid of total level ``train_level``,
    solved in generation order; its iteration counts define I^, which orders
    the samples ``y`` into ensembles of S.  ``solve_groups`` selects which of
    the resulting ensembles are solved (all by default).  ``progress(done,
    total)`` is called after each solved ensemble (serial solves only)."""
    opts = opts or E.SolverOptions()
    wss = _Workspaces(prob, opts, device)
    lv, ix = G.full_grid(prob.d, train_level)
    yt = G.coords(lv, ix)
    acc = [0.0, 0, 0.0, 0.0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it_train, _, _ = _solve_groups(prob, yt, G.chunk(list(range(len(yt))), S), opts, wss,
                                   device, [0.0, 0, 0.0, 0.0], streams)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    groups, pred = G.group_samples(lv, ix, it_train, y, S)
    sel = range(len(groups)) if solve_groups is None else solve_groups
    chosen = np.asarray([groups[k] for k in sel])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters, _, ens_iters = _solve_groups(prob, y, chosen, opts, wss, device, acc, streams,
                                        progress)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return NonAdaptiveResult(it_train, groups, pred, iters, ens_iters, dt, t_train,
                             acc[0], int(acc[1]), acc[2])
