"""Oracle solves in worker processes for the GPU parity tests.

The oracle's per-sample PCG is plain numpy/scipy and single-threaded; the
parity tests at 256^2 and 512^2 need dozens of such solves, so they run in a
pool of spawned CPU processes (the workers import only ``oracle`` and never
touch the GPU).
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from oracle import pcg as opcg
from oracle import problem as oprob


def solve_pair(job):
    """Oracle PCG to rtol (count and status), then the oracle run for exactly
    ``iters`` iterations (the iterate at the GPU's count).  job = (y, n,
    eps_model, amp, precond, rtol, max_iter, iters)."""
    y, n, eps_model, amp, precond, rtol, max_iter, iters = job
    A, b, diag = oprob.assemble(np.asarray(y), n, eps_model, amp)
    _, I, st, _ = opcg.pcg(A, b, diag, rtol, max_iter, precond)
    xe, _, _, _ = opcg.pcg(A, b, diag, 0.0, int(iters), precond)
    return int(I), int(st), xe


def workers() -> int:
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 2
    return max(1, min(12, avail - 1))


def run(jobs):
    """Results of solve_pair for every job, in job order (a progress line per
    finished job)."""
    out = []
    if len(jobs) == 1:
        out.append(solve_pair(jobs[0]))
        print(f"oracle solve 1/1 done", flush=True)
        return out
    # one BLAS thread per worker: the workers inherit this environment
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})
    try:
        ctx = mp.get_context("spawn")
        with ProcessPoolExecutor(max_workers=min(workers(), len(jobs)), mp_context=ctx) as ex:
            for k, r in enumerate(ex.map(solve_pair, jobs)):
                out.append(r)
                print(f"oracle solve {k + 1}/{len(jobs)} done", flush=True)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return out
