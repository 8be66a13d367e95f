"""Autotuner for the launch shapes of the solver.

Stencil shape: for a grid size n and ensemble width S it times
fixed-iteration solves (rtol 0) of a synthetic ensemble for each candidate
(member tile width, tile height) and keeps the fastest per iteration.  The
member tile is the "ensemble width" the kernel sweeps at once: a 64-member
ensemble can be swept as two 32-member halves, which halves the one-point
halo each tile reads.

Batch wave size: the batched solver advances every live ensemble in each
step, so a small ensemble batched with large ones waits for their steps.
Solving smallest first in waves lets the small ones retire early; a wave
must still hold enough work per step to keep the GPU busy.  ``tune_wave``
times fixed-iteration batched solves of stacks of identical small ensembles
of growing total size and returns the smallest bytes per CG step whose
throughput reaches a set share of the largest measured.

Results are cached in a JSON file keyed by device name, the kernel source
(a hash of the library file) and the shape.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import _lib as L
from . import ensemble as E

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "_build", "autotune.json")


def _library_hash() -> str:
    h = hashlib.sha256()
    with open(L.LIB_PATH, "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:12]


def _key(*parts) -> str:
    name = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    return "|".join([name, _library_hash()] + [str(p) for p in parts])


def _load(cache: Optional[str]) -> dict:
    if cache and os.path.exists(cache):
        try:
            with open(cache) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            return {}
    return {}


def _store(cache: Optional[str], table: dict) -> None:
    if not cache:
        return
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    tmp = cache + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, cache)


def candidates(n: int, S: int) -> Iterable[Tuple[int, int]]:
    """(member_tile, tile_lines) pairs worth timing."""
    widths = sorted({w for w in (S, S // 2, S // 4) if w >= 2 and 512 // w <= n} or {S})
    for sw in widths:
        for ty in (8, 16, 32):
            if ty <= n:
                yield sw, ty


def _ensemble(n: int, S: int):
    prob = E.Problem(n, 4, 0, 0.4)
    g = torch.Generator(device="cpu").manual_seed(n * 131 + S)
    y = torch.rand((S, 4), generator=g, dtype=torch.float64) * 2 - 1
    V, b = E.assemble(prob, y)
    return prob, V, b


def measure(n: int, S: int, sw: int, ty: int, iters: int = 20, groups: int = 0) -> float:
    """Seconds per Jacobi-PCG iteration for one launch shape."""
    prob, V, b = _ensemble(n, S)
    opts = E.SolverOptions(rtol=0.0, max_iter=iters, tile_lines=ty, member_tile=sw,
                           max_groups=groups, poll_every=iters)
    ws = E.workspace(prob, S, opts)
    E.solve(prob, V, b, opts, ws=ws)
    torch.cuda.synchronize()
    t = time.perf_counter()
    E.solve(prob, V, b, opts, ws=ws)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / iters


def tune(n: int, S: int, cache: Optional[str] = DEFAULT_CACHE, iters: int = 20,
         refresh: bool = False) -> Dict[str, int]:
    """Best {"member_tile", "tile_lines"} for (n, S), from the cache if present."""
    table = _load(cache)
    key = _key(f"n={n}", f"S={S}")
    if key in table and not refresh:
        return table[key]
    best = None
    trials = {}
    for sw, ty in candidates(n, S):
        dt = measure(n, S, sw, ty, iters)
        trials[f"{sw}x{ty}"] = round(dt * 1e6, 2)
        if best is None or dt < best[0]:
            best = (dt, sw, ty)
    choice = {"member_tile": best[1], "tile_lines": best[2],
              "us_per_iteration": round(best[0] * 1e6, 2), "trials_us": trials}
    table[key] = choice
    _store(cache, table)
    return choice


def tune_wave(cache: Optional[str] = DEFAULT_CACHE, share: float = 0.9, iters: int = 64,
              n: int = 256, S: int = 8, counts=(1, 2, 4, 8, 16, 32, 64),
              refresh: bool = False) -> Dict[str, float]:
    """Bytes per CG step a wave of the batched solver should hold: stacks of
    `count` identical (n, S) Jacobi ensembles are solved together for a fixed
    number of steps; the wave size is the smallest stack whose rate (bytes of
    a CG step, 120 per member-row, per second) reaches `share` of the best."""
    table = _load(cache)
    key = _key("wave", f"n={n}", f"S={S}", f"share={share}")
    if key in table and not refresh:
        return table[key]
    prob, V, b = _ensemble(n, S)
    opts = E.SolverOptions(rtol=0.0, max_iter=iters, poll_every=iters)
    per = 120 * prob.rows * S
    rates = {}
    for c in counts:
        items = [{"prob": prob, "V": V, "b": b} for _ in range(c)]
        E.batch_solve(items, opts, max_wave_bytes=None)
        torch.cuda.synchronize()
        t = time.perf_counter()
        E.batch_solve(items, opts, max_wave_bytes=None)
        torch.cuda.synchronize()
        rates[c] = per * c * iters / (time.perf_counter() - t)
    top = max(rates.values())
    c = min(k for k, r in rates.items() if r >= share * top)
    choice = {"wave_bytes": float(per * c), "ensembles": c, "share": share,
              "GBs": {str(k): round(r / 1e9, 1) for k, r in rates.items()}}
    table[key] = choice
    _store(cache, table)
    return choice
