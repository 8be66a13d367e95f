"""Autotuner for the stencil kernel's launch shape.

For a grid size n and ensemble width S it times fixed-iteration solves
(rtol 0) of a synthetic ensemble for each candidate (member tile width,
tile height) and keeps the fastest per iteration.  The member tile is the
"ensemble width" the kernel sweeps at once: a 64-member ensemble can be
swept as two 32-member halves, which halves the one-point halo each tile
reads.  Results are cached in a JSON file keyed by device name, n and S.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import ensemble as E

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "_build", "autotune.json")


def _key(n: int, S: int) -> str:
    name = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    return f"{name}|n={n}|S={S}"


def candidates(n: int, S: int) -> Iterable[Tuple[int, int]]:
    """(member_tile, tile_lines) pairs worth timing."""
    widths = sorted({w for w in (S, S // 2, S // 4) if w >= 2 and 512 // w <= n} or {S})
    for sw in widths:
        for ty in (8, 16, 32):
            if ty <= n:
                yield sw, ty


def measure(n: int, S: int, sw: int, ty: int, iters: int = 20, groups: int = 0) -> float:
    """Seconds per Jacobi-PCG iteration for one launch shape."""
    prob = E.Problem(n, 4, 0, 0.4)
    g = torch.Generator(device="cpu").manual_seed(n * 131 + S)
    y = (torch.rand((S, 4), generator=g, dtype=torch.float64) * 2 - 1).cuda()
    V, b = E.assemble(prob, y)
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
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as fh:
                table = json.load(fh)
        except (OSError, ValueError):
            table = {}
    key = _key(n, S)
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
    if cache:
        os.makedirs(os.path.dirname(cache), exist_ok=True)
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return choice
