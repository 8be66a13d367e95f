"""Python front end of libens: torch tensors in, torch tensors out.

Every operation is a call into the HIP library (include/ens.h); this module
only checks shapes and dtypes, allocates outputs and workspaces with torch,
and passes pointers and the current HIP stream.  There is no fallback: if the
library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass
from typing import NamedTuple, Optional

import numpy as np
import torch

from . import _lib as L


@dataclass(frozen=True)
class Problem:
    """dim 2: -div(a(x) K(y) grad u) = 1 on an n x n interior grid (nine-point
    scheme); dim 3: the paper's 3-D test problem on an n x n x n interior grid
    (trilinear finite elements, 27 matrix slots).  See ens_problem."""

    n: int
    d: int
    eps_model: int = 0
    amp: float = 0.0
    dim: int = 2

    @property
    def rows(self) -> int:
        return self.n ** self.dim

    @property
    def slots(self) -> int:
        return 27 if self.dim == 3 else 9

    def c(self) -> L.ens_problem:
        return L.ens_problem(self.n, self.d, self.eps_model, self.dim, float(self.amp))


@dataclass
class SolverOptions:
    precond: str = "jacobi"       # "jacobi", "chebyshev" or "multigrid" (3-D, n + 1 = 2^k)
    cheb_degree: int = 4
    cheb_ratio: float = 30.0
    rtol: float = 1e-8
    max_iter: int = 20000
    poll_every: int = 0           # 0: adaptive (see ens_opts.poll_every)
    tile_lines: int = 0           # 0: heuristic
    max_groups: int = 0           # 0: heuristic
    time_spmv: bool = False
    member_tile: int = 0          # members per stencil tile, 0: the whole ensemble
    full_stencil: bool = False    # read all nine matrix values (no symmetric reuse)
    mg_levelwise: bool = False    # multigrid: one launch per level operation (no fused coarse tail)

    def c(self) -> L.ens_opts:
        pre = {"jacobi": L.PRECOND_JACOBI, "chebyshev": L.PRECOND_CHEBYSHEV,
               "multigrid": L.PRECOND_MULTIGRID}[self.precond]
        return L.ens_opts(pre, self.cheb_degree, float(self.cheb_ratio), float(self.rtol),
                          self.max_iter, self.poll_every, self.tile_lines, self.max_groups,
                          (L.FLAG_TIME_SPMV if self.time_spmv else 0)
                          | (L.FLAG_FULL_STENCIL if self.full_stencil else 0)
                          | (L.FLAG_MG_LEVELWISE if self.mg_levelwise else 0),
                          int(self.member_tile))


class SolveResult(NamedTuple):
    x: torch.Tensor          # (N_r, S)
    iters: np.ndarray        # (S,) int32
    status: np.ndarray       # (S,) int32
    relres: np.ndarray       # (S,) float64
    ens_iters: int           # max_s iters_s
    stats: dict


def _require_cuda(t: torch.Tensor, name: str, shape=None, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _p(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _stream(dev: torch.device) -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ensemble_width(t: torch.Tensor) -> int:
    return int(t.shape[-1])


def _host_params(y, d: int, name: str = "y") -> np.ndarray:
    """Parameters (S, d) as a contiguous float64 host array (the library
    reads them from host memory).  Accepts a torch tensor on any device or
    anything numpy converts."""
    if isinstance(y, torch.Tensor):
        y = y.detach().to("cpu", torch.float64)
        y = y.numpy()
    y = np.ascontiguousarray(y, dtype=np.float64)
    if y.ndim != 2 or y.shape[1] != d:
        raise ValueError(f"{name} must have shape (S, {d}), got {y.shape}")
    return y


def _device_of(y, device):
    if device is not None:
        return torch.device(device)
    if isinstance(y, torch.Tensor) and y.is_cuda:
        return y.device
    return torch.device("cuda")


def workspace_bytes(prob: Problem, S: int, opts: Optional[SolverOptions] = None) -> int:
    """Bytes of the workspace `workspace` allocates (ens_pcg_workspace_bytes;
    with Jacobi, the larger Chebyshev layout that cheb_apply also needs)."""
    opts = opts or SolverOptions()
    o = opts.c()
    pc = prob.c()
    nb = L.lib().ens_pcg_workspace_bytes(C.byref(pc), C.byref(o), S)
    if opts.precond == "jacobi":
        o2 = SolverOptions(precond="chebyshev").c()
        nb = max(nb, L.lib().ens_pcg_workspace_bytes(C.byref(pc), C.byref(o2), S))
    if nb == 0:
        raise ValueError("invalid problem / options / ensemble width")
    return int(nb)


def workspace(prob: Problem, S: int, opts: Optional[SolverOptions] = None,
              device=None) -> torch.Tensor:
    """A device workspace large enough for solve / adjoint_grad / cheb_apply."""
    return torch.empty(workspace_bytes(prob, S, opts), dtype=torch.uint8, device=device or "cuda")


def matrix_slot_stride(prob: Problem, S: int) -> int:
    """Elements from one matrix slot to the next (ens_matrix_slot_stride)."""
    pc = prob.c()
    L_ = int(L.lib().ens_matrix_slot_stride(C.byref(pc), S))
    if L_ == 0:
        raise ValueError("invalid problem / ensemble width")
    return L_


def empty_matrix(prob: Problem, S: int, device=None) -> torch.Tensor:
    """An uninitialised ensemble matrix: a (slots, N_r, S) view with the
    library's slot stride (slot k starts at element k * matrix_slot_stride)."""
    Ls = matrix_slot_stride(prob, S)
    buf = torch.empty(prob.slots * Ls, dtype=torch.float64, device=device or "cuda")
    return buf.as_strided((prob.slots, prob.rows, S), (Ls, S, 1))


def _require_matrix(V: torch.Tensor, prob: Problem, S: int):
    if not isinstance(V, torch.Tensor) or not V.is_cuda or V.dtype != torch.float64:
        raise ValueError("V must be a float64 CUDA (HIP) tensor")
    if tuple(V.shape) != (prob.slots, prob.rows, S):
        raise ValueError(f"V has shape {tuple(V.shape)}, expected {(prob.slots, prob.rows, S)}")
    if V.stride() != (matrix_slot_stride(prob, S), S, 1):
        raise ValueError("V must have the library's slot stride (use assemble or empty_matrix)")


def assemble(prob: Problem, y, device=None):
    """Ensemble matrix V (slots, N_r, S; slot stride matrix_slot_stride) and
    right-hand side b (N_r, S) for parameters y (S, d), any S in [1, 64].
    The outputs live on ``device`` (default: y's GPU, else the current one)."""
    yh = _host_params(y, prob.d)
    S = int(yh.shape[0])
    dev = _device_of(y, device)
    V = empty_matrix(prob, S, dev)
    b = torch.empty((prob.rows, S), dtype=torch.float64, device=dev)
    pc = prob.c()
    L.check(L.lib().ens_assemble_ensemble(C.byref(pc), S, yh.ctypes.data_as(L.f64p), _p(V), _p(b),
                                          _stream(dev)), "ens_assemble_ensemble")
    return V, b


def solve(prob: Problem, V: torch.Tensor, b: torch.Tensor, opts: Optional[SolverOptions] = None,
          x: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> SolveResult:
    """Ensemble PCG for every member; blocks until the counts are known."""
    opts = opts or SolverOptions()
    S = _ensemble_width(b)
    _require_matrix(V, prob, S)
    _require_cuda(b, "b", (prob.rows, S))
    if x is None:
        x = torch.empty_like(b)
    _require_cuda(x, "x", (prob.rows, S))
    if ws is None:
        ws = workspace(prob, S, opts, V.device)
    _require_cuda(ws, "ws", dtype=torch.uint8)
    iters = np.zeros(S, np.int32)
    status = np.zeros(S, np.int32)
    relres = np.zeros(S, np.float64)
    ens_iters = C.c_int32(0)
    stats = L.ens_stats()
    pc, oc = prob.c(), opts.c()
    L.check(L.lib().ens_pcg_solve(
        C.byref(pc), C.byref(oc), S, _p(V), _p(b), _p(x),
        iters.ctypes.data_as(L.i32p), status.ctypes.data_as(L.i32p),
        relres.ctypes.data_as(L.f64p), C.byref(ens_iters), C.byref(stats),
        _p(ws), ws.numel(), _stream(V.device)), "ens_pcg_solve")
    st = {"ens_iters": stats.ens_iters, "spmv_timed": stats.spmv_timed,
          "spmv_ms": stats.spmv_ms, "spmv_groups": stats.spmv_groups,
          "tile_lines": stats.tile_lines}
    return SolveResult(x, iters, status, relres, int(ens_iters.value), st)


def solve_noalloc(prob: Problem, V: torch.Tensor, b: torch.Tensor,
                  opts: Optional[SolverOptions] = None, x: Optional[torch.Tensor] = None):
    """The solve of `solve` through ens_pcg_solve_noalloc: the library's own
    per-device workspace, nothing allocated by the call (x must be given for
    that).  Calls that overlap on one device race.  Returns SolveResult
    (stats empty)."""
    opts = opts or SolverOptions()
    S = _ensemble_width(b)
    _require_matrix(V, prob, S)
    _require_cuda(b, "b", (prob.rows, S))
    if x is None:
        x = torch.empty_like(b)
    _require_cuda(x, "x", (prob.rows, S))
    iters = np.zeros(S, np.int32)
    status = np.zeros(S, np.int32)
    relres = np.zeros(S, np.float64)
    ens_iters = C.c_int32(0)
    pc, oc = prob.c(), opts.c()
    L.check(L.lib().ens_pcg_solve_noalloc(
        C.byref(pc), C.byref(oc), S, _p(V), _p(b), _p(x),
        iters.ctypes.data_as(L.i32p), status.ctypes.data_as(L.i32p),
        relres.ctypes.data_as(L.f64p), C.byref(ens_iters), _stream(V.device)),
        "ens_pcg_solve_noalloc")
    return SolveResult(x, iters, status, relres, int(ens_iters.value), {})


def spmv(prob: Problem, V: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    S = _ensemble_width(p)
    _require_matrix(V, prob, S)
    _require_cuda(p, "p", (prob.rows, S))
    q = torch.empty_like(p)
    pc = prob.c()
    L.check(L.lib().ens_spmv(C.byref(pc), S, _p(V), _p(p), _p(q), _stream(p.device)), "ens_spmv")
    return q


def cheb_apply(prob: Problem, V: torch.Tensor, r: torch.Tensor,
               opts: Optional[SolverOptions] = None, ws: Optional[torch.Tensor] = None):
    """z = M^-1 r for the Chebyshev preconditioner; returns (z, lambda_max per member)."""
    opts = opts or SolverOptions(precond="chebyshev")
    S = _ensemble_width(r)
    _require_matrix(V, prob, S)
    _require_cuda(r, "r", (prob.rows, S))
    if ws is None:
        ws = workspace(prob, S, SolverOptions(precond="chebyshev"), r.device)
    z = torch.empty_like(r)
    lmax = np.zeros(S, np.float64)
    pc, oc = prob.c(), opts.c()
    L.check(L.lib().ens_cheb_apply(C.byref(pc), C.byref(oc), S, _p(V), _p(r), _p(z),
                                   lmax.ctypes.data_as(L.f64p), _p(ws), ws.numel(),
                                   _stream(r.device)), "ens_cheb_apply")
    return z, lmax


def mg_apply(prob: Problem, V: torch.Tensor, r: torch.Tensor,
             opts: Optional[SolverOptions] = None, ws: Optional[torch.Tensor] = None):
    """z = V(r), one multigrid V-cycle (3-D model, n + 1 a power of two);
    returns (z, fine-level lambda_max per member)."""
    opts = opts or SolverOptions(precond="multigrid")
    S = _ensemble_width(r)
    _require_matrix(V, prob, S)
    _require_cuda(r, "r", (prob.rows, S))
    if ws is None:
        ws = workspace(prob, S, SolverOptions(precond="multigrid"), r.device)
    z = torch.empty_like(r)
    lmax = np.zeros(S, np.float64)
    pc, oc = prob.c(), opts.c()
    L.check(L.lib().ens_mg_apply(C.byref(pc), C.byref(oc), S, _p(V), _p(r), _p(z),
                                 lmax.ctypes.data_as(L.f64p), _p(ws), ws.numel(),
                                 _stream(r.device)), "ens_mg_apply")
    return z, lmax


def member_dot(a: torch.Tensor, b: torch.Tensor, ws: Optional[torch.Tensor] = None) -> np.ndarray:
    """Per-member dot products; b may be (N_r, S) or a shared (N_r,) vector."""
    S = _ensemble_width(a)
    Nr = int(a.shape[0])
    _require_cuda(a, "a", (Nr, S))
    bcast = b.dim() == 1
    _require_cuda(b, "b", (Nr,) if bcast else (Nr, S))
    if ws is None:
        ws = workspace(Problem(2, 2), S, None, a.device)
    out = np.zeros(S, np.float64)
    L.check(L.lib().ens_member_dot(Nr, S, _p(a), _p(b), 1 if bcast else 0,
                                   out.ctypes.data_as(L.f64p), _p(ws), ws.numel(),
                                   _stream(a.device)), "ens_member_dot")
    return out


def param_indicator(prob: Problem, y, ws: Optional[torch.Tensor] = None,
                    device=None) -> np.ndarray:
    """H(y) per member (S,): the largest eigenvalue ratio of the diffusion
    tensor over the domain (the parameter-based grouping indicator)."""
    yh = _host_params(y, prob.d)
    S = int(yh.shape[0])
    dev = ws.device if ws is not None else _device_of(y, device)
    if ws is None:
        ws = workspace(Problem(2, 2), S, None, dev)
    h = np.zeros(S, np.float64)
    pc = prob.c()
    L.check(L.lib().ens_param_indicator(C.byref(pc), S, yh.ctypes.data_as(L.f64p),
                                        h.ctypes.data_as(L.f64p), _p(ws), ws.numel(), _stream(dev)),
            "ens_param_indicator")
    return h


def param_indicator_samples(prob: Problem, ys: np.ndarray, device="cuda") -> np.ndarray:
    """H for any number of samples (M, d), in member batches of 64."""
    ys = np.asarray(ys, dtype=np.float64)
    out = np.zeros(len(ys))
    ws = workspace(Problem(2, 2), 64, None, device)
    for a in range(0, len(ys), 64):
        blk = ys[a:a + 64]
        out[a:a + len(blk)] = param_indicator(prob, blk, ws)
    return out


def dqdy(prob: Problem, y, u: torch.Tensor, lam: torch.Tensor,
         ws: Optional[torch.Tensor] = None) -> np.ndarray:
    """-lambda^T (dA/dy_j) u per member, shape (S, d)."""
    yh = _host_params(y, prob.d)
    S = int(yh.shape[0])
    _require_cuda(u, "u", (prob.rows, S))
    _require_cuda(lam, "lam", (prob.rows, S))
    if ws is None:
        ws = workspace(Problem(2, 2), S, None, u.device)
    g = np.zeros((S, prob.d), np.float64)
    pc = prob.c()
    L.check(L.lib().ens_dqdy(C.byref(pc), S, yh.ctypes.data_as(L.f64p), _p(u), _p(lam),
                             g.ctypes.data_as(L.f64p), _p(ws), ws.numel(), _stream(u.device)),
            "ens_dqdy")
    return g


def adjoint_grad(prob: Problem, y, V: torch.Tensor, u: torch.Tensor,
                 w: torch.Tensor, opts: Optional[SolverOptions] = None,
                 ws: Optional[torch.Tensor] = None):
    """(lambda, dQ/dy (S, d), iters, status) for Q = w^T u."""
    opts = opts or SolverOptions()
    yh = _host_params(y, prob.d)
    S = int(yh.shape[0])
    _require_matrix(V, prob, S)
    _require_cuda(u, "u", (prob.rows, S))
    _require_cuda(w, "w", (prob.rows,))
    if ws is None:
        ws = workspace(prob, S, opts, u.device)
    lam = torch.empty_like(u)
    g = np.zeros((S, prob.d), np.float64)
    iters = np.zeros(S, np.int32)
    status = np.zeros(S, np.int32)
    pc, oc = prob.c(), opts.c()
    L.check(L.lib().ens_adjoint_grad(
        C.byref(pc), C.byref(oc), S, yh.ctypes.data_as(L.f64p), _p(V), _p(u), _p(w), _p(lam),
        g.ctypes.data_as(L.f64p), iters.ctypes.data_as(L.i32p), status.ctypes.data_as(L.i32p),
        _p(ws), ws.numel(), _stream(u.device)), "ens_adjoint_grad")
    return lam, g, iters, status


def qoi_weights(n: int, device=None, dim: int = 2) -> torch.Tensor:
    """The QoI weights w (N_r,) of Q = w^T u, the mean over the interior nodes
    of [0.4, 0.6]^dim (ens_qoi_weights)."""
    prob = Problem(n, 4, 0, 0.0, dim=dim) if dim == 3 else Problem(n, 2)
    w = torch.empty(prob.rows, dtype=torch.float64, device=device or "cuda")
    pc = prob.c()
    L.check(L.lib().ens_qoi_weights(C.byref(pc), _p(w), _stream(w.device)), "ens_qoi_weights")
    return w


class BatchResult(NamedTuple):
    x: torch.Tensor
    iters: np.ndarray
    status: np.ndarray
    relres: np.ndarray
    ens_iters: int
    seconds: float           # device time from the batch start to this ensemble's retirement


def plan_waves(items, max_wave_bytes: float):
    """The waves of ``batch_solve``: item indices sorted by the bytes one CG
    iteration moves (120 B per member-row; ties by index) and packed greedily
    into waves of at most ``max_wave_bytes`` (a larger ensemble forms a wave
    of its own)."""
    cost = [120 * it["prob"].rows * _ensemble_width(it["b"]) for it in items]
    order = sorted(range(len(items)), key=lambda i: (cost[i], i))
    waves, cur, tot = [], [], 0
    for i in order:
        if cur and tot + cost[i] > max_wave_bytes:
            waves.append(cur)
            cur, tot = [], 0
        cur.append(i)
        tot += cost[i]
    waves.append(cur)
    return waves


def _solve_as_batch_item(it, opts: Optional[SolverOptions], start: float) -> "BatchResult":
    """One batch item through the single-ensemble solver; ``seconds`` is
    ``start`` plus the solve's wall time (it blocks until the counts are
    known)."""
    from dataclasses import replace
    o = replace(opts or SolverOptions(), tile_lines=int(it.get("tile_lines", 0)),
                member_tile=int(it.get("member_tile", 0)))
    t = time.perf_counter()
    r = solve(it["prob"], it["V"], it["b"], o, x=it.get("x"), ws=it.get("ws"))
    torch.cuda.synchronize()
    return BatchResult(r.x, r.iters, r.status, r.relres, int(r.ens_iters),
                       start + time.perf_counter() - t)


def batch_solve(items, opts: Optional[SolverOptions] = None, batch_ws: Optional[torch.Tensor] = None,
                max_wave_bytes="auto"):
    """Solve several ensembles together (ens_batch_solve).

    ``items``: sequence of dicts with keys ``prob`` (Problem), ``V``, ``b`` and
    optionally ``x``, ``ws`` (a Jacobi workspace of that ensemble) and
    ``tile_lines``.  Returns one BatchResult per item, in item order.

    ``max_wave_bytes``: solve the ensembles in waves instead of all at once,
    smallest first: ensembles sorted by the bytes one CG iteration moves
    (120 B per member-row) and packed greedily into waves of at most that
    many bytes (a larger ensemble forms a wave of its own).  The small
    ensembles retire early.  "auto" (the default) takes the autotuner's wave
    size (``autotune.tune_wave``), None solves all ensembles in one batch.
    A result's ``seconds`` then counts from the start of the first wave.  A
    wave of one ensemble is solved by the single-ensemble solver (``solve``,
    with the item's launch shape), which is faster than a batch of one:
    the batched kernels' unit tables and per-step graph cost it 2-4 % at
    512^2 and up to a third on small grids."""
    if isinstance(max_wave_bytes, str):
        if max_wave_bytes != "auto":
            raise ValueError("max_wave_bytes: a number of bytes, 'auto' or None")
        from . import autotune
        max_wave_bytes = autotune.tune_wave()["wave_bytes"] if len(items) > 1 else None
    if max_wave_bytes is not None and len(items) > 1:
        waves = plan_waves(items, max_wave_bytes)
        out = [None] * len(items)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for wv in waves:
            start = time.perf_counter() - t0
            if len(wv) == 1:
                out[wv[0]] = _solve_as_batch_item(items[wv[0]], opts, start)
                continue
            for i, r in zip(wv, batch_solve([items[i] for i in wv], opts, batch_ws, None)):
                out[i] = r._replace(seconds=start + r.seconds)
        return out
    opts = opts or SolverOptions()
    n = len(items)
    if n == 0:
        return []
    c_items = (L.ens_batch_item * n)()
    keep = []
    outs = []
    dev = None
    for k, it in enumerate(items):
        prob, V, b = it["prob"], it["V"], it["b"]
        S = _ensemble_width(b)
        _require_matrix(V, prob, S)
        _require_cuda(b, "b", (prob.rows, S))
        x = it.get("x")
        if x is None:
            x = torch.empty_like(b)
        _require_cuda(x, "x", (prob.rows, S))
        ws = it.get("ws")
        if ws is None:
            ws = workspace(prob, S, SolverOptions(), V.device)
        _require_cuda(ws, "ws", dtype=torch.uint8)
        iters = np.zeros(S, np.int32)
        status = np.zeros(S, np.int32)
        relres = np.zeros(S, np.float64)
        ci = c_items[k]
        ci.prob = prob.c()
        ci.S = S
        ci.tile_lines = int(it.get("tile_lines", 0))
        ci.member_tile = int(it.get("member_tile", 0))
        ci.V_dev, ci.b_dev, ci.x_dev = V.data_ptr(), b.data_ptr(), x.data_ptr()
        ci.ws_dev, ci.ws_bytes = ws.data_ptr(), ws.numel()
        ci.iters_host = iters.ctypes.data_as(L.i32p)
        ci.status_host = status.ctypes.data_as(L.i32p)
        ci.relres_host = relres.ctypes.data_as(L.f64p)
        keep.append((x, ws))
        outs.append((x, iters, status, relres))
        dev = V.device
    nb = L.lib().ens_batch_workspace_bytes(n)
    if batch_ws is None or batch_ws.numel() < nb:
        batch_ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    oc = opts.c()
    L.check(L.lib().ens_batch_solve(C.byref(oc), n, c_items, _p(batch_ws), batch_ws.numel(),
                                    _stream(dev)), "ens_batch_solve")
    return [BatchResult(x, it_, st_, rr_, int(c_items[k].ens_iters), float(c_items[k].seconds))
            for k, (x, it_, st_, rr_) in enumerate(outs)]


def stream_triad(a: torch.Tensor, b: torch.Tensor, c: torch.Tensor, scalar: float) -> None:
    """c = a + scalar * b on the device (ens_stream_triad); asynchronous."""
    for t, name in ((a, "a"), (b, "b"), (c, "c")):
        _require_cuda(t, name)
    if not (a.numel() == b.numel() == c.numel()):
        raise ValueError("a, b, c must have the same number of elements")
    L.check(L.lib().ens_stream_triad(_p(a), _p(b), _p(c), float(scalar), a.numel(),
                                     _stream(a.device)), "ens_stream_triad")


def stream_mix(src: torch.Tensor, dst: torch.Tensor, stride: int, n: int, nread: int,
               nwrite: int) -> None:
    """dst[w * stride + e] = sum_k src[k * stride + e] (ens_stream_mix);
    asynchronous."""
    _require_cuda(src, "src")
    _require_cuda(dst, "dst")
    if src.numel() < (nread - 1) * stride + n or dst.numel() < (nwrite - 1) * stride + n:
        raise ValueError("src / dst too small for the requested streams")
    L.check(L.lib().ens_stream_mix(_p(src), _p(dst), int(stride), int(n), int(nread), int(nwrite),
                                   _stream(src.device)), "ens_stream_mix")
