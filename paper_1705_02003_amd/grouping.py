"""Sparse-grid surrogate, grouping and refinement: host calls into libens.

Nodes are integer arrays ``level`` and ``index`` of shape (M, d) (see
ens_group_samples in include/ens.h for the 1-D hierarchy).  The cost ratio R
of the paper's eqs. (Rl) and (R) is plain integer bookkeeping and lives here.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from . import _lib as L


def _i32(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def group_samples(level, index, values, y_new, S: int) -> Tuple[np.ndarray, np.ndarray]:
    """Ensembles (n_groups, S) of sample ids ordered by the surrogate of
    ``values``, and the surrogate predictions at ``y_new``."""
    y_new = _f64(y_new)
    M_new, d = y_new.shape
    M = 0 if level is None else len(level)
    lv = _i32(level if M else np.zeros((0, d)), (M, d))
    ix = _i32(index if M else np.zeros((0, d)), (M, d))
    vv = _f64(values if M else np.zeros(0), (M,))
    ng = (M_new + S - 1) // S
    groups = np.zeros((ng, S), np.int32)
    pred = np.zeros(M_new, np.float64)
    L.check(L.lib().ens_group_samples(d, M, lv.ctypes.data_as(L.i32p), ix.ctypes.data_as(L.i32p),
                                      vv.ctypes.data_as(L.f64p), M_new,
                                      y_new.ctypes.data_as(L.f64p), S,
                                      groups.ctypes.data_as(L.i32p),
                                      pred.ctypes.data_as(L.f64p)), "ens_group_samples")
    return groups, pred


def group_variable(pred, widths, iter_seconds):
    """Ensembles of varying width with the least predicted time (Section 5):
    returns (groups, cost), groups a list of id arrays, each padded to its
    width by repeating its last sample, in ascending order of prediction."""
    pred = _f64(pred)
    M = len(pred)
    wd = _i32(widths)
    ts = _f64(iter_seconds, (len(wd),))
    order = np.zeros(M, np.int32)
    gw = np.zeros(max(M, 1), np.int32)
    gc = np.zeros(max(M, 1), np.int32)
    ng = L.i32(0)
    cost = L.f64(0.0)
    import ctypes as C
    L.check(L.lib().ens_group_variable(M, pred.ctypes.data_as(L.f64p), len(wd),
                                       wd.ctypes.data_as(L.i32p), ts.ctypes.data_as(L.f64p),
                                       order.ctypes.data_as(L.i32p), gw.ctypes.data_as(L.i32p),
                                       gc.ctypes.data_as(L.i32p), C.byref(ng), C.byref(cost)),
            "ens_group_variable")
    groups, at = [], 0
    for g in range(int(ng.value)):
        ids = order[at:at + gc[g]].tolist()
        at += int(gc[g])
        groups.append(np.array(ids + [ids[-1]] * (int(gw[g]) - len(ids)), np.int32))
    return groups, float(cost.value)


def surpluses(level, index, values) -> np.ndarray:
    lv, ix = _i32(level), _i32(index)
    M, d = lv.shape
    vv = _f64(values, (M,))
    out = np.zeros(M, np.float64)
    L.check(L.lib().ens_sg_surpluses(d, M, lv.ctypes.data_as(L.i32p), ix.ctypes.data_as(L.i32p),
                                     vv.ctypes.data_as(L.f64p), out.ctypes.data_as(L.f64p)),
            "ens_sg_surpluses")
    return out


def expectation(level, index, values) -> float:
    """Mean of the sparse-grid interpolant of ``values`` under the uniform
    density on [-1, 1]^d: the quantity of interest E[G^] (Section 2.1)."""
    lv, ix = _i32(level), _i32(index)
    M, d = lv.shape
    vv = _f64(values, (M,))
    out = np.zeros(1, np.float64)
    L.check(L.lib().ens_sg_expectation(d, M, lv.ctypes.data_as(L.i32p), ix.ctypes.data_as(L.i32p),
                                       vv.ctypes.data_as(L.f64p), out.ctypes.data_as(L.f64p)),
            "ens_sg_expectation")
    return float(out[0])


def coords(level, index) -> np.ndarray:
    lv, ix = _i32(level), _i32(index)
    M, d = lv.shape
    out = np.zeros((M, d), np.float64)
    L.check(L.lib().ens_sg_coords(d, M, lv.ctypes.data_as(L.i32p), ix.ctypes.data_as(L.i32p),
                                  out.ctypes.data_as(L.f64p)), "ens_sg_coords")
    return out


def refine(level, index, values, newest_level: int, tau_rel: float, budget: int):
    """New nodes (level, index) of the next adaptive level, canonical order."""
    lv, ix = _i32(level), _i32(index)
    M, d = lv.shape
    vv = _f64(values, (M,))
    cap = max(1, 2 * d * M)
    nl = np.zeros((cap, d), np.int32)
    ni = np.zeros((cap, d), np.int32)
    cnt = L.i32(0)
    import ctypes as C
    L.check(L.lib().ens_sg_refine(d, M, lv.ctypes.data_as(L.i32p), ix.ctypes.data_as(L.i32p),
                                  vv.ctypes.data_as(L.f64p), newest_level, float(tau_rel),
                                  budget, cap, nl.ctypes.data_as(L.i32p),
                                  ni.ctypes.data_as(L.i32p), C.byref(cnt)), "ens_sg_refine")
    k = int(cnt.value)
    return nl[:k].copy(), ni[:k].copy()


def initial_grid(d: int):
    """The level <= 1 grid: the centre and its 2d children."""
    root_l = np.zeros((1, d), np.int32)
    root_i = np.zeros((1, d), np.int32)
    nl, ni = refine(root_l, root_i, [1.0], 0, 0.0, 1 + 2 * d)
    return np.vstack([root_l, nl]), np.vstack([root_i, ni])


def chunk(order: Sequence[int], S: int) -> np.ndarray:
    """Cut an order into ensembles of S, padding with the last sample."""
    order = list(order)
    out = []
    for g in range(0, len(order), S):
        ids = order[g:g + S]
        ids = ids + [ids[-1]] * (S - len(ids))
        out.append(ids)
    return np.array(out, dtype=np.int32).reshape(-1, S)


def cost_ratio(groups: np.ndarray, iters: Sequence[int], S: int) -> float:
    """R: S * sum over ensembles of the max member count, over the sum of
    counts of the real samples (padding replicas counted once)."""
    iters = np.asarray(iters)
    num = S * int(sum(int(iters[g].max()) for g in np.asarray(groups)))
    real = np.unique(np.asarray(groups).reshape(-1))
    return num / float(iters[real].sum())


def cost_ratio_variable(groups, iters: Sequence[int]) -> float:
    """R for ensembles of any widths: sum over ensembles of width times the
    max member count, over the sum of counts of the real samples."""
    iters = np.asarray(iters)
    num = sum(len(g) * int(iters[np.asarray(g)].max()) for g in groups)
    real = np.unique(np.concatenate([np.asarray(g) for g in groups]))
    return num / float(iters[real].sum())


def ensemble_iteration_total(groups: np.ndarray, iters: Sequence[int]) -> int:
    iters = np.asarray(iters)
    return int(sum(int(iters[g].max()) for g in np.asarray(groups)))


def full_grid(d: int, L: int):
    """Every node of total level <= L (refine all nodes level by level)."""
    lv = np.zeros((1, d), np.int32)
    ix = np.zeros((1, d), np.int32)
    for level in range(L):
        vals = np.ones(len(lv))
        nl, ni = refine(lv, ix, vals, level, 0.0, 1 << 30)
        if len(nl) == 0:
            break
        lv, ix = np.vstack([lv, nl]), np.vstack([ix, ni])
    return lv, ix
