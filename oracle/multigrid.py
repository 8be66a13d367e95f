"""Geometric multigrid V-cycle for the 3-D trilinear model, as the CG
preconditioner.

Paper, Section 4: CG preconditioned by smoothed-aggregation AMG, a degree-2
Chebyshev smoother on every level of the hierarchy and a sparse direct solve
on the coarsest.  On the structured trilinear mesh the geometric counterpart
is built here; readings (the paper leaves the hierarchy to the AMG package):

  * hierarchy: a mesh of n + 1 = 2^k cells per direction (n interior nodes)
    is coarsened by two per level down to 2 cells (one interior node); the
    coarsest system is solved exactly (one unknown);
  * prolongation P: trilinear interpolation -- per direction weight 1 where a
    fine node coincides with a coarse one and 1/2 from each neighbour at a
    midpoint, boundary nodes carrying 0 -- restriction P^T, and the Galerkin
    coarse operator A_c = P^T A P;
  * smoother: the Chebyshev polynomial of degree 2 in D^-1 A on
    [lmax / 30, lmax], lmax the Gershgorin bound of D^-1 A (the reading of the
    solver's own Chebyshev preconditioner), applied to the residual equation
    from a zero start, before and after the coarse correction; pre- and
    post-smoother are the same polynomial, so the V-cycle is a symmetric
    positive definite operator and may precondition CG.

Unknown ordering as in fe3d: row (k m + j) m + i, x fastest.
"""
from __future__ import annotations

from typing import List

import numpy as np
import scipy.sparse as sp

from . import pcg as opcg

SMOOTH_DEGREE = 2
SMOOTH_RATIO = 30.0


def levels_of(n: int) -> List[int]:
    """Interior nodes per direction on each level, fine to coarsest: n, (n -
    1) / 2, ..., 1; n + 1 must be a power of two (at least 2)."""
    if n < 1 or (n + 1) & n:
        raise ValueError("multigrid needs n + 1 = 2^k cells per direction")
    out = [n]
    while out[-1] > 1:
        out.append((out[-1] - 1) // 2)
    return out


def prolongation_1d(mc: int) -> sp.csr_matrix:
    """(2 mc + 1) x mc: fine node 2I (1-based) takes coarse node I with weight
    1, fine node 2I +- 1 takes it with weight 1/2."""
    mf = 2 * mc + 1
    rows, cols, vals = [], [], []
    for I in range(1, mc + 1):
        for i, w in ((2 * I - 1, 0.5), (2 * I, 1.0), (2 * I + 1, 0.5)):
            rows.append(i - 1)
            cols.append(I - 1)
            vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mf, mc))


def prolongation(mc: int) -> sp.csr_matrix:
    """The trilinear interpolation from the mc^3 coarse to the (2 mc + 1)^3
    fine interior nodes (tensor product of the 1-D one, x fastest)."""
    P1 = prolongation_1d(mc)
    return sp.kron(P1, sp.kron(P1, P1)).tocsr()


def hierarchy(A, n: int):
    """Per level (fine first): (A_l, diag_l, lmax_l, P_l) with P_l the
    prolongation from level l + 1 (None on the coarsest)."""
    out = []
    ms = levels_of(n)
    Al = sp.csr_matrix(A)
    for l, m in enumerate(ms):
        dl = Al.diagonal().copy()
        lm = opcg.gershgorin_lmax(Al, dl)
        Pl = prolongation(ms[l + 1]) if l + 1 < len(ms) else None
        out.append((Al, dl, lm, Pl))
        if Pl is not None:
            Al = (Pl.T @ Al @ Pl).tocsr()
    return out


def smooth(A, diag, lmax, r):
    """The degree-2 Chebyshev polynomial in D^-1 A applied to r (zero start)."""
    return opcg.chebyshev_apply(A, diag, r, lmax, SMOOTH_RATIO, SMOOTH_DEGREE)


def vcycle(levels, b, l: int = 0):
    """x = V(b): pre-smoothing, coarse correction with the restricted
    residual, post-smoothing; the coarsest level (one unknown) exactly."""
    A, diag, lmax, P = levels[l]
    if P is None:
        return b / diag
    x = smooth(A, diag, lmax, b)
    rc = P.T @ (b - A @ x)
    x = x + P @ vcycle(levels, rc, l + 1)
    x = x + smooth(A, diag, lmax, b - A @ x)
    return x


def pcg(A, b, n: int, rtol: float, max_iter: int):
    """CG preconditioned by one V-cycle per application (see pcg.pcg)."""
    lv = hierarchy(A, n)
    return opcg.pcg(A, b, lv[0][1], rtol, max_iter, precond=lambda v: vcycle(lv, v))
