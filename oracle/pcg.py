"""Per-sample preconditioned CG and the lock-step ensemble emulator.

PCG is the textbook Hestenes-Stiefel recurrence (x0 = 0).  The paper solves
each sample with CG (Section 4) and, for ensembles, computes inner products
and norms per member so that every member converges at its own rate, while
the ensemble keeps iterating until all members are done (Section 2.3, the
paragraph after the commuted Kronecker system; Section 4, the convergence
test paragraph).

Readings of silent points (each listed in the design notes):
  * convergence: member i stops at the first k with ||r_k||_2 <= rtol ||b||_2,
    and its iteration count is I_i = k;
  * b = 0: I = 0, status ZERO_RHS, x = 0;
  * the A-conjugate-norm guard (Section 4, the paragraph on underflow): if
    sigma = p^T A p is not a positive finite number, the update is replaced by
    zero, the member is frozen with status BREAKDOWN and I = k;
  * k reaching max_iter without convergence: status MAX_ITER, I = max_iter.

Chebyshev: degree-4 semi-iteration on D^-1 A from z0 = 0 (residual
polynomial T_4), three operator applications per preconditioner call,
lambda_max from the Gershgorin bound of D^-1 A and lambda_min = lambda_max/30.
"""
from __future__ import annotations

import math

import numpy as np

from . import BREAKDOWN, CONVERGED, MAX_ITER, ZERO_RHS

CHEB_RATIO = 30.0
CHEB_DEGREE = 4


def gershgorin_lmax(A, diag):
    """max_i sum_j |a_ij| / a_ii: an upper bound on the spectrum of D^-1 A."""
    rowsum = np.asarray(abs(A).sum(axis=1)).reshape(-1)
    return float(np.max(rowsum / diag))


def chebyshev_apply(A, diag, r, lmax, ratio=CHEB_RATIO, degree=CHEB_DEGREE):
    """z = p(D^-1 A) D^-1 r with 1 - t p(t) = T_deg((theta - t)/delta) / T_deg(theta/delta).

    Chebyshev semi-iteration for D^-1 A z = D^-1 r started at z = 0
    (three-term form: theta, delta the centre and half-width of
    [lmax/ratio, lmax]).
    """
    lmin = lmax / ratio
    theta = (lmax + lmin) / 2.0
    delta = (lmax - lmin) / 2.0
    sigma1 = theta / delta
    rho0 = 1.0 / sigma1
    d = (r / diag) / theta
    z = d.copy()
    for _ in range(degree - 1):
        rho1 = 1.0 / (2.0 * sigma1 - rho0)
        d = (rho1 * rho0) * d + (2.0 * rho1 / delta) * ((r - A @ z) / diag)
        z = z + d
        rho0 = rho1
    return z


def pcg(A, b, diag, rtol, max_iter, precond="jacobi", lmax=None):
    """Solve A x = b by PCG.  Returns (x, I, status, relres).

    relres = ||r_I|| / ||b|| for the recurrence residual at exit.  `precond`
    is "jacobi", "chebyshev" or a callable v -> M^-1 v (an SPD operator).
    """
    n = b.shape[0]
    x = np.zeros(n)
    r = b.copy()
    bnorm = math.sqrt(float(np.dot(b, b)))
    if bnorm == 0.0:
        return x, 0, ZERO_RHS, 0.0
    if precond == "chebyshev" and lmax is None:
        lmax = gershgorin_lmax(A, diag)

    def M(v):
        if callable(precond):
            return precond(v)
        if precond == "jacobi":
            return v / diag
        return chebyshev_apply(A, diag, v, lmax)

    z = M(r)
    p = z.copy()
    rho = float(np.dot(r, z))
    for k in range(1, max_iter + 1):
        q = A @ p
        sigma = float(np.dot(p, q))
        if not (math.isfinite(sigma) and sigma > 0.0):
            rn = math.sqrt(float(np.dot(r, r)))
            return x, k, BREAKDOWN, rn / bnorm
        alpha = rho / sigma
        x = x + alpha * p
        r = r - alpha * q
        rn = math.sqrt(float(np.dot(r, r)))
        if rn <= rtol * bnorm:
            return x, k, CONVERGED, rn / bnorm
        z = M(r)
        rho_new = float(np.dot(r, z))
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return x, max_iter, MAX_ITER, rn / bnorm


def ensemble_pcg(As, bs, diags, rtol, max_iter, precond="jacobi"):
    """Lock-step ensemble PCG over S members with per-member masks.

    Emulates the ensemble solver's semantics: one loop counter for the whole
    ensemble, per-member inner products (not summed across members), a
    member freezes at its own convergence or breakdown and keeps its x, and
    the loop runs until every member is frozen.  Each member's arithmetic is
    the same sequence of numpy calls as ``pcg`` so results agree bitwise with
    the per-sample oracle.

    Returns (xs, iters, status, ensemble_iters) with ensemble_iters = max_i I_i.
    """
    S = len(As)
    lmaxs = [gershgorin_lmax(A, d) if precond == "chebyshev" else None
             for A, d in zip(As, diags)]

    def M(s, v):
        if precond == "jacobi":
            return v / diags[s]
        return chebyshev_apply(As[s], diags[s], v, lmaxs[s])

    xs = [np.zeros(b.shape[0]) for b in bs]
    rs = [b.copy() for b in bs]
    bnorm = [math.sqrt(float(np.dot(b, b))) for b in bs]
    iters = [0] * S
    status = [MAX_ITER] * S
    active = [True] * S
    ps, rhos = [None] * S, [0.0] * S
    for s in range(S):
        if bnorm[s] == 0.0:
            active[s], status[s] = False, ZERO_RHS
            continue
        z = M(s, rs[s])
        ps[s] = z.copy()
        rhos[s] = float(np.dot(rs[s], z))
    k = 0
    while any(active) and k < max_iter:
        k += 1
        for s in range(S):
            if not active[s]:
                continue
            q = As[s] @ ps[s]
            sigma = float(np.dot(ps[s], q))
            if not (math.isfinite(sigma) and sigma > 0.0):
                active[s], status[s], iters[s] = False, BREAKDOWN, k
                continue
            alpha = rhos[s] / sigma
            xs[s] = xs[s] + alpha * ps[s]
            rs[s] = rs[s] - alpha * q
            rn = math.sqrt(float(np.dot(rs[s], rs[s])))
            if rn <= rtol * bnorm[s]:
                active[s], status[s], iters[s] = False, CONVERGED, k
                continue
            z = M(s, rs[s])
            rho_new = float(np.dot(rs[s], z))
            beta = rho_new / rhos[s]
            rhos[s] = rho_new
            ps[s] = z + beta * ps[s]
    for s in range(S):
        if active[s]:
            iters[s], status[s] = max_iter, MAX_ITER
    return xs, iters, status, max(iters) if S else 0
