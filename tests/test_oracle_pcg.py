"""Pins of the oracle's PCG, Chebyshev preconditioner and ensemble emulator.

Pinned against dense direct solves (n <= 8), scipy's CG (a library
cross-check on iteration counts), the true residual, finite termination,
the closed-form Chebyshev polynomial on Laplacian eigenvectors, and the
member-by-member equality of the lock-step emulator with per-sample solves.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import BREAKDOWN, CONVERGED, MAX_ITER, ZERO_RHS, pcg, problem


def sample(seed, d=4, eps_model=0):
    return np.random.default_rng(seed).uniform(-1, 1, d)


@pytest.mark.parametrize("n", [4, 6, 8])
def test_matches_dense_direct_solve(n):
    for seed in range(3):
        y = sample(seed)
        A, b, diag = problem.assemble(y, n, 0, 0.4)
        Ad = A.toarray()
        xd = np.linalg.solve(Ad, b)
        rtol = 1e-8
        x, I, st, _ = pcg.pcg(A, b, diag, rtol, 5000)
        assert st == CONVERGED
        kappa = np.linalg.cond(Ad)
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= kappa * rtol
        # finite termination: a tight tolerance is reached within N_r (+ slack)
        x2, I2, st2, _ = pcg.pcg(A, b, diag, 1e-13, 5000)
        assert st2 == CONVERGED and I2 <= n * n + 5
        np.testing.assert_allclose(x2, xd, rtol=1e-10)


@pytest.mark.parametrize("eps_model,d,n", [(0, 4, 32), (1, 8, 24), (0, 2, 40)])
def test_iteration_counts_match_scipy_cg(eps_model, d, n):
    for seed in range(3):
        y = sample(seed + 10, d)
        A, b, diag = problem.assemble(y, n, eps_model, 0.4)
        rtol = 1e-8
        x, I, st, _ = pcg.pcg(A, b, diag, rtol, 20000)
        count = [0]

        def cb(_):
            count[0] += 1
        Minv = sp.diags(1.0 / diag)
        xs, info = spla.cg(A, b, rtol=rtol, atol=0.0, M=Minv, maxiter=20000, callback=cb)
        assert info == 0 and st == CONVERGED
        assert abs(count[0] - I) <= 1
        np.testing.assert_allclose(x, xs, rtol=1e-6)


def test_true_residual_within_twice_rtol():
    for seed in range(4):
        y = sample(seed + 20, 6)
        A, b, diag = problem.assemble(y, 48, 0, 0.4)
        for rtol in (1e-6, 1e-8, 1e-10):
            x, I, st, rel = pcg.pcg(A, b, diag, rtol, 20000)
            assert st == CONVERGED and rel <= rtol
            assert np.linalg.norm(b - A @ x) <= 2 * rtol * np.linalg.norm(b)


def test_status_codes():
    A, b, diag = problem.assemble(sample(1), 10, 0, 0.4)
    x, I, st, _ = pcg.pcg(A, np.zeros_like(b), diag, 1e-8, 100)
    assert (I, st) == (0, ZERO_RHS) and not x.any()
    x, I, st, _ = pcg.pcg(A, b, diag, 1e-8, 1)
    assert (I, st) == (1, MAX_ITER)
    # a negative definite member breaks down at its first step (the guard)
    x, I, st, _ = pcg.pcg(-A, b, -diag, 1e-8, 100)
    assert st == BREAKDOWN and I == 1 and np.all(np.isfinite(x))


def _cheb_T(k, x):
    # closed forms of the Chebyshev polynomials of the first kind
    return {1: x, 2: 2 * x**2 - 1, 3: 4 * x**3 - 3 * x, 4: 8 * x**4 - 8 * x**2 + 1}[k]


def test_chebyshev_closed_form_on_laplacian_eigenvectors():
    # isotropic, a == 1: D = (4/h^2) I, D^-1 A has eigenvectors
    # sin(p pi i h) sin(q pi j h) with eigenvalues mu = sin^2(p pi h/2) + sin^2(q pi h/2).
    n = 9
    A, _, diag = problem.assemble(np.array([-1.0, 0.0]), n, 0, 0.0)
    h = 1.0 / (n + 1)
    lmax = pcg.gershgorin_lmax(A, diag)
    assert lmax == pytest.approx(2.0, rel=1e-14)
    lmin = lmax / 30.0
    th, de = (lmax + lmin) / 2, (lmax - lmin) / 2
    ii = np.arange(1, n + 1)
    for p, q in [(1, 1), (2, 5), (9, 9), (4, 7)]:
        v = np.outer(np.sin(q * math.pi * ii * h), np.sin(p * math.pi * ii * h)).reshape(-1)
        mu = math.sin(p * math.pi * h / 2) ** 2 + math.sin(q * math.pi * h / 2) ** 2
        P = (1 - _cheb_T(4, (th - mu) / de) / _cheb_T(4, th / de)) / mu
        z = pcg.chebyshev_apply(A, diag, v, lmax)
        np.testing.assert_allclose(z, P * (h * h / 4) * v, rtol=1e-11, atol=1e-14 * np.abs(z).max())


@pytest.mark.parametrize("y,n,eps_model,amp", [
    (np.array([0.7, 0.35, -0.9, 0.8]), 7, 0, 0.4),
    (np.array([-0.2, -0.6, 0.9, -0.7, 0.5, -0.4, 0.3, 0.8]), 6, 1, 0.45),
])
def test_gershgorin_bound_is_the_infinity_norm_of_jacobi_scaled_matrix(y, n, eps_model, amp):
    # max_i sum_j |a_ij| / a_ii is the maximum absolute row sum of D^-1 A,
    # i.e. its infinity norm, which numpy computes independently from the
    # dense matrix.  Anisotropic (theta off the axes) and variable a, so the
    # ratio differs from row to row and max(row sum) / max(diag) is another
    # number (checked, so that a mistake of that kind would fail here).
    A, _, diag = problem.assemble(y, n, eps_model, amp)
    Ad = A.toarray()
    DA = Ad / diag[:, None]
    lmax = pcg.gershgorin_lmax(A, diag)
    assert lmax == pytest.approx(np.linalg.norm(DA, np.inf), rel=1e-14)
    rowsum = np.abs(Ad).sum(axis=1)
    assert abs(rowsum.max() / diag.max() - lmax) > 1e-6 * lmax
    assert abs(np.mean(rowsum / diag) - lmax) > 1e-6 * lmax
    # Gershgorin: every eigenvalue of D^-1/2 A D^-1/2 (those of D^-1 A) lies
    # in [0, lmax]; its diagonal is 1, so the largest is at least 1
    ev = np.linalg.eigvalsh(Ad / np.sqrt(np.outer(diag, diag)))
    assert 1.0 <= ev.max() <= lmax * (1 + 1e-14) and ev.min() > 0


def test_gershgorin_bound_closed_form_constant_coefficient():
    # a == 1: every interior row is the same stencil, centre 2(k11 + k22),
    # E, W -k11, N, S -k22, corners +-k12/2 (times 1/h^2), so the largest
    # ratio is 2 + |k12| / (k11 + k22) = 2 + |(1 - eps) sin(theta) cos(theta)| / (1 + eps)
    for y1, y2 in [(0.3, 0.4), (-0.8, -0.25), (0.9, 0.9)]:
        A, _, diag = problem.assemble(np.array([y1, y2]), 9, 0, 0.0)
        eps = 10.0 ** (-(1.0 + y1))
        th = math.pi / 4 * (1 + y2)
        want = 2.0 + abs((1 - eps) * math.sin(th) * math.cos(th)) / (1 + eps)
        assert pcg.gershgorin_lmax(A, diag) == pytest.approx(want, rel=1e-13)


def test_chebyshev_pcg_converges_to_same_solution():
    y = sample(5, 8)
    A, b, diag = problem.assemble(y, 40, 1, 0.45)
    xj, Ij, sj, _ = pcg.pcg(A, b, diag, 1e-10, 20000)
    xc, Ic, sc, _ = pcg.pcg(A, b, diag, 1e-10, 20000, precond="chebyshev")
    assert sj == sc == CONVERGED
    assert Ic < Ij
    np.testing.assert_allclose(xc, xj, rtol=1e-7)
    assert np.linalg.norm(b - A @ xc) <= 2e-10 * np.linalg.norm(b)


def test_chebyshev_preconditioner_is_spd():
    # M^-1 = p(D^-1 A) D^-1 with p > 0 on (0, lmax]: symmetric positive definite
    y = sample(6, 8)
    n = 7
    A, _, diag = problem.assemble(y, n, 1, 0.45)
    lmax = pcg.gershgorin_lmax(A, diag)
    Minv = np.column_stack([pcg.chebyshev_apply(A, diag, e, lmax) for e in np.eye(n * n)])
    np.testing.assert_allclose(Minv, Minv.T, rtol=1e-10, atol=1e-18)
    assert np.linalg.eigvalsh((Minv + Minv.T) / 2)[0] > 0


@pytest.mark.parametrize("precond", ["jacobi", "chebyshev"])
def test_ensemble_emulator_equals_per_sample(precond):
    n, S = 20, 6
    ys = np.random.default_rng(42).uniform(-1, 1, (S, 4))
    sys_ = [problem.assemble(y, n, 0, 0.4) for y in ys]
    As = [s[0] for s in sys_]
    bs = [s[1].copy() for s in sys_]
    ds = [s[2] for s in sys_]
    bs[2] = np.zeros_like(bs[2])                        # a zero-rhs member
    As[4], ds[4] = -As[4], -ds[4]                       # an indefinite member
    xs, its, st, K = pcg.ensemble_pcg(As, bs, ds, 1e-8, 5000, precond)
    assert st[2] == ZERO_RHS and its[2] == 0
    assert st[4] == BREAKDOWN
    for s in range(S):
        x1, I1, st1, _ = pcg.pcg(As[s], bs[s], ds[s], 1e-8, 5000, precond)
        assert (its[s], st[s]) == (I1, st1)
        assert np.array_equal(xs[s], x1)
    assert K == max(its)


def test_ensemble_emulator_max_iter():
    n = 16
    ys = np.random.default_rng(1).uniform(-1, 1, (3, 4))
    sys_ = [problem.assemble(y, n, 0, 0.4) for y in ys]
    xs, its, st, K = pcg.ensemble_pcg([s[0] for s in sys_], [s[1] for s in sys_],
                                      [s[2] for s in sys_], 1e-8, 7)
    assert its == [7, 7, 7] and st == [MAX_ITER] * 3 and K == 7
