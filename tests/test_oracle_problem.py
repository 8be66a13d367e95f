"""Pins of the oracle's assembly against closed forms and invariants.

The reading of the discretisation (a conservative symmetric nine-point scheme
for -div(a K grad u)) is pinned by the textbook constant-coefficient stencil,
the closed-form spectrum of the anisotropic five-point Laplacian, symmetry,
positive definiteness, zero row sums, second-order convergence on a
manufactured solution, and the two geometric symmetries of the problem.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import problem

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def dense(y, n, eps_model=0, amp=0.4):
    A, b, diag = problem.assemble(np.asarray(y, float), n, eps_model, amp)
    return A.toarray(), b, diag


def test_constant_coefficient_reduces_to_textbook_nine_point():
    # a == 1 (d = 2): -(k11 u_11 + 2 k12 u_12 + k22 u_22) with the standard
    # central mixed difference (u_NE - u_NW - u_SE + u_SW) / (4 h^2).
    n = 7
    y = np.array([0.3, -0.45])
    _, _, k11, k22, k12 = problem.anisotropy(y, 0)
    h2 = 1.0 / (n + 1) ** 2
    text = {(0, 0): (2 * k11 + 2 * k22), (1, 0): -k11, (-1, 0): -k11,
            (0, 1): -k22, (0, -1): -k22,
            (1, 1): -2 * k12 / 4, (-1, -1): -2 * k12 / 4,
            (-1, 1): 2 * k12 / 4, (1, -1): 2 * k12 / 4}
    A, _, _ = dense(y, n)
    for j in range(n):
        for i in range(n):
            r = j * n + i
            for (di, dj), v in text.items():
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:
                    assert A[r, jj * n + ii] == pytest.approx(v / h2, rel=1e-13)
            assert np.count_nonzero(A[r]) <= 9


def test_five_point_anisotropic_spectrum_closed_form():
    # theta = 0 (y2 = -1) gives k12 = 0: the five-point operator with
    # eigenvectors sin(p pi i h) sin(q pi j h) and eigenvalues
    # (4/h^2)(k11 sin^2(p pi h / 2) + k22 sin^2(q pi h / 2)).
    n = 8
    y = np.array([0.2, -1.0])
    _, _, k11, k22, k12 = problem.anisotropy(y, 0)
    assert k12 == 0.0
    A, _, _ = dense(y, n)
    h = 1.0 / (n + 1)
    ii = np.arange(1, n + 1)
    expect = []
    for p in range(1, n + 1):
        for q in range(1, n + 1):
            lam = 4 / h**2 * (k11 * math.sin(p * math.pi * h / 2) ** 2
                              + k22 * math.sin(q * math.pi * h / 2) ** 2)
            v = np.outer(np.sin(q * math.pi * ii * h), np.sin(p * math.pi * ii * h)).reshape(-1)
            np.testing.assert_allclose(A @ v, lam * v, rtol=0, atol=1e-10 * lam)
            expect.append(lam)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(expect), rtol=1e-12)


def test_isotropic_limit_is_scaled_laplacian():
    # y1 = -1 gives eps = 1: K = I, k12 = 0 for any theta; diag = 4/h^2.
    n = 6
    A, _, diag = dense([-1.0, 0.37], n)
    h = 1.0 / (n + 1)
    np.testing.assert_allclose(diag, 4 / h**2, rtol=1e-14)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_symmetric_bitwise_and_positive_definite(seed):
    rng = np.random.default_rng(100 + seed)
    for eps_model, d, amp in [(0, 4, 0.4), (1, 8, 0.45), (0, 6, 0.4)]:
        y = rng.uniform(-1, 1, d)
        A, _, _ = dense(y, 12, eps_model, amp)
        assert np.array_equal(A, A.T)
        np.linalg.cholesky(A)
        assert np.linalg.eigvalsh(A)[0] > 0


def test_interior_rows_sum_to_zero():
    n = 10
    rng = np.random.default_rng(7)
    y = rng.uniform(-1, 1, 6)
    A, _, diag = dense(y, n, 0, 0.4)
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            r = j * n + i
            assert abs(A[r].sum()) <= 1e-13 * diag[r]


def test_boundary_couplings_dropped():
    vals = problem.stencil_values(np.array([0.1, 0.2, 0.3, -0.4]), 5, 0, 0.4).reshape(9, 5, 5)
    assert np.all(vals[[0, 3, 6], :, 0] == 0) and np.all(vals[[2, 5, 8], :, 4] == 0)
    assert np.all(vals[[0, 1, 2], 0, :] == 0) and np.all(vals[[6, 7, 8], 4, :] == 0)


def _mms(y, n, eps_model, amp):
    """Max nodal error for u = sin(pi x1) sin(pi x2) with the matching f."""
    _, _, k11, k22, k12 = problem.anisotropy(y, eps_model)
    x = np.arange(1, n + 1) / (n + 1)
    X1, X2 = np.meshgrid(x, x)               # [j, i]: X1 varies along i
    pi = math.pi
    u = np.sin(pi * X1) * np.sin(pi * X2)
    u1 = pi * np.cos(pi * X1) * np.sin(pi * X2)
    u2 = pi * np.sin(pi * X1) * np.cos(pi * X2)
    a = np.ones_like(X1)
    a1 = np.zeros_like(X1)
    a2 = np.zeros_like(X1)
    for k in range(1, len(y) - 1):
        c = amp * y[k + 1] / k**2
        a = a + c * np.sin(k * pi * X1) * np.sin(k * pi * X2)
        a1 = a1 + c * k * pi * np.cos(k * pi * X1) * np.sin(k * pi * X2)
        a2 = a2 + c * k * pi * np.sin(k * pi * X1) * np.cos(k * pi * X2)
    div_K_grad = -pi**2 * (k11 + k22) * u + 2 * k12 * pi**2 * np.cos(pi * X1) * np.cos(pi * X2)
    f = -a * div_K_grad - (a1 * (k11 * u1 + k12 * u2) + a2 * (k12 * u1 + k22 * u2))
    A, _, _ = problem.assemble(np.asarray(y), n, eps_model, amp)
    uh = spla.spsolve(A.tocsc(), f.reshape(-1))
    return np.max(np.abs(uh - u.reshape(-1)))


@pytest.mark.parametrize("y,eps_model,amp", [
    ([0.3, 0.4, 0.7, -0.5], 0, 0.4),
    ([-0.2, -0.6, 0.9, 0.8, -0.7, 0.5, 0.3, -0.9], 1, 0.45),
])
def test_manufactured_solution_second_order(y, eps_model, amp):
    errs = [_mms(np.array(y), n, eps_model, amp) for n in (15, 31, 63, 127)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in ratios), ratios
    assert errs[-1] < 2e-3


def test_transpose_and_centro_symmetry():
    # a(x1, x2) = a(x2, x1) = a(1 - x1, 1 - x2); y2 -> -y2 maps theta to
    # pi/2 - theta, which swaps k11 and k22: the solution transposes.
    n = 21
    y = np.array([0.25, 0.55, -0.4, 0.8])
    A, b, _ = problem.assemble(y, n, 0, 0.4)
    u = spla.spsolve(A.tocsc(), b).reshape(n, n)
    y2 = y.copy()
    y2[1] = -y2[1]
    A2, b2, _ = problem.assemble(y2, n, 0, 0.4)
    u2 = spla.spsolve(A2.tocsc(), b2).reshape(n, n)
    np.testing.assert_allclose(u2, u.T, rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(u[::-1, ::-1], u, rtol=1e-11, atol=1e-14)


def test_qoi_weights_window():
    for n, lo, hi in [(64, 26, 39), (512, 206, 307)]:
        w = problem.qoi_weights(n).reshape(n, n)
        idx = np.nonzero(w[lo - 1])[0] + 1
        assert idx[0] == lo and idx[-1] == hi
        assert w.sum() == pytest.approx(1.0, rel=1e-14)
        assert np.count_nonzero(w) == (hi - lo + 1) ** 2


@pytest.mark.parametrize("eps_model", [0, 1])
def test_tensor_is_rotated_diag(eps_model):
    # K = R(theta) diag(1, eps) R(theta)^T with R the counter-clockwise
    # rotation: (cos, sin) is the unit-eigenvalue direction, (-sin, cos) the
    # eps direction; eps and theta follow the two coefficient models.
    rng = np.random.default_rng(3)
    for y in rng.uniform(-1, 1, (5, 2)):
        eps, theta, k11, k22, k12 = problem.anisotropy(y, eps_model)
        expect_eps = 10 ** (-(1 + y[0])) if eps_model == 0 else 10 ** (-(1.5 + 1.5 * y[0]))
        assert eps == pytest.approx(expect_eps, rel=1e-14)
        assert theta == pytest.approx(math.pi / 4 * (1 + y[1]), rel=1e-14)
        K = np.array([[k11, k12], [k12, k22]])
        v1 = np.array([math.cos(theta), math.sin(theta)])
        v2 = np.array([-math.sin(theta), math.cos(theta)])
        np.testing.assert_allclose(K @ v1, v1, atol=1e-15)
        np.testing.assert_allclose(K @ v2, eps * v2, atol=1e-15)


def test_param_indicator_is_the_tensor_eigenvalue_ratio():
    rng = np.random.default_rng(3)
    for eps_model in (0, 1):
        for _ in range(5):
            y = rng.uniform(-1, 1, 4)
            _, _, k11, k22, k12 = problem.anisotropy(y, eps_model)
            for a in (0.6, 1.0, 1.7):      # a(x) > 0 scales both eigenvalues
                ev = np.linalg.eigvalsh(a * np.array([[k11, k12], [k12, k22]]))
                assert problem.param_indicator(y, eps_model) == pytest.approx(ev[-1] / ev[0], rel=1e-12)
