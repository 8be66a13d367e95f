"""Pins of the oracle's adjoint gradient.

The face/node bilinear form is pinned against the assembled CSR matrix; the
gradient against a complex-step derivative with complex sparse direct solves
(exact to round-off) and against central finite differences with direct
solves; plus the identity lambda^T b = w^T u and the y2 -> -y2 symmetry.
"""
import numpy as np
import pytest

from oracle import adjoint, problem


@pytest.mark.parametrize("eps_model,d,amp", [(0, 6, 0.4), (1, 8, 0.45), (0, 2, 0.0)])
def test_bilinear_form_matches_assembled_matrix(eps_model, d, amp):
    n = 13
    rng = np.random.default_rng(3)
    y = rng.uniform(-1, 1, d)
    A, _, _ = problem.assemble(y, n, eps_model, amp)
    lam, u = rng.standard_normal(n * n), rng.standard_normal(n * n)
    ref = lam @ (A @ u)
    assert adjoint.bilinear(lam, u, y, n, eps_model, amp) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("eps_model,d,amp", [(0, 6, 0.4), (1, 8, 0.45)])
def test_gradient_matches_complex_step(eps_model, d, amp):
    n = 24
    y = np.random.default_rng(8).uniform(-1, 1, d)
    Q, g, u, lam = adjoint.qoi_and_grad(y, n, eps_model, amp)
    assert lam @ problem.rhs(n) == pytest.approx(Q, rel=1e-12)
    for j in range(d):
        cs = adjoint.qoi_complex_step(y, n, eps_model, amp, j)
        assert g[j] == pytest.approx(cs, rel=1e-9, abs=1e-12 * np.abs(g).max())


def test_gradient_matches_central_differences():
    n, d = 32, 6
    y = np.random.default_rng(12).uniform(-1, 1, d)
    _, g, _, _ = adjoint.qoi_and_grad(y, n, 0, 0.4)
    h = 1e-6
    for j in range(d):
        e = np.zeros(d)
        e[j] = h
        fd = (adjoint.qoi_direct(y + e, n, 0, 0.4) - adjoint.qoi_direct(y - e, n, 0, 0.4)) / (2 * h)
        # FD noise is (rounding of Q) / h, about 1e-9 of ||g||_inf here, so the
        # relative error of each component is taken against
        # max(|g_j|, 1e-2 ||g||_inf).
        assert abs(fd - g[j]) <= 1e-6 * max(abs(g[j]), 1e-2 * np.abs(g).max())


def test_gradient_in_y2_vanishes_at_zero_angle_offset():
    # Q(y1, y2, ...) = Q(y1, -y2, ...) because the QoI window is symmetric
    # under x1 <-> x2, so dQ/dy2 = 0 at y2 = 0.
    y = np.array([0.3, 0.0, 0.5, -0.2, 0.7, 0.1])
    _, g, _, _ = adjoint.qoi_and_grad(y, 30, 0, 0.4)
    assert abs(g[1]) <= 1e-10 * np.abs(g).max()
