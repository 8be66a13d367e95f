"""Pins of the oracle's 3-D trilinear finite-element model.

Pinned against: the eigen-decomposition of a fine Nystrom discretisation of
the 1-D exponential covariance (a library eigensolver), orthonormality, the
textbook 27-point stencil of the trilinear Laplacian, the closed-form
eigenpairs of the constant-coefficient anisotropic matrix (tensor products of
1-D stiffness and mass eigenvalues), symmetry and zero row sums, positive
definiteness, and second-order convergence of a manufactured solution.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import fe3d


def test_kl_1d_matches_nystrom_eigenpairs():
    n = 3000
    s = (np.arange(n) + 0.5) / n
    K = np.exp(-np.abs(s[:, None] - s[None, :]) / fe3d.DELTA) / n
    ev, evec = np.linalg.eigh(K)
    ev, evec = ev[::-1], evec[:, ::-1]
    modes = fe3d.kl_1d(6)
    for k, md in enumerate(modes):
        assert md[2] == pytest.approx(ev[k], rel=2e-4)
        phi = fe3d.phi_1d(md, s)
        # unit norm, and the same function as the discrete eigenvector
        assert np.sum(phi * phi) / n == pytest.approx(1.0, abs=1e-5)
        v = evec[:, k] * math.sqrt(n)
        v = v * np.sign(v @ phi)
        assert np.max(np.abs(v - phi)) < 2e-3
        # the integral equation itself
        np.testing.assert_allclose(K @ phi, md[2] * phi, atol=2e-3 * md[2])
    for a, b in itertools.combinations(modes, 2):
        assert abs(np.sum(fe3d.phi_1d(a, s) * fe3d.phi_1d(b, s)) / n) < 1e-5


def test_kl_3d_order_and_ties():
    terms, m1 = fe3d.kl_3d(10)
    lams = [t[0] ** 2 for t in terms]
    assert all(a >= b for a, b in zip(lams, lams[1:]))
    assert terms[0][1] == (0, 0, 0)
    # the three permutations of (0, 0, 1) tie exactly and come in index order
    assert [t[1] for t in terms[1:4]] == [(0, 0, 1), (0, 1, 0), (1, 0, 0)]
    assert terms[1][0] == terms[2][0] == terms[3][0]
    assert lams[0] == pytest.approx(fe3d.SIGMA0 * m1[0][2] ** 3, rel=1e-15)


def test_trilinear_laplacian_stencil():
    m = 5
    h = 1.0 / (m + 1)
    A = fe3d.assemble_from_cells(np.ones((m + 1,) * 3), m, 1.0, 1.0)
    V = fe3d.slot_values(A, m)
    r = (2 * m + 2) * m + 2           # the centre node: no boundary neighbour
    for s, (di, dj, dk) in enumerate(fe3d.SLOT_OFFSETS):
        nz = abs(di) + abs(dj) + abs(dk)
        want = {0: 8.0 / 3.0, 1: 0.0, 2: -1.0 / 6.0, 3: -1.0 / 12.0}[nz] * h
        assert V[s, r] == pytest.approx(want, abs=1e-15)


@pytest.mark.parametrize("a0,ay,az", [(1.0, 1.0, 1.0), (0.3, 2.0, 5.0)])
def test_constant_coefficient_eigenpairs(a0, ay, az):
    # 1-D Dirichlet stiffness and mass share the sine eigenvectors:
    # mu_p = (2/h)(1 - cos(p pi h)), nu_p = (h/3)(2 + cos(p pi h)); the cube
    # matrix a0 Kx My Mz + ay Mx Ky Mz + az Mx My Kz has eigenvalue
    # a0 mu_p nu_q nu_r + ay nu_p mu_q nu_r + az nu_p nu_q mu_r.
    m = 6
    h = 1.0 / (m + 1)
    A = fe3d.assemble_from_cells(np.full((m + 1,) * 3, a0), m, ay, az)
    x = np.arange(1, m + 1) * h
    for p, q, r in [(1, 1, 1), (2, 3, 1), (6, 5, 4)]:
        v = np.einsum("k,j,i->kji", np.sin(r * np.pi * x), np.sin(q * np.pi * x),
                      np.sin(p * np.pi * x)).reshape(-1)
        mu = lambda k: (2 / h) * (1 - math.cos(k * math.pi * h))
        nu = lambda k: (h / 3) * (2 + math.cos(k * math.pi * h))
        lam = a0 * mu(p) * nu(q) * nu(r) + ay * nu(p) * mu(q) * nu(r) + az * nu(p) * nu(q) * mu(r)
        np.testing.assert_allclose(A @ v, lam * v, atol=1e-12 * lam)


def test_symmetric_zero_row_sums_and_spd():
    rng = np.random.default_rng(0)
    m = 4
    acell = rng.uniform(0.05, 20.0, (m + 1,) * 3)
    A = fe3d.assemble_from_cells(acell, m)
    D = A.toarray()
    assert np.array_equal(D, D.T)
    np.linalg.cholesky(D)
    # rows of nodes with no boundary neighbour: constants are in the kernel
    m2 = 5
    A2 = fe3d.assemble_from_cells(rng.uniform(0.05, 20.0, (m2 + 1,) * 3), m2)
    r = (2 * m2 + 2) * m2 + 2
    assert abs(A2[r].sum()) < 1e-13 * abs(A2[r, r])


def test_sample_matrix_is_spd_and_its_diagonal_is_slot_13():
    y = np.array([0.7, -0.4, 0.2, -0.9])
    m = 4
    A, b, dg = fe3d.assemble(y, m)
    np.linalg.cholesky(A.toarray())
    V = fe3d.slot_values(A, m)
    assert np.array_equal(V[fe3d.CENTER], dg)
    assert np.all(b == (1.0 / (m + 1)) ** 3)
    # the cell coefficients are a_min + a_hat exp(g) at the cube centres
    ac = fe3d.element_coefficients(y, m)
    assert ac.min() > fe3d.A_MIN


def test_manufactured_solution_second_order():
    # u = sin(pi x) sin(pi y) sin(pi z) with a constant: f = pi^2 (a0 + ay + az) u;
    # lumped load b = h^3 f(nodes); nodal error falls ~4x per halving of h
    a0, ay, az = 2.0, 1.0, 0.5
    errs = []
    for m in (5, 11, 23):
        h = 1.0 / (m + 1)
        A = fe3d.assemble_from_cells(np.full((m + 1,) * 3, a0), m, ay, az)
        x = np.arange(1, m + 1) * h
        u = np.einsum("k,j,i->kji", np.sin(np.pi * x), np.sin(np.pi * x), np.sin(np.pi * x)).reshape(-1)
        f = np.pi ** 2 * (a0 + ay + az) * u
        uh = sla.spsolve(A.tocsc(), h ** 3 * f)
        errs.append(np.max(np.abs(uh - u)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.6 < r2 < 4.4


def test_param_indicator():
    m = 5
    # y = 0: a = a_min + a_hat everywhere
    assert fe3d.param_indicator(np.zeros(4), m) == pytest.approx(fe3d.A_MIN + fe3d.A_HAT, rel=1e-15)
    y = np.array([0.9, -0.7, 0.3, 0.5])
    ac = fe3d.element_coefficients(y, m)
    ratios = [np.linalg.eigvalsh(np.diag([a, fe3d.A_Y, fe3d.A_Z])) for a in ac.reshape(-1)]
    assert fe3d.param_indicator(y, m) == pytest.approx(max(r[-1] / r[0] for r in ratios), rel=1e-15)


def test_anisotropic_stencil_closed_form():
    # constant coefficients: the assembled stencil is the tensor product of
    # the 1-D stencils K = (-1, 2, -1) / h and M = (1, 4, 1) h / 6:
    # a0 K(di) M(dj) M(dk) + ay M(di) K(dj) M(dk) + az M(di) M(dj) K(dk)
    m, a0, ay, az = 5, 0.3, 2.0, 5.0
    h = 1.0 / (m + 1)
    V = fe3d.slot_values(fe3d.assemble_from_cells(np.full((m + 1,) * 3, a0), m, ay, az), m)
    K = {-1: -1.0 / h, 0: 2.0 / h, 1: -1.0 / h}
    M = {-1: h / 6, 0: 4 * h / 6, 1: h / 6}
    r = (2 * m + 2) * m + 2
    for s, (di, dj, dk) in enumerate(fe3d.SLOT_OFFSETS):
        want = a0 * K[di] * M[dj] * M[dk] + ay * M[di] * K[dj] * M[dk] + az * M[di] * M[dj] * K[dk]
        assert V[s, r] == pytest.approx(want, abs=1e-14)


def test_cell_coefficients_are_taken_at_cube_centres():
    # the leading KL term is even about 1/2 in every direction, so with only
    # that term the cube-centre values are mirror-symmetric along each axis;
    # the second term (odd along z) flips sign under the z mirror
    m = 6
    a1 = fe3d.element_coefficients(np.array([0.8, 0.0, 0.0, 0.0]), m)
    for ax in range(3):
        np.testing.assert_allclose(a1, np.flip(a1, axis=ax), rtol=1e-13)
    g2 = np.log(fe3d.element_coefficients(np.array([0.0, 0.6, 0.0, 0.0]), m) - fe3d.A_MIN)
    np.testing.assert_allclose(g2, -np.flip(g2, axis=0), atol=1e-13)


@pytest.mark.parametrize("y", [[0.4, -0.7, 0.2, 0.9], [-0.9, 0.5, -0.3, 0.1, 0.8, -0.6]])
def test_adjoint_gradient_matches_complex_step(y):
    # Im Q(y + i h e_j) / h with a complex sparse direct solve is exact to
    # round-off; the adjoint form must agree to round-off
    y = np.asarray(y)
    m = 5
    Q, g, u, lam = fe3d.qoi_and_grad(y, m)
    cs = np.array([fe3d.qoi_complex_step(y, m, j) for j in range(len(y))])
    assert np.max(np.abs(g - cs)) <= 1e-12 * np.max(np.abs(cs))
    # lambda^T b = w^T u = Q
    A, b, _ = fe3d.assemble(y, m)
    assert lam @ b == pytest.approx(Q, rel=1e-13)


def test_qoi_weights_window():
    for m in (9, 14, 31):
        w = fe3d.qoi_weights(m).reshape(m, m, m)
        x = np.arange(1, m + 1) / (m + 1)
        inside = (x >= 0.4 - 1e-12) & (x <= 0.6 + 1e-12)
        assert np.array_equal(w > 0, inside[:, None, None] & inside[None, :, None] & inside[None, None, :])
        assert w.sum() == pytest.approx(1.0, rel=1e-14)


def _band_exact(y):
    """Test 2's band of y by exact rational arithmetic on the FP64 inputs:
    r^2 = sum y_i^2 against d^2/16 = 3/16 and d^2/4 = 3/4 (d = sqrt(3))."""
    from fractions import Fraction
    r2 = sum(Fraction(float(v)) ** 2 for v in y)
    return 1.0 if r2 < Fraction(3, 16) else (100.0 if r2 < Fraction(3, 4) else 10.0)


def test_test2_a_hat_bands():
    """a_hat(y) of the Test 2 equation: inside each band, exactly on both band
    edges (dyadic sparse-grid coordinates, where the squares are exact), just
    either side of the edges, and random points, against exact rational
    arithmetic; Test 1 is a_hat = 1 everywhere."""
    cases = [
        ([0.0, 0.0, 0.0, 0.0], 1.0), ([0.3, -0.2, 0.1, 0.0], 1.0),
        ([0.25, 0.25, 0.25, 0.0], 100.0),          # r = d/4 exactly: the middle band
        ([0.25, -0.25, 0.0, 0.25], 100.0),
        ([0.5, 0.0, 0.0, 0.0], 100.0), ([0.5, 0.5, 0.25, -0.25], 100.0),
        ([0.5, 0.5, 0.5, 0.0], 10.0),              # r = d/2 exactly: the outer band
        ([-0.5, 0.5, 0.0, -0.5], 10.0), ([1.0, 0.0, 0.0, 0.0], 10.0),
        ([0.4330127, 0.0, 0.0, 0.0], 1.0),         # d/4 = 0.43301270189...
        ([0.4330128, 0.0, 0.0, 0.0], 100.0),
        ([0.8660254, 0.0, 0.0, 0.0], 100.0),       # d/2 = 0.86602540378...
        ([0.8660255, 0.0, 0.0, 0.0], 10.0),
    ]
    for y, want in cases:
        assert fe3d.a_hat(y, 2) == want, y
        assert fe3d.a_hat(y, 1) == 1.0
        assert _band_exact(y) == want
    rng = np.random.default_rng(7)
    for y in rng.uniform(-1, 1, (400, 4)):
        assert fe3d.a_hat(y, 2) == _band_exact(y)
        r = math.sqrt(float(np.sum(y ** 2)))
        d = math.sqrt(3.0)
        assert fe3d.a_hat(y, 2) == (1.0 if r < d / 4 else (100.0 if r < d / 2 else 10.0))


@pytest.mark.parametrize("y,ah", [([0.1, -0.2, 0.1, 0.0], 1.0), ([0.5, 0.2, -0.3, 0.1], 100.0),
                                  ([0.7, -0.6, 0.4, 0.3], 10.0)])
def test_test2_field_and_matrix_scale_with_a_hat(y, ah):
    """Test 2 only rescales the exponential part: a - a_min = a_hat (a_1 -
    a_min) cell by cell, exactly, and the assembled matrix is that of the
    rescaled cells."""
    m = 6
    a1 = fe3d.element_coefficients(y, m, 1)
    a2 = fe3d.element_coefficients(y, m, 2)
    assert fe3d.a_hat(y, 2) == ah
    assert np.array_equal(a2 - fe3d.A_MIN, ah * (a1 - fe3d.A_MIN)) or \
        np.max(np.abs((a2 - fe3d.A_MIN) - ah * (a1 - fe3d.A_MIN))) <= 1e-15 * np.max(np.abs(a2))
    A2, _, _ = fe3d.assemble(y, m, 2)
    ref = fe3d.assemble_from_cells(fe3d.A_MIN + ah * (a1 - fe3d.A_MIN), m)
    assert abs(A2 - ref).max() <= 1e-14 * abs(ref).max()


@pytest.mark.parametrize("y", [[0.5, 0.2, -0.3, 0.1], [0.7, -0.6, 0.4, 0.3]])
def test_test2_adjoint_gradient_matches_complex_step(y):
    """Inside a band a_hat is constant, so dQ/dy is the Test 1 form with the
    band's factor; the adjoint form against a complex step."""
    y = np.asarray(y)
    m = 5
    Q, g, _, _ = fe3d.qoi_and_grad(y, m, test=2)
    cs = np.array([fe3d.qoi_complex_step(y, m, j, test=2) for j in range(len(y))])
    assert np.max(np.abs(g - cs)) <= 1e-12 * np.max(np.abs(cs))
