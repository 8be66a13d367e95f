"""Pins of the oracle's multigrid V-cycle (3-D trilinear model).

Pinned against: the coarse hat functions (the columns of the prolongation
are the coarse basis functions sampled at the fine nodes), the variational
property of nested finite-element spaces (with a constant coefficient the
Galerkin operator P^T A P is exactly the matrix assembled on the coarse
mesh, with three different axis coefficients so a transposed axis order
fails), the V-cycle against the matrix of its error propagation written in
closed form (the smoother as T_2 of the scaled D^-1 A), symmetry and
positivity of the V-cycle operator, the exact coarsest solve, and the
multigrid property that CG iteration counts stay bounded as the mesh is
refined where the Chebyshev polynomial's grow.
"""
import numpy as np
import pytest

from oracle import fe3d
from oracle import multigrid as mg


def test_levels():
    assert mg.levels_of(31) == [31, 15, 7, 3, 1]
    assert mg.levels_of(1) == [1]
    for bad in (0, 30, 32, 6):
        with pytest.raises(ValueError):
            mg.levels_of(bad)


@pytest.mark.parametrize("mc", [1, 3, 7])
def test_prolongation_columns_are_coarse_hats(mc):
    mf = 2 * mc + 1
    H, h = 1.0 / (mc + 1), 1.0 / (mf + 1)
    xf = np.arange(1, mf + 1) * h
    P1 = mg.prolongation_1d(mc).toarray()
    for I in range(1, mc + 1):
        hat = np.maximum(0.0, 1.0 - np.abs(xf - I * H) / H)
        assert np.array_equal(P1[:, I - 1], hat)
    # 3-D: products of the 1-D hats, x fastest
    P = mg.prolongation(mc).toarray()
    rng = np.random.default_rng(mc)
    for _ in range(5):
        I, J, K = rng.integers(1, mc + 1, 3)
        col = ((K - 1) * mc + (J - 1)) * mc + (I - 1)
        hx = np.maximum(0.0, 1.0 - np.abs(xf - I * H) / H)
        hy = np.maximum(0.0, 1.0 - np.abs(xf - J * H) / H)
        hz = np.maximum(0.0, 1.0 - np.abs(xf - K * H) / H)
        ref = (hz[:, None, None] * hy[None, :, None] * hx[None, None, :]).reshape(-1)
        assert np.array_equal(P[:, col], ref)


@pytest.mark.parametrize("mc,a0,ay,az", [(3, 1.0, 1.0, 1.0), (3, 2.5, 0.3, 7.0), (7, 0.4, 3.0, 1.5)])
def test_galerkin_operator_is_the_coarse_assembly(mc, a0, ay, az):
    mf = 2 * mc + 1
    Af = fe3d.assemble_from_cells(np.full((mf + 1,) * 3, a0), mf, ay, az)
    Ac = fe3d.assemble_from_cells(np.full((mc + 1,) * 3, a0), mc, ay, az)
    P = mg.prolongation(mc)
    G = (P.T @ Af @ P).toarray()
    assert np.max(np.abs(G - Ac.toarray())) <= 1e-12 * np.abs(Ac.toarray()).max()


@pytest.mark.parametrize("m,seed", [(7, 0), (15, 1)])
def test_vcycle_is_symmetric_positive_definite(m, seed):
    rng = np.random.default_rng(seed)
    A, _, _ = fe3d.assemble(rng.uniform(-1, 1, 4), m)
    lv = mg.hierarchy(A, m)
    for _ in range(3):
        u, v = rng.standard_normal(m ** 3), rng.standard_normal(m ** 3)
        uv, vu = u @ mg.vcycle(lv, v), v @ mg.vcycle(lv, u)
        assert abs(uv - vu) <= 1e-11 * abs(uv)
        assert u @ mg.vcycle(lv, u) > 0


def test_coarsest_level_is_exact():
    A, b, d = fe3d.assemble([0.3, -0.2, 0.5, 0.1], 1)
    lv = mg.hierarchy(A, 1)
    assert np.array_equal(mg.vcycle(lv, b), b / d)
    x, I, st, _ = mg.pcg(A, b, 1, 1e-12, 10)
    assert I == 1 and st == 0 and np.allclose(A @ x, b, rtol=1e-14)


def test_iterations_stay_bounded_under_refinement():
    """Constant-coefficient and a variable-coefficient sample: MG-PCG counts
    at 7^3, 15^3, 31^3 interior nodes stay within a few iterations of each
    other (Jacobi-Chebyshev grows like 1/h), and the solutions are right."""
    for y in ([0.0, 0.0, 0.0, 0.0], [0.7, -0.4, 0.2, -0.9]):
        counts = []
        for m in (7, 15, 31):
            A, b, d = fe3d.assemble(y, m)
            x, I, st, _ = mg.pcg(A, b, m, 1e-8, 200)
            assert st == 0
            assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b) * 1.0001
            counts.append(I)
        assert max(counts) <= 20 and max(counts) - min(counts) <= 4, counts


def dense_vcycle_operator(A, n):
    """The V-cycle as a matrix, from its error propagation (test helper,
    dense, small n).  With G_l = T_2((theta I - D^-1 A)/delta) / T_2(theta /
    delta) the smoother's error propagation in closed form (T_2(x) = 2x^2 - 1,
    [theta -+ delta] = [lmax / 30, lmax]), a level's cycle has error
    propagation E_l = G_l (I - P_l V_{l+1} P_l^T A_l) G_l and is
    V_l = (I - E_l) A_l^-1; the one-node coarsest level has V = A^-1."""
    ms = mg.levels_of(n)
    As = [A.toarray()]
    Ps = []
    for l in range(len(ms) - 1):
        P = mg.prolongation(ms[l + 1]).toarray()
        Ps.append(P)
        As.append(P.T @ As[-1] @ P)

    def V(l):
        Al = As[l]
        if l == len(ms) - 1:
            return np.linalg.inv(Al)
        B = Al / np.diag(Al)[:, None]
        lmax = np.max(np.abs(Al).sum(axis=1) / np.diag(Al))
        lmin = lmax / 30.0
        th, de = (lmax + lmin) / 2, (lmax - lmin) / 2
        X = (th * np.eye(len(Al)) - B) / de
        G = (2 * X @ X - np.eye(len(Al))) / (2 * (th / de) ** 2 - 1)
        C = np.eye(len(Al)) - Ps[l] @ V(l + 1) @ Ps[l].T @ Al
        E = G @ C @ G
        return (np.eye(len(Al)) - E) @ np.linalg.inv(Al)

    return V(0)


@pytest.mark.parametrize("m,seed", [(3, 80), (7, 81)])
def test_vcycle_equals_its_error_propagation_form(m, seed):
    # pre-smoothing, residual restriction, coarse correction, prolongation
    # and post-smoothing each enter E: dropping or misplacing any of them
    # (or a wrong smoother interval) changes the operator
    rng = np.random.default_rng(seed)
    A, _, _ = fe3d.assemble(rng.uniform(-1, 1, 4), m)
    M = dense_vcycle_operator(A, m)
    lv = mg.hierarchy(A, m)
    for _ in range(3):
        b = rng.standard_normal(m ** 3)
        ref = M @ b
        assert np.linalg.norm(mg.vcycle(lv, b) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_multigrid_beats_the_chebyshev_polynomial_under_refinement():
    # Chebyshev-4 on D^-1 A grows like 1/h; one V-cycle per step does not
    from oracle import pcg as opcg
    y = [0.5, -0.3, 0.2, 0.4]
    mgc, chc = [], []
    for m in (7, 15, 31):
        A, b, d = fe3d.assemble(y, m)
        mgc.append(mg.pcg(A, b, m, 1e-8, 200)[1])
        chc.append(opcg.pcg(A, b, d, 1e-8, 2000, "chebyshev")[1])
    assert chc[2] >= 2 * chc[0] and mgc[2] <= mgc[0] + 3 and mgc[2] < chc[2], (mgc, chc)
