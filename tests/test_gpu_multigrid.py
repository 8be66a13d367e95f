"""GPU parity of the multigrid preconditioner of the 3-D model (one geometric
V-cycle per application: Galerkin coarse operators, degree-2 Chebyshev
smoothing, exact one-node coarsest solve) against the oracle's V-cycle and
MG-PCG, through the C ABI.

Every oracle computation takes the oracle's own assembled matrix (the
device's matches it to the last bits of the diffusivity's exp / cos / sin).
Tolerances: the fine-level Gershgorin bound within 1e-14 relative; one
V-cycle application within 1e-12 relative per member (the coarse operators,
the coarse bounds and the transfers differ from the oracle's in summation
order, and the smoother polynomials amplify that and the matrix's last-bit
differences by their norm, a few units; a 1e-13 relative perturbation of
every matrix entry moves the oracle's own V-cycle by 1e-13); MG-PCG
iteration counts within +-1 of the oracle's, the solution at equal count
within 1e-9 relative, true residual <= 2 rtol ||b||.  Reductions are
deterministic: permuting members permutes results bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import CONVERGED
from oracle import fe3d as ofe
from oracle import multigrid as omg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on an MI355X")
    from paper_1705_02003_amd import _lib
    _lib.lib()
    yield


def E():
    from paper_1705_02003_amd import ensemble
    return ensemble


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def log_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def assemble(m, ys, eps_model=0):
    ens = E()
    prob = ens.Problem(m, ys.shape[1], eps_model, dim=3)
    V, b = ens.assemble(prob, ys)
    return prob, V, b


def members_to_check(S):
    return list(range(S)) if S <= 8 else sorted({0, 1, S // 2, S - 2, S - 1})


@pytest.mark.parametrize("m,S,d,seed", [(7, 3, 4, 60), (15, 8, 4, 61), (3, 1, 2, 62), (15, 64, 3, 63),
                                        (31, 2, 4, 64)])
def test_vcycle_matches_oracle(m, S, d, seed):
    # odd S (idle member slots), a two-level hierarchy (m = 3), the widest
    # ensemble and a five-level one
    log_case(test="mg-apply", m=m, S=S, d=d)
    ens = E()
    rng = np.random.default_rng(seed)
    ys = rng.uniform(-1, 1, (S, d))
    prob, V, _ = assemble(m, ys)
    R = rng.standard_normal((m ** 3, S))
    z, lmax = ens.mg_apply(prob, V, to_dev(R))
    z = z.cpu().numpy()
    for s in members_to_check(S):
        A = ofe.assemble(ys[s], m)[0]
        lv = omg.hierarchy(A, m)
        assert lmax[s] == pytest.approx(lv[0][2], rel=1e-14)
        ref = omg.vcycle(lv, R[:, s])
        err = np.linalg.norm(z[:, s] - ref) / np.linalg.norm(ref)
        assert err <= 1e-12, (s, err)


def test_vcycle_is_symmetric_and_positive():
    # a property of the V-cycle at any size: u^T V(w) = w^T V(u), u^T V(u) > 0
    log_case(test="mg-symmetric")
    ens = E()
    m, S = 15, 4
    rng = np.random.default_rng(65)
    prob, V, _ = assemble(m, rng.uniform(-1, 1, (S, 4)))
    U = rng.standard_normal((m ** 3, S))
    W = rng.standard_normal((m ** 3, S))
    zu = ens.mg_apply(prob, V, to_dev(U))[0].cpu().numpy()
    zw = ens.mg_apply(prob, V, to_dev(W))[0].cpu().numpy()
    for s in range(S):
        a, b = W[:, s] @ zu[:, s], U[:, s] @ zw[:, s]
        assert abs(a - b) <= 1e-12 * np.linalg.norm(U[:, s]) * np.linalg.norm(zw[:, s])
        assert U[:, s] @ zu[:, s] > 0


def check_mg_solution(res, ys, m, rtol, test=1, real=None):
    x = res.x.cpu().numpy()
    worst = 0.0
    for s in (range(x.shape[1]) if real is None else real):
        A, b, _ = ofe.assemble(ys[s], m, test)
        xo, Io, so, _ = omg.pcg(A, b, m, rtol, 2000)
        assert so == CONVERGED and res.status[s] == CONVERGED
        assert abs(int(res.iters[s]) - Io) <= 1, (s, res.iters[s], Io)
        xe, _, _, _ = omg.pcg(A, b, m, 0.0, int(res.iters[s]))
        worst = max(worst, np.linalg.norm(x[:, s] - xe) / np.linalg.norm(xe))
        assert np.linalg.norm(b - A @ x[:, s]) <= 2 * rtol * np.linalg.norm(b)
    return worst


@pytest.mark.parametrize("m,S,d,seed,eps_model", [(15, 8, 4, 66, 0), (7, 5, 4, 67, 0), (15, 16, 4, 68, 1),
                                                  (31, 4, 4, 69, 0)])
def test_mg_pcg_matches_oracle(m, S, d, seed, eps_model):
    log_case(test="mg-pcg", m=m, S=S, d=d, eps_model=eps_model)
    ens = E()
    ys = np.random.default_rng(seed).uniform(-1, 1, (S, d))
    if eps_model == 1:   # one member in each of Test 2's bands
        for s, r in enumerate((0.2, 0.6, 1.2)):
            ys[s] = ys[s] / np.linalg.norm(ys[s]) * r
    prob, V, b = assemble(m, ys, eps_model)
    res = ens.solve(prob, V, b, ens.SolverOptions(precond="multigrid", rtol=1e-8))
    worst = check_mg_solution(res, ys, m, 1e-8, test=1 + eps_model, real=members_to_check(S))
    print("multigrid max rel diff", worst, "iters", res.iters.tolist())
    assert worst <= 1e-9


def test_mg_iterations_bounded_under_refinement():
    # the point of a multigrid preconditioner: the counts hardly grow with
    # the grid, where the Chebyshev polynomial's grow like 1 / h
    log_case(test="mg-refinement")
    ens = E()
    S = 4
    ys = np.random.default_rng(70).uniform(-1, 1, (S, 4))
    counts, cheb = {}, {}
    for m in (7, 15, 31):
        prob, V, b = assemble(m, ys)
        counts[m] = ens.solve(prob, V, b, ens.SolverOptions(precond="multigrid")).ens_iters
        cheb[m] = ens.solve(prob, V, b, ens.SolverOptions(precond="chebyshev")).ens_iters
    print("multigrid", counts, "chebyshev", cheb)
    assert counts[31] <= counts[7] + 3
    assert counts[31] < cheb[31]


def test_mg_permutation_bitwise_and_noalloc():
    log_case(test="mg-permutation")
    ens = E()
    m, S = 15, 6
    ys = np.random.default_rng(71).uniform(-1, 1, (S, 4))
    perm = np.array([3, 0, 5, 1, 4, 2])
    opts = ens.SolverOptions(precond="multigrid", rtol=1e-9)
    prob, V, b = assemble(m, ys)
    ref = ens.solve(prob, V, b, opts)
    _, Vp, bp = assemble(m, ys[perm])
    res = ens.solve(prob, Vp, bp, opts)
    assert np.array_equal(res.iters, ref.iters[perm])
    assert torch.equal(res.x, ref.x[:, perm])
    x = torch.empty_like(b)
    na = ens.solve_noalloc(prob, V, b, opts, x=x)
    assert np.array_equal(na.iters, ref.iters)
    assert torch.equal(na.x, ref.x)


def test_mg_adjoint_gradient_matches_jacobi():
    # the adjoint solve with the multigrid preconditioner: the same gradient
    # as with Jacobi, to the solves' tolerance
    log_case(test="mg-adjoint")
    ens = E()
    m, S, d = 15, 4, 4
    ys = np.random.default_rng(72).uniform(-1, 1, (S, d))
    prob, V, b = assemble(m, ys)
    w = ens.qoi_weights(m, dim=3)
    g = {}
    for pre in ("jacobi", "multigrid"):
        opts = ens.SolverOptions(precond=pre, rtol=1e-11)
        u = ens.solve(prob, V, b, opts).x
        _, g[pre], _, status = ens.adjoint_grad(prob, ys, V, u, w, opts)
        assert np.all(status == 0)
    np.testing.assert_allclose(g["multigrid"], g["jacobi"], rtol=1e-7, atol=1e-9 * np.abs(g["jacobi"]).max())


@pytest.mark.parametrize("m,S", [(7, 5), (15, 8), (31, 3), (15, 64)])
def test_fused_coarse_tail_equals_levelwise_bitwise(m, S):
    # the coarse levels of at most 7^3 nodes in one launch (one workgroup
    # per member, levels in LDS) against one launch per level operation:
    # the same operations in the same order, so the same bits
    log_case(test="mg-tail", m=m, S=S)
    ens = E()
    rng = np.random.default_rng(73 + m + S)
    ys = rng.uniform(-1, 1, (S, 4))
    prob, V, b = assemble(m, ys)
    R = to_dev(rng.standard_normal((m ** 3, S)))
    z_tail, _ = ens.mg_apply(prob, V, R)
    z_lw, _ = ens.mg_apply(prob, V, R, ens.SolverOptions(precond="multigrid", mg_levelwise=True))
    assert torch.equal(z_tail, z_lw)
    r_tail = ens.solve(prob, V, b, ens.SolverOptions(precond="multigrid", rtol=1e-9))
    r_lw = ens.solve(prob, V, b, ens.SolverOptions(precond="multigrid", rtol=1e-9, mg_levelwise=True))
    assert np.array_equal(r_tail.iters, r_lw.iters)
    assert torch.equal(r_tail.x, r_lw.x)
