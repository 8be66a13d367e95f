"""Ensemble widths that are not powers of two (any S in [1, 64]; the paper's
Table 1 uses S = 20), through the C ABI against the oracle.

A width S runs on a power-of-two group of lanes per point; the extra slots
are idle.  Checks:
  * assembly, product and PCG solves (Jacobi, Chebyshev, member tiles with a
    ragged last tile, the 3-D model) against the oracle: counts +-1, the
    iterate at equal count within 1e-9 norm-wise and element-wise;
  * bitwise: an ensemble of S members equals the first S members of the same
    samples in an ensemble padded to the next power of two when both run on
    the same lanes (even S: S = 20, 24 against 32, S = 48 against 64), and
    replicas of a sample inside an odd-width ensemble equal the sample;
  * the dQ/dy kernel, the adjoint gradient and the grouping indicator at
    odd and even non-power-of-two widths;
  * the QoI weights from the library equal the oracle's, bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import CONVERGED
from oracle import adjoint as oadj
from oracle import fe3d as ofe
from oracle import pcg as opcg
from oracle import problem as oprob

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


def log_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def check_members(res, ys, n, eps_model, amp, rtol, precond="jacobi"):
    x = res.x.cpu().numpy()
    worst = 0.0
    for s in range(x.shape[1]):
        A, b, diag = oprob.assemble(ys[s], n, eps_model, amp)
        _, I, st, _ = opcg.pcg(A, b, diag, rtol, 20000, precond)
        assert st == CONVERGED and res.status[s] == CONVERGED, (s, st, res.status[s])
        assert abs(int(res.iters[s]) - I) <= 1, (s, res.iters[s], I)
        xe, _, _, _ = opcg.pcg(A, b, diag, 0.0, int(res.iters[s]), precond)
        worst = max(worst, np.linalg.norm(x[:, s] - xe) / np.linalg.norm(xe),
                    np.abs(x[:, s] - xe).max() / np.abs(xe).max())
        assert np.linalg.norm(b - A @ x[:, s]) <= 2 * rtol * np.linalg.norm(b)
    return worst


@pytest.mark.parametrize("n,S,d,eps_model,amp,kw", [
    (40, 3, 4, 0, 0.4, {}),
    (37, 20, 4, 0, 0.4, {}),
    (33, 24, 8, 1, 0.45, {}),
    (29, 48, 6, 0, 0.4, {}),
    (31, 5, 4, 0, 0.4, {"tile_lines": 3}),
    (26, 63, 4, 0, 0.4, {}),
    (35, 48, 4, 0, 0.4, {"member_tile": 32}),
    (30, 20, 4, 0, 0.4, {"member_tile": 8, "max_groups": 40}),
    (27, 45, 4, 0, 0.4, {"member_tile": 16}),
])
def test_widths_jacobi_match_oracle(n, S, d, eps_model, amp, kw):
    log_case(test="width-jacobi", n=n, S=S, **kw)
    ens = E()
    prob = ens.Problem(n, d, eps_model, amp)
    ys = np.random.default_rng(1000 + S).uniform(-1, 1, (S, d))
    V, b = ens.assemble(prob, ys)
    Vh = V.cpu().numpy()
    assert np.all(b.cpu().numpy() == 1.0)
    for s in range(S):
        ref = oprob.stencil_values(ys[s], n, eps_model, amp)
        assert np.array_equal(Vh[:, :, s] == 0.0, ref == 0.0)
        assert np.max(np.abs(Vh[:, :, s] - ref) / np.abs(ref[4])[None, :]) <= 4e-15
    P = np.random.default_rng(S).standard_normal((n * n, S))
    q = ens.spmv(prob, V, torch.tensor(P, device="cuda")).cpu().numpy()
    for s in (0, S // 2, S - 1):
        A = oprob.to_csr(oprob.stencil_values(ys[s], n, eps_model, amp), n)
        assert np.max(np.abs(q[:, s] - A @ P[:, s])) <= 1e-13 * np.abs(A).sum(axis=1).max() * np.abs(P[:, s]).max()
    res = ens.solve(prob, V, b, ens.SolverOptions(rtol=1e-8, **kw))
    worst = check_members(res, ys, n, eps_model, amp, 1e-8)
    print(f"S={S} {kw}: max rel diff {worst:.2e}")
    assert worst <= 1e-9


@pytest.mark.parametrize("n,S,kw", [(34, 20, {}), (28, 7, {}), (30, 48, {"member_tile": 32})])
def test_widths_chebyshev_match_oracle(n, S, kw):
    log_case(test="width-cheb", n=n, S=S, **kw)
    ens = E()
    prob = ens.Problem(n, 8, 1, 0.45)
    ys = np.random.default_rng(2000 + S).uniform(-1, 1, (S, 8))
    V, b = ens.assemble(prob, ys)
    R = np.random.default_rng(S + 1).standard_normal((n * n, S))
    z, lmax = ens.cheb_apply(prob, V, torch.tensor(R, device="cuda"),
                             ens.SolverOptions(precond="chebyshev", **kw))
    z = z.cpu().numpy()
    Vh = V.cpu().numpy()
    for s in (0, S - 1):
        A, _, dg = oprob.assemble(ys[s], n, 1, 0.45)
        lm = opcg.gershgorin_lmax(A, dg)
        assert lmax[s] == pytest.approx(lm, rel=1e-14)
        ref = opcg.chebyshev_apply(A, dg, R[:, s], lm)
        assert np.linalg.norm(z[:, s] - ref) <= 1e-13 * np.linalg.norm(ref)
    res = ens.solve(prob, V, b, ens.SolverOptions(precond="chebyshev", rtol=1e-8, **kw))
    worst = check_members(res, ys, n, 1, 0.45, 1e-8, "chebyshev")
    print(f"chebyshev S={S}: max rel diff {worst:.2e}")
    assert worst <= 1e-9


@pytest.mark.parametrize("S,Sp,kw", [(20, 32, {}), (24, 32, {}), (48, 64, {}),
                                     (20, 32, {"precond": "chebyshev"}),
                                     (48, 64, {"member_tile": 32})])
def test_width_equals_padded_power_of_two_bitwise(S, Sp, kw):
    """Same lanes, same reduction trees: the S-member ensemble's results are
    the first S members of the padded ensemble's, bit for bit."""
    log_case(test="width-bitwise", S=S, Sp=Sp, **kw)
    ens = E()
    n = 41
    prob = ens.Problem(n, 4, 0, 0.4)
    ys = np.random.default_rng(3000 + S).uniform(-1, 1, (S, 4))
    pad = np.vstack([ys, np.repeat(ys[-1:], Sp - S, axis=0)])
    V, b = ens.assemble(prob, ys)
    Vp, bp = ens.assemble(prob, pad)
    assert torch.equal(V, Vp[:, :, :S]) and torch.equal(b, bp[:, :S])
    opts = ens.SolverOptions(rtol=1e-8, **kw)
    r = ens.solve(prob, V, b, opts)
    rp = ens.solve(prob, Vp, bp, opts)
    assert np.array_equal(r.iters, rp.iters[:S]) and np.array_equal(r.status, rp.status[:S])
    assert np.array_equal(r.relres, rp.relres[:S])
    assert torch.equal(r.x, rp.x[:, :S])


@pytest.mark.parametrize("S", [3, 9, 21])
def test_odd_width_replicas_bitwise(S):
    """Replicas of a sample (the paper's padding of a last ensemble) inside
    an odd-width ensemble give that sample's results bit for bit."""
    log_case(test="width-replicas", S=S)
    ens = E()
    n = 36
    prob = ens.Problem(n, 4, 0, 0.4)
    ys = np.random.default_rng(4000 + S).uniform(-1, 1, (S, 4))
    ys[S // 2 + 1:] = ys[S // 2]
    V, b = ens.assemble(prob, ys)
    r = ens.solve(prob, V, b)
    x = r.x.cpu().numpy()
    for s in range(S // 2 + 1, S):
        assert np.array_equal(x[:, s], x[:, S // 2]) and r.iters[s] == r.iters[S // 2]


@pytest.mark.parametrize("S", [5, 20])
def test_widths_dqdy_adjoint_indicator(S):
    log_case(test="width-adjoint", S=S)
    ens = E()
    n, d = 44, 6
    prob = ens.Problem(n, d, 0, 0.4)
    ys = np.random.default_rng(5000 + S).uniform(-1, 1, (S, d))
    rng = np.random.default_rng(S)
    U, Lm = rng.standard_normal((n * n, S)), rng.standard_normal((n * n, S))
    g = ens.dqdy(prob, ys, torch.tensor(U, device="cuda"), torch.tensor(Lm, device="cuda"))
    for s in range(S):
        ref = -oadj.dA_bilinear(Lm[:, s], U[:, s], ys[s], n, 0, 0.4)
        np.testing.assert_allclose(g[s], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    V, b = ens.assemble(prob, ys)
    opts = ens.SolverOptions(rtol=1e-12)
    u = ens.solve(prob, V, b, opts).x
    w = ens.qoi_weights(n)
    _, gr, _, status = ens.adjoint_grad(prob, ys, V, u, w, opts)
    assert np.all(status == CONVERGED)
    for s in (0, S - 1):
        _, gref, _, _ = oadj.qoi_and_grad(ys[s], n, 0, 0.4)
        scale = np.maximum(np.abs(gref), 1e-3 * np.abs(gref).max())
        assert np.max(np.abs(gr[s] - gref) / scale) <= 1e-8
    h = ens.param_indicator(prob, ys)
    for s in range(S):
        assert h[s] == pytest.approx(oprob.param_indicator(ys[s], 0), rel=1e-15)


@pytest.mark.parametrize("S", [3, 20])
def test_widths_3d(S):
    log_case(test="width-3d", S=S)
    ens = E()
    m, d = 9, 4
    prob = ens.Problem(m, d, dim=3)
    ys = np.random.default_rng(6000 + S).uniform(-1, 1, (S, d))
    V, b = ens.assemble(prob, ys)
    Vh = V.cpu().numpy()
    res = ens.solve(prob, V, b, ens.SolverOptions(rtol=1e-7))
    x = res.x.cpu().numpy()
    for s in (0, S - 1):
        A, bo, dg = ofe.assemble(ys[s], m)
        ref = ofe.slot_values(A, m)
        assert np.max(np.abs(Vh[:, :, s] - ref)) <= 1e-14 * np.abs(ref).max()
        _, I, st, _ = opcg.pcg(A, bo, dg, 1e-7, 20000)
        assert st == CONVERGED and abs(int(res.iters[s]) - I) <= 1
        xe, _, _, _ = opcg.pcg(A, bo, dg, 0.0, int(res.iters[s]))
        assert np.linalg.norm(x[:, s] - xe) <= 1e-9 * np.linalg.norm(xe)
    rng = np.random.default_rng(S)
    U, Lm = rng.standard_normal((m ** 3, S)), rng.standard_normal((m ** 3, S))
    g = ens.dqdy(prob, ys, torch.tensor(U, device="cuda"), torch.tensor(Lm, device="cuda"))
    for s in (0, S - 1):
        ref = -ofe.dA_bilinear(Lm[:, s], U[:, s], ys[s], m)
        np.testing.assert_allclose(g[s], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    h = ens.param_indicator(prob, ys)
    for s in range(S):
        assert h[s] == pytest.approx(ofe.param_indicator(ys[s], m), rel=1e-13)


@pytest.mark.parametrize("dim,n", [(2, 64), (2, 511), (2, 3), (3, 31), (3, 8)])
def test_qoi_weights_match_oracle_bitwise(dim, n):
    ens = E()
    w = ens.qoi_weights(n, dim=dim).cpu().numpy()
    ref = oprob.qoi_weights(n) if dim == 2 else ofe.qoi_weights(n)
    assert np.array_equal(w, ref)
