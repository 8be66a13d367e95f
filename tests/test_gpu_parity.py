"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances (derivations in the design notes):
  * assembly: every entry within 4 ulp-scale relative error (the only
    difference is the last bit of sin / cos / pow);
  * SpMV and Chebyshev application: 1e-13 relative (summation order);
  * PCG: iteration counts within +-1 of the oracle; at equal iteration count
    (the oracle re-run for exactly the GPU's count) ||x_gpu - x_orc|| /
    ||x_orc|| <= 1e-9 and max|x_gpu - x_orc| / max|x_orc| <= 1e-9; true
    residual ||b - A x|| <= 2 rtol ||b||;
  * reductions are deterministic: permuting members permutes results bit for
    bit, a padded replica equals its original bit for bit.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import BREAKDOWN, CONVERGED, MAX_ITER, ZERO_RHS
from oracle import adjoint as oadj
from oracle import pcg as opcg
from oracle import problem as oprob

pytestmark = pytest.mark.gpu

DEV = "cuda"


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
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def gpu_stencil(prob, ys):
    ens = E()
    V, b = ens.assemble(prob, to_dev(ys))
    return V, b


def log_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


@pytest.mark.parametrize("n,d,eps_model,amp,S,seed", [
    (64, 2, 0, 0.0, 8, 0), (37, 4, 0, 0.4, 16, 1), (33, 8, 1, 0.45, 64, 2),
    (20, 6, 0, 0.4, 1, 3), (50, 4, 0, 0.4, 2, 4)])
def test_assembly_matches_oracle(n, d, eps_model, amp, S, seed):
    log_case(test="assembly", n=n, d=d, S=S)
    ens = E()
    prob = ens.Problem(n, d, eps_model, amp)
    ys = np.random.default_rng(seed).uniform(-1, 1, (S, d))
    V, b = gpu_stencil(prob, ys)
    Vh = V.cpu().numpy()
    assert np.all(b.cpu().numpy() == 1.0)
    worst = 0.0
    for s in range(S):
        ref = oprob.stencil_values(ys[s], n, eps_model, amp)
        got = Vh[:, :, s]
        assert np.array_equal(got == 0.0, ref == 0.0)
        scale = np.abs(ref[4])[None, :]
        err = np.abs(got - ref) / scale
        worst = max(worst, float(err.max()))
    print("assembly max rel err", worst)
    assert worst <= 4e-15


@pytest.mark.parametrize("n,S", [(64, 8), (45, 32), (31, 1), (19, 64), (70, 4)])
def test_spmv_matches_oracle(n, S):
    log_case(test="spmv", n=n, S=S)
    ens = E()
    prob = ens.Problem(n, 4, 0, 0.4)
    rng = np.random.default_rng(n * 100 + S)
    ys = rng.uniform(-1, 1, (S, 4))
    V, _ = gpu_stencil(prob, ys)
    P = rng.standard_normal((n * n, S))
    q = ens.spmv(prob, V, to_dev(P)).cpu().numpy()
    Vh = V.cpu().numpy()
    for s in range(S):
        A = oprob.to_csr(oprob.stencil_values(ys[s], n, 0, 0.4), n)
        ref = A @ P[:, s]
        assert np.max(np.abs(q[:, s] - ref)) <= 1e-13 * np.max(np.abs(A).sum(axis=1)) * np.abs(P[:, s]).max()


def oracle_system(y, n, eps_model, amp):
    A, b, diag = oprob.assemble(np.asarray(y), n, eps_model, amp)
    return A, b, diag


def check_solution(res, ys, n, eps_model, amp, rtol, precond="jacobi", real=None):
    x = res.x.cpu().numpy()
    S = x.shape[1]
    worst = 0.0
    for s in range(S if real is None else real):
        A, b, diag = oracle_system(ys[s], n, eps_model, amp)
        xo, Io, so, _ = opcg.pcg(A, b, diag, rtol, 20000, precond)
        assert so == CONVERGED and res.status[s] == CONVERGED
        assert abs(int(res.iters[s]) - Io) <= 1, (s, res.iters[s], Io)
        # same iteration count: rerun the oracle for exactly the GPU's count
        xe, Ie, _, _ = opcg.pcg(A, b, diag, 0.0, int(res.iters[s]), precond)
        rel = np.linalg.norm(x[:, s] - xe) / np.linalg.norm(xe)
        # element-wise, against the largest entry
        rel_e = np.abs(x[:, s] - xe).max() / np.abs(xe).max()
        worst = max(worst, rel, rel_e)
        assert np.linalg.norm(b - A @ x[:, s]) <= 2 * rtol * np.linalg.norm(b)
    return worst


def test_small_workload_solves_match_oracle():
    """64 x 64, d = 2, 32 samples (seed 0) in ensembles of 8, Jacobi, rtol 1e-8."""
    ens = E()
    w = workloads.SMALL
    prob = ens.Problem(w.n, w.d, w.eps_model, w.amp)
    ys_all = workloads.uniform_samples(w.seed, w.n_samples, w.d)
    opts = ens.SolverOptions(rtol=w.rtol, max_iter=w.max_iter)
    worst = 0.0
    for g in range(0, 32, 8):
        log_case(test="small", group=g)
        ys = ys_all[g:g + 8]
        V, b = gpu_stencil(prob, ys)
        res = ens.solve(prob, V, b, opts)
        assert res.ens_iters == int(res.iters.max())
        worst = max(worst, check_solution(res, ys, w.n, w.eps_model, w.amp, w.rtol))
    print("small workload: max rel diff at equal iteration count", worst)
    assert worst <= 1e-9


@pytest.mark.parametrize("n,S,d,eps_model,amp,seed", [
    (45, 16, 4, 0, 0.4, 5), (33, 32, 8, 1, 0.45, 6), (30, 1, 4, 0, 0.4, 7), (27, 64, 6, 0, 0.4, 8),
    (40, 2, 4, 0, 0.4, 9)])
def test_ragged_sizes_match_oracle(n, S, d, eps_model, amp, seed):
    log_case(test="ragged", n=n, S=S)
    ens = E()
    prob = ens.Problem(n, d, eps_model, amp)
    ys = np.random.default_rng(seed).uniform(-1, 1, (S, d))
    V, b = gpu_stencil(prob, ys)
    res = ens.solve(prob, V, b, ens.SolverOptions(rtol=1e-8))
    worst = check_solution(res, ys, n, eps_model, amp, 1e-8)
    print("ragged", n, S, "max rel diff", worst)
    assert worst <= 1e-9


def test_tile_shapes_agree():
    """Different tile heights / workgroup counts give the same counts and
    solutions to rounding (only the order of partial sums changes)."""
    ens = E()
    n, S = 64, 16
    prob = ens.Problem(n, 4, 0, 0.4)
    ys = np.random.default_rng(11).uniform(-1, 1, (S, 4))
    V, b = gpu_stencil(prob, ys)
    base = ens.solve(prob, V, b, ens.SolverOptions())
    for tl, mg in [(1, 8), (3, 40), (64, 0), (5, 2048)]:
        log_case(test="tiles", tile_lines=tl, max_groups=mg)
        r = ens.solve(prob, V, b, ens.SolverOptions(tile_lines=tl, max_groups=mg))
        assert np.all(np.abs(r.iters - base.iters) <= 1)
        rel = (torch.linalg.norm(r.x - base.x, dim=0) / torch.linalg.norm(base.x, dim=0)).max().item()
        assert rel <= 1e-8


@pytest.mark.parametrize("dim,n,S", [(2, 256, 32), (2, 48, 4), (3, 17, 32)])
def test_poll_interval_does_not_change_the_solve(dim, n, S):
    """The host's poll interval only decides how many early-exit launches
    follow convergence: iterations, status and x are the same bits for the
    adaptive interval (the first two cases span both of its regimes) and for
    fixed ones."""
    ens = E()
    d = 4
    prob = ens.Problem(n, d, 0, 0.4 if dim == 2 else 0.0, dim=dim)
    ys = np.random.default_rng(n + S).uniform(-1, 1, (S, d))
    V, b = gpu_stencil(prob, ys)
    rtol = 1e-8 if dim == 2 else 1e-7
    base = ens.solve(prob, V, b, ens.SolverOptions(rtol=rtol))
    assert np.all(base.status == CONVERGED)
    for poll in (1, 3, 16, 64):
        log_case(test="poll", dim=dim, n=n, S=S, poll=poll)
        r = ens.solve(prob, V, b, ens.SolverOptions(rtol=rtol, poll_every=poll))
        assert np.array_equal(r.iters, base.iters) and np.array_equal(r.status, base.status)
        assert r.ens_iters == base.ens_iters
        assert torch.equal(r.x, base.x)


def test_permutation_and_padding_bitwise():
    ens = E()
    n, S = 48, 16
    prob = ens.Problem(n, 4, 0, 0.4)
    rng = np.random.default_rng(12)
    ys = rng.uniform(-1, 1, (S, 4))
    ys[12:] = ys[11]                       # padding replicas of sample 11
    V, b = gpu_stencil(prob, ys)
    r0 = ens.solve(prob, V, b)
    x0 = r0.x.cpu().numpy()
    for s in range(12, S):
        assert np.array_equal(x0[:, s], x0[:, 11]) and r0.iters[s] == r0.iters[11]
    perm = rng.permutation(S)
    V2, b2 = gpu_stencil(prob, ys[perm])
    r1 = ens.solve(prob, V2, b2)
    assert np.array_equal(r1.x.cpu().numpy(), x0[:, perm])
    assert np.array_equal(r1.iters, r0.iters[perm])
    # run twice: bitwise identical
    r2 = ens.solve(prob, V, b)
    assert np.array_equal(r2.x.cpu().numpy(), x0)


def test_member_width_independence():
    """A sample solved alone (S = 1) and inside an ensemble (S = 32) agree."""
    ens = E()
    n = 40
    prob = ens.Problem(n, 4, 0, 0.4)
    ys = np.random.default_rng(13).uniform(-1, 1, (32, 4))
    V, b = gpu_stencil(prob, ys)
    rS = ens.solve(prob, V, b)
    for s in (0, 17, 31):
        V1, b1 = gpu_stencil(prob, ys[s:s + 1])
        r1 = ens.solve(prob, V1, b1)
        assert abs(int(r1.iters[0]) - int(rS.iters[s])) <= 1
        if r1.iters[0] == rS.iters[s]:
            a, c = r1.x[:, 0], rS.x[:, s]
            assert (torch.linalg.norm(a - c) / torch.linalg.norm(c)).item() <= 1e-9


def test_status_codes():
    ens = E()
    n, S = 24, 4
    prob = ens.Problem(n, 4, 0, 0.4)
    ys = np.random.default_rng(14).uniform(-1, 1, (S, 4))
    V, b = gpu_stencil(prob, ys)
    b[:, 2] = 0.0                                            # zero right-hand side
    res = ens.solve(prob, V, b)
    assert res.status[2] == ZERO_RHS and res.iters[2] == 0
    assert torch.count_nonzero(res.x[:, 2]).item() == 0
    assert all(res.status[s] == CONVERGED for s in (0, 1, 3))
    res1 = ens.solve(prob, V, b, ens.SolverOptions(max_iter=1))
    assert [int(v) for v in res1.status] == [MAX_ITER, MAX_ITER, ZERO_RHS, MAX_ITER]
    assert [int(v) for v in res1.iters] == [1, 1, 0, 1]
    # an indefinite member (negated matrix) breaks down at its first step and
    # stays finite while the others converge normally (the paper's guard)
    V[:, :, 1] = -V[:, :, 1]
    res2 = ens.solve(prob, V, b)
    assert res2.status[1] == BREAKDOWN and res2.iters[1] == 1
    assert torch.isfinite(res2.x).all()
    assert res2.status[0] == CONVERGED and res2.iters[0] == res.iters[0]
    assert torch.equal(res2.x[:, 0], res.x[:, 0])


def test_chebyshev_apply_matches_oracle():
    ens = E()
    n, S = 36, 8
    prob = ens.Problem(n, 8, 1, 0.45)
    rng = np.random.default_rng(15)
    ys = rng.uniform(-1, 1, (S, 8))
    V, _ = gpu_stencil(prob, ys)
    R = rng.standard_normal((n * n, S))
    z, lmax = ens.cheb_apply(prob, V, to_dev(R))
    z = z.cpu().numpy()
    Vh = V.cpu().numpy()
    for s in range(S):
        A, _, diag = oprob.assemble(ys[s], n, 1, 0.45)
        lm = opcg.gershgorin_lmax(A, diag)
        assert lmax[s] == pytest.approx(lm, rel=1e-14)
        ref = opcg.chebyshev_apply(A, diag, R[:, s], lm)
        assert np.linalg.norm(z[:, s] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_chebyshev_pcg_matches_oracle():
    ens = E()
    n, S = 48, 16
    prob = ens.Problem(n, 8, 1, 0.45)
    ys = np.random.default_rng(16).uniform(-1, 1, (S, 8))
    V, b = gpu_stencil(prob, ys)
    res = ens.solve(prob, V, b, ens.SolverOptions(precond="chebyshev"))
    worst = check_solution(res, ys, n, 1, 0.45, 1e-8, precond="chebyshev")
    print("chebyshev max rel diff", worst)
    assert worst <= 1e-9


@pytest.mark.parametrize("degree,S,kw", [
    (2, 8, {}), (3, 20, {}), (5, 64, {"member_tile": 16}), (6, 1, {}), (8, 5, {"tile_lines": 3}),
])
def test_chebyshev_degrees_match_oracle(degree, S, kw):
    """Every polynomial degree the solver takes (2..8): the application
    within 1e-13 of the oracle, and Chebyshev-PCG counts within +-1 and
    equal-count solutions within 1e-9.  The oracle keeps the three-term
    recurrence with a stored increment; the 2-D steps form the increment
    from the iterates and, from the third step on, overwrite z_{k-2} with z_k
    in place, so degrees above 4 run that alternation several times."""
    ens = E()
    n = 41
    prob = ens.Problem(n, 8, 1, 0.45)
    ys = np.random.default_rng(100 + degree).uniform(-1, 1, (S, 8))
    V, b = gpu_stencil(prob, ys)
    log_case(test="cheb_degree", degree=degree, S=S, **kw)
    opts = ens.SolverOptions(precond="chebyshev", cheb_degree=degree, **kw)
    R = np.random.default_rng(7).standard_normal((n * n, S))
    z, lmax = ens.cheb_apply(prob, V, to_dev(R), opts)
    z = z.cpu().numpy()
    res = ens.solve(prob, V, b, opts)
    xg = res.x.cpu().numpy()
    for s in sorted({0, S // 2, S - 1}):
        A, bo, dg = oracle_system(ys[s], n, 1, 0.45)
        lm = opcg.gershgorin_lmax(A, dg)
        assert lmax[s] == pytest.approx(lm, rel=1e-14)
        ref = opcg.chebyshev_apply(A, dg, R[:, s], lm, degree=degree)
        assert np.linalg.norm(z[:, s] - ref) <= 1e-13 * np.linalg.norm(ref)

        def M(v, A=A, dg=dg, lm=lm):
            return opcg.chebyshev_apply(A, dg, v, lm, degree=degree)

        xo, Io, so, _ = opcg.pcg(A, bo, dg, 1e-8, 20000, M)
        assert so == CONVERGED and res.status[s] == CONVERGED
        assert abs(int(res.iters[s]) - Io) <= 1, (s, res.iters[s], Io)
        xe, _, _, _ = opcg.pcg(A, bo, dg, 0.0, int(res.iters[s]), M)
        assert np.linalg.norm(xg[:, s] - xe) <= 1e-9 * np.linalg.norm(xe)
        assert np.abs(xg[:, s] - xe).max() <= 1e-9 * np.abs(xe).max()


def test_member_dot():
    ens = E()
    rng = np.random.default_rng(17)
    for Nr, S in [(1000, 8), (4097, 32), (77, 1), (300, 64)]:
        a, c = rng.standard_normal((Nr, S)), rng.standard_normal((Nr, S))
        w = rng.standard_normal(Nr)
        got = ens.member_dot(to_dev(a), to_dev(c))
        np.testing.assert_allclose(got, np.einsum("rs,rs->s", a, c), rtol=1e-12, atol=1e-12)
        got = ens.member_dot(to_dev(a), to_dev(w))
        np.testing.assert_allclose(got, w @ a, rtol=1e-12, atol=1e-12)


def test_dqdy_kernel_matches_oracle_form():
    """Given identical u and lambda, the kernel's -lambda^T (dA/dy) u equals the
    oracle's face/node form to rounding."""
    ens = E()
    n, S, d = 40, 8, 6
    prob = ens.Problem(n, d, 0, 0.4)
    rng = np.random.default_rng(18)
    ys = rng.uniform(-1, 1, (S, d))
    U, Lm = rng.standard_normal((n * n, S)), rng.standard_normal((n * n, S))
    g = ens.dqdy(prob, to_dev(ys), to_dev(U), to_dev(Lm))
    for s in range(S):
        ref = -oadj.dA_bilinear(Lm[:, s], U[:, s], ys[s], n, 0, 0.4)
        np.testing.assert_allclose(g[s], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_adjoint_gradient_matches_oracle():
    ens = E()
    n, S, d = 48, 8, 6
    prob = ens.Problem(n, d, 0, 0.4)
    ys = np.random.default_rng(19).uniform(-1, 1, (S, d))
    y = to_dev(ys)
    V, b = ens.assemble(prob, y)
    opts = ens.SolverOptions(rtol=1e-12)
    u = ens.solve(prob, V, b, opts).x
    w = ens.qoi_weights(n)
    lam, g, iters, status = ens.adjoint_grad(prob, y, V, u, w, opts)
    assert all(status == CONVERGED)
    for s in range(S):
        Q, gref, _, _ = oadj.qoi_and_grad(ys[s], n, 0, 0.4)
        scale = np.maximum(np.abs(gref), 1e-2 * np.abs(gref).max())
        assert np.max(np.abs(g[s] - gref) / scale) <= 1e-8


@pytest.mark.parametrize("S,tiles", [(64, (32, 16, 8)), (32, (16, 2)), (8, (4, 2))])
def test_member_tiles_agree(S, tiles):
    """Sweeping a wide ensemble in member tiles changes only which threads
    hold which members: counts agree, solutions agree to rounding, and each
    member's reduction tree stays member-independent (bitwise permutation)."""
    ens = E()
    n = 56
    prob = ens.Problem(n, 4, 0, 0.4)
    ys = np.random.default_rng(S).uniform(-1, 1, (S, 4))
    V, b = gpu_stencil(prob, ys)
    base = ens.solve(prob, V, b)
    for sw in tiles:
        log_case(test="member_tiles", S=S, member_tile=sw)
        r = ens.solve(prob, V, b, ens.SolverOptions(member_tile=sw))
        assert np.all(np.abs(r.iters - base.iters) <= 1)
        rel = (torch.linalg.norm(r.x - base.x, dim=0) / torch.linalg.norm(base.x, dim=0)).cpu().numpy()
        assert np.all(rel[r.iters == base.iters] <= 1e-9)
        perm = np.random.default_rng(sw).permutation(S)
        V2, b2 = gpu_stencil(prob, ys[perm])
        r2 = ens.solve(prob, V2, b2, ens.SolverOptions(member_tile=sw))
        assert torch.equal(r2.x, r.x[:, perm]) and np.array_equal(r2.iters, r.iters[perm])


@pytest.mark.parametrize("n,S,kw", [
    (64, 32, {}),
    (45, 8, {"tile_lines": 1}),
    (37, 1, {"tile_lines": 3, "max_groups": 40}),
    (70, 64, {"member_tile": 16}),
    (19, 2, {"tile_lines": 5, "max_groups": 2048}),
    (33, 16, {"precond": "chebyshev"}),
    (29, 4, {"precond": "chebyshev", "cheb_degree": 3, "tile_lines": 2}),
])
def test_symmetric_sweep_bitwise(n, S, kw):
    """The default sweep reads five matrix values per row and takes the other
    four from the neighbouring rows; on the bitwise-symmetric assembled
    matrix it must reproduce the nine-value sweep bit for bit, including the
    tile edges (one-point halos, first line of a band, last partial chunk)."""
    ens = E()
    d = 8 if kw.get("precond") == "chebyshev" else 4
    prob = ens.Problem(n, d, 1 if d == 8 else 0, 0.45 if d == 8 else 0.4)
    ys = np.random.default_rng(n * 7 + S).uniform(-1, 1, (S, d))
    V, b = gpu_stencil(prob, ys)
    log_case(test="symmetric", n=n, S=S, **kw)
    Vh = V.cpu().numpy()
    # the assembled storage is bitwise symmetric: W(i,j) = E(i-1,j), ...
    V4 = Vh.reshape(9, n, n, S)                      # [slot][j][i][s]
    assert np.array_equal(V4[3][:, 1:], V4[5][:, :-1])
    assert np.array_equal(V4[1][1:], V4[7][:-1])
    assert np.array_equal(V4[0][1:, 1:], V4[8][:-1, :-1])
    assert np.array_equal(V4[2][1:, :-1], V4[6][:-1, 1:])
    sym = ens.solve(prob, V, b, ens.SolverOptions(**kw))
    full = ens.solve(prob, V, b, ens.SolverOptions(full_stencil=True, **kw))
    assert np.array_equal(sym.iters, full.iters)
    assert np.array_equal(sym.status, full.status)
    assert torch.equal(sym.x, full.x)
    if kw.get("precond") == "chebyshev":
        R = to_dev(np.random.default_rng(5).standard_normal((n * n, S)))
        kc = {k: v for k, v in kw.items() if k != "precond"}
        z1, l1 = ens.cheb_apply(prob, V, R, ens.SolverOptions(precond="chebyshev", **kc))
        z2, l2 = ens.cheb_apply(prob, V, R, ens.SolverOptions(precond="chebyshev",
                                                             full_stencil=True, **kc))
        assert torch.equal(z1, z2) and np.array_equal(l1, l2)


@pytest.mark.parametrize("n", [1, 2, 7, 4096, 1000003])
def test_stream_triad(n):
    """c = a + s b exactly (s a power of two makes s b exact, so the fused
    multiply-add rounds like the separate expression)."""
    ens = E()
    g = torch.Generator(device="cpu").manual_seed(n)
    a = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    b = torch.randn(n, generator=g, dtype=torch.float64).cuda()
    c = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    for s in (0.5, -2.0):
        ens.stream_triad(a, b, c, s)
        torch.cuda.synchronize()
        assert torch.equal(c, a + s * b)


def test_stream_triad_rejects_bad_arguments():
    from paper_1705_02003_amd import _lib as L
    ens = E()
    a = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(L.EnsError):
        ens.stream_triad(a[1:], a[1:], a[1:], 1.0)        # 8-byte aligned only
    with pytest.raises(L.EnsError):
        ens.stream_triad(a, a, a, float("inf"))


@pytest.mark.parametrize("nread,nwrite,n", [(8, 3, 4098), (2, 1, 2), (3, 1, 1000), (1, 1, 64)])
def test_stream_mix(nread, nwrite, n):
    """dst_w = src_0 + src_1 + ... (summed in that order) for every output
    stream; strides a few KiB past n."""
    ens = E()
    stride = ((n + 31) // 32) * 32 + 512
    g = torch.Generator(device="cpu").manual_seed(n + nread)
    src = torch.randn(nread * stride, generator=g, dtype=torch.float64).cuda()
    dst = torch.full((nwrite * stride,), float("nan"), dtype=torch.float64, device="cuda")
    ens.stream_mix(src, dst, stride, n, nread, nwrite)
    torch.cuda.synchronize()
    ref = torch.zeros(n, dtype=torch.float64, device="cuda")
    for k in range(nread):
        ref = ref + src[k * stride:k * stride + n]
    for w in range(nwrite):
        assert torch.equal(dst[w * stride:w * stride + n], ref)
        assert torch.isnan(dst[w * stride + n:(w + 1) * stride]).all() if w + 1 < nwrite else True
