"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (512 workgroups, 32-line tiles, the
symmetric read), on outputs the oracle can compute one by one:

  * 512^2, d = 4, S = 32 (the benchmark's adaptive workload; inputs are the
    workload's first sparse-grid nodes): assembly at every row of sampled
    members, the product at sampled members, the solve of two members
    against full oracle solves (counts +-1, the solution within 1e-9 at
    equal count for one of them), the true residual of every member;
  * 1024^2, d = 8, S = 32 and 64, Chebyshev-4 (the Chebyshev workload,
    uniform samples of its seed): the preconditioner application of sampled members
    and the true residual of sampled members of the solve;
  * 512^2, d = 6, S = 32 (the adjoint workload): the dQ/dy kernel against
    the oracle's form for sampled members, given the GPU's u and lambda;
  * 31^3, d = 4, S = 32 (the 3-D workload): solves of two members against
    full oracle solves; the dQ/dy kernel and the grouping indicator of
    sampled members;
  * 512^2, d = 4, S = 64 (the widest ensemble of the speed-up curve): the
    product and the solve's true residual at sampled members;
  * the batched workload's first six ensembles (grids 256^2, 512^2 and
    1024^2, widths 4, 8 and 64, d = 8) in one batched solve with the
    autotuner's launch shapes: every ensemble against its single-ensemble
    solve, sampled members' true residuals and one member's oracle solve.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import CONVERGED
from oracle import adjoint as oadj
from oracle import fe3d as ofe
from oracle import multigrid as omg
from oracle import pcg as opcg
from oracle import problem as oprob
from oracle import sparse_grid as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on an MI355X")
    yield


def E():
    from paper_1705_02003_amd import ensemble
    return ensemble


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def log_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def adaptive_first_nodes(d, count):
    """The benchmark workload's first samples: the level-1 grid, then the
    level-2 nodes, in generation (canonical) order."""
    nodes = sg.full_grid(d, 1) + [nd for nd in sg.full_grid(d, 2) if sg.total_level(nd) == 2]
    return np.array([sg.coords(nd) for nd in nodes[:count]])


def test_benchmark_size_512_s32():
    ens = E()
    n, d, S, amp = 512, 4, 32, 0.4
    log_case(test="fullsize-512", n=n, S=S)
    ys = adaptive_first_nodes(d, S)
    prob = ens.Problem(n, d, 0, amp)
    V, b = ens.assemble(prob, to_dev(ys))
    Vh = V.cpu().numpy()
    # assembly: every row of three members
    for s in (0, 13, 31):
        ref = oprob.stencil_values(ys[s], n, 0, amp)
        err = np.abs(Vh[:, :, s] - ref).max(axis=0)
        assert np.all(err <= 4e-15 * np.abs(ref[oprob.CENTER]))
    # the product at three members
    rng = np.random.default_rng(7)
    P = rng.standard_normal((n * n, S))
    q = ens.spmv(prob, V, to_dev(P)).cpu().numpy()
    for s in (2, 17, 30):
        A = oprob.to_csr(oprob.stencil_values(ys[s], n, 0, amp), n)
        ref = A @ P[:, s]
        assert np.max(np.abs(q[:, s] - ref)) <= 1e-13 * np.abs(A).sum(axis=1).max() * np.abs(P[:, s]).max()
    # the solve, benchmark options
    res = ens.solve(prob, V, b, ens.SolverOptions(rtol=1e-8, max_iter=20000))
    assert np.all(res.status == CONVERGED)
    x = res.x.cpu().numpy()
    for s in range(S):
        A, bo, _ = oprob.assemble(ys[s], n, 0, amp)
        assert np.linalg.norm(bo - A @ x[:, s]) <= 2e-8 * np.linalg.norm(bo)
    for s, equal in ((0, True), (9, False)):
        A, bo, dg = oprob.assemble(ys[s], n, 0, amp)
        _, I, st, _ = opcg.pcg(A, bo, dg, 1e-8, 20000)
        assert st == CONVERGED and abs(int(res.iters[s]) - I) <= 1, (s, res.iters[s], I)
        if equal:
            xe, _, _, _ = opcg.pcg(A, bo, dg, 0.0, int(res.iters[s]))
            assert np.linalg.norm(x[:, s] - xe) <= 1e-9 * np.linalg.norm(xe)


@pytest.mark.parametrize("S", [32, 64])
def test_chebyshev_size_1024(S):
    ens = E()
    w = workloads.CHEB_1024
    n = w.n
    log_case(test="fullsize-1024-cheb", n=n, S=S)
    ys = workloads.uniform_samples(w.seed, S, w.d)
    prob = ens.Problem(n, w.d, w.eps_model, w.amp)
    V, b = ens.assemble(prob, to_dev(ys))
    rng = np.random.default_rng(8)
    R = rng.standard_normal((n * n, S))
    z, lmax = ens.cheb_apply(prob, V, to_dev(R))
    z = z.cpu().numpy()
    for s in (5, S - 6):
        A, _, dg = oprob.assemble(ys[s], n, w.eps_model, w.amp)
        lm = opcg.gershgorin_lmax(A, dg)
        assert lmax[s] == pytest.approx(lm, rel=1e-14)
        ref = opcg.chebyshev_apply(A, dg, R[:, s], lm)
        assert np.linalg.norm(z[:, s] - ref) <= 1e-13 * np.linalg.norm(ref)
    res = ens.solve(prob, V, b, ens.SolverOptions(precond="chebyshev", rtol=w.rtol,
                                                  max_iter=w.max_iter))
    assert np.all(res.status == CONVERGED)
    x = res.x.cpu().numpy()
    for s in (0, 11, S - 1):
        A, bo, _ = oprob.assemble(ys[s], n, w.eps_model, w.amp)
        assert np.linalg.norm(bo - A @ x[:, s]) <= 2 * w.rtol * np.linalg.norm(bo)


def test_adjoint_size_512_s32():
    ens = E()
    w = workloads.ADJOINT_512
    n, S = w.n, 32
    log_case(test="fullsize-512-dqdy", n=n, S=S)
    ys = workloads.uniform_samples(w.seed, S, w.d)
    prob = ens.Problem(n, w.d, w.eps_model, w.amp)
    rng = np.random.default_rng(9)
    U, Lm = rng.standard_normal((n * n, S)), rng.standard_normal((n * n, S))
    g = ens.dqdy(prob, to_dev(ys), to_dev(U), to_dev(Lm))
    for s in (3, 28):
        ref = -oadj.dA_bilinear(Lm[:, s], U[:, s], ys[s], n, w.eps_model, w.amp)
        np.testing.assert_allclose(g[s], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_fe3d_size_31cube_s32():
    ens = E()
    w = workloads.FE3D_32
    m, S = w.n, 32
    log_case(test="fullsize-fe3d", m=m, S=S)
    ys = workloads.uniform_samples(w.seed, S, w.d)
    prob = ens.Problem(m, w.d, dim=3)
    V, b = ens.assemble(prob, to_dev(ys))
    res = ens.solve(prob, V, b, ens.SolverOptions(rtol=w.rtol, max_iter=w.max_iter))
    assert np.all(res.status == CONVERGED)
    x = res.x.cpu().numpy()
    for s in (4, 21):
        A, bo, dg = ofe.assemble(ys[s], m)
        _, I, st, _ = opcg.pcg(A, bo, dg, w.rtol, 20000)
        assert st == CONVERGED and abs(int(res.iters[s]) - I) <= 1
        xe, _, _, _ = opcg.pcg(A, bo, dg, 0.0, int(res.iters[s]))
        assert np.linalg.norm(x[:, s] - xe) <= 1e-9 * np.linalg.norm(xe)
        assert np.linalg.norm(bo - A @ x[:, s]) <= 2 * w.rtol * np.linalg.norm(bo)


@pytest.mark.parametrize("precond", ["chebyshev", "multigrid"])
def test_fe3d_size_31cube_s32_polynomial_and_multigrid(precond):
    """The 3-D workload's own size and width (31^3, S = 32), where the
    product kernel takes pairs of points per thread (smaller grids and
    narrower ensembles take single points): Chebyshev-4 and multigrid PCG
    against the oracle for two members (counts +-1, equal-count solutions
    1e-9, true residual), and for multigrid the fused coarse tail against
    the level-by-level launches bit for bit."""
    ens = E()
    w = workloads.FE3D_32
    m, S = w.n, 32
    log_case(test="fullsize-fe3d-" + precond, m=m, S=S)
    ys = workloads.uniform_samples(w.seed, S, w.d)
    prob = ens.Problem(m, w.d, dim=3)
    V, b = ens.assemble(prob, to_dev(ys))
    res = ens.solve(prob, V, b, ens.SolverOptions(precond=precond, rtol=w.rtol, max_iter=w.max_iter))
    assert np.all(res.status == CONVERGED)
    x = res.x.cpu().numpy()
    for s in (3, 30):
        A, bo, dg = ofe.assemble(ys[s], m)
        if precond == "multigrid":
            _, I, st, _ = omg.pcg(A, bo, m, w.rtol, 2000)
            xe, _, _, _ = omg.pcg(A, bo, m, 0.0, int(res.iters[s]))
        else:
            lm = opcg.gershgorin_lmax(A, dg)

            def M(v, A=A, dg=dg, lm=lm):
                return opcg.chebyshev_apply(A, dg, v, lm)

            _, I, st, _ = opcg.pcg(A, bo, dg, w.rtol, 20000, M)
            xe, _, _, _ = opcg.pcg(A, bo, dg, 0.0, int(res.iters[s]), M)
        assert st == CONVERGED and abs(int(res.iters[s]) - I) <= 1, (s, res.iters[s], I)
        assert np.linalg.norm(x[:, s] - xe) <= 1e-9 * np.linalg.norm(xe)
        assert np.linalg.norm(bo - A @ x[:, s]) <= 2 * w.rtol * np.linalg.norm(bo)
    if precond == "multigrid":
        lw = ens.solve(prob, V, b, ens.SolverOptions(precond=precond, rtol=w.rtol, max_iter=w.max_iter,
                                                     mg_levelwise=True))
        assert np.array_equal(lw.iters, res.iters) and torch.equal(lw.x, res.x)


def test_batch_full_grid_sizes():
    ens = E()
    from paper_1705_02003_amd import autotune
    w = workloads.BATCHED
    draw = workloads.batched_draw(w.seed)
    k = 6
    log_case(test="fullsize-batch", shapes=list(zip(draw.grids[:k], draw.widths[:k])))
    items = []
    for S, n, y in zip(draw.widths[:k], draw.grids[:k], draw.samples[:k]):
        prob = ens.Problem(n, w.d, w.eps_model, w.amp)
        V, b = ens.assemble(prob, to_dev(y))
        sh = autotune.tune(n, S, cache=None)
        items.append({"prob": prob, "V": V, "b": b, "tile_lines": sh["tile_lines"],
                      "member_tile": sh["member_tile"]})
    opts = ens.SolverOptions(rtol=w.rtol, max_iter=w.max_iter)
    res = ens.batch_solve(items, opts)
    for e, (it, r, y) in enumerate(zip(items, res, draw.samples[:k])):
        assert np.all(r.status == CONVERGED), e
        single = ens.solve(it["prob"], it["V"], it["b"], opts)
        assert np.all(np.abs(r.iters - single.iters) <= 1), e
        same = r.iters == single.iters
        num = torch.linalg.norm(r.x - single.x, dim=0).cpu().numpy()
        den = torch.linalg.norm(single.x, dim=0).cpu().numpy()
        assert np.all((num / den)[same] <= 1e-9), e
        x = r.x.cpu().numpy()
        n = it["prob"].n
        for s in (0, x.shape[1] - 1):
            A, bo, _ = oprob.assemble(y[s], n, w.eps_model, w.amp)
            assert np.linalg.norm(bo - A @ x[:, s]) <= 2 * w.rtol * np.linalg.norm(bo), (e, s)
    # one member of the 256^2 ensemble against the oracle's own solve
    e = draw.grids[:k].index(256)
    y = draw.samples[e][0]
    A, bo, dg = oprob.assemble(y, 256, w.eps_model, w.amp)
    _, I, st, _ = opcg.pcg(A, bo, dg, w.rtol, w.max_iter)
    assert st == CONVERGED and abs(int(res[e].iters[0]) - I) <= 1
    xe, _, _, _ = opcg.pcg(A, bo, dg, 0.0, int(res[e].iters[0]))
    x0 = res[e].x[:, 0].cpu().numpy()
    assert np.linalg.norm(x0 - xe) <= 1e-9 * np.linalg.norm(xe)


def test_fe3d_dqdy_and_indicator_31cube_s32():
    ens = E()
    w = workloads.FE3D_32
    m, S = w.n, 32
    log_case(test="fullsize-fe3d-dqdy", m=m, S=S)
    ys = workloads.uniform_samples(w.seed, S, w.d)
    prob = ens.Problem(m, w.d, dim=3)
    rng = np.random.default_rng(12)
    U, Lm = rng.standard_normal((m ** 3, S)), rng.standard_normal((m ** 3, S))
    g = ens.dqdy(prob, to_dev(ys), to_dev(U), to_dev(Lm))
    for s in (1, 30):
        ref = -ofe.dA_bilinear(Lm[:, s], U[:, s], ys[s], m)
        np.testing.assert_allclose(g[s], ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())
    h = ens.param_indicator(prob, to_dev(ys))
    for s in (0, 17, 31):
        assert h[s] == pytest.approx(ofe.param_indicator(ys[s], m), rel=1e-13)


def test_benchmark_grid_s64():
    ens = E()
    n, d, S, amp = 512, 4, 64, 0.4
    log_case(test="fullsize-512-s64", n=n, S=S)
    ys = workloads.uniform_samples(21, S, d)
    prob = ens.Problem(n, d, 0, amp)
    V, b = ens.assemble(prob, to_dev(ys))
    rng = np.random.default_rng(13)
    P = rng.standard_normal((n * n, S))
    q = ens.spmv(prob, V, to_dev(P)).cpu().numpy()
    for s in (0, 37, 63):
        A, _, _ = oprob.assemble(ys[s], n, 0, amp)
        ref = A @ P[:, s]
        assert np.max(np.abs(q[:, s] - ref)) <= 1e-13 * np.abs(A).sum(axis=1).max() * np.abs(P[:, s]).max()
    res = ens.solve(prob, V, b, ens.SolverOptions(rtol=1e-8, max_iter=20000))
    assert np.all(res.status == CONVERGED)
    x = res.x.cpu().numpy()
    for s in (0, 21, 42, 63):
        A, bo, _ = oprob.assemble(ys[s], n, 0, amp)
        assert np.linalg.norm(bo - A @ x[:, s]) <= 2e-8 * np.linalg.norm(bo)
