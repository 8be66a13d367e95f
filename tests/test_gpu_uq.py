"""The adaptive loop (Section 3.1, Fig. 2) end to end on the GPU against the
oracle, on a small grid.

Per sample: the iteration count within +-1 of the oracle's PCG and
G(y) = ||u||^2 within 1e-9 relative (two PCG solves stopped at rtol 1e-8,
even one iteration apart, differ in G by about 1e-11 here).  The host steps
are exact functions of the recorded numbers, so they are compared bit for bit
with the oracle fed the same numbers: each level's new nodes (refinement on
the GPU's G values), each level's ensembles (surrogate of the GPU's
iteration counts), and E[G^] after each level.
"""
import numpy as np
import pytest
import torch

from oracle import pcg as opcg
from oracle import problem as oprob
from oracle import sparse_grid as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on an MI355X")
    yield


def nodes_of(level, index):
    return [tuple((int(l), int(k)) for l, k in zip(lr, kr)) for lr, kr in zip(level, index)]


@pytest.mark.parametrize("n,S,budget,max_level,tau", [(24, 8, 70, 3, 1e-3), (17, 4, 45, 4, 5e-3)])
def test_adaptive_loop_matches_oracle(n, S, budget, max_level, tau):
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq
    print(f"CASE adaptive n={n} S={S} budget={budget}", flush=True)
    d, rtol = 4, 1e-8
    prob = E.Problem(n, d, 0, 0.4)
    res = uq.adaptive(prob, S, budget=budget, max_level=max_level, tau_rel=tau,
                      strategy="surrogate", opts=E.SolverOptions(rtol=rtol))
    nodes = nodes_of(res.level, res.index)
    assert len(nodes) == len(set(nodes)) == len(res.y) <= budget
    assert len(res.levels) >= 2

    # per sample: the solve
    for m, nd in enumerate(nodes):
        y = sg.coords(nd)
        assert np.array_equal(y, res.y[m])
        A, b, dg = oprob.assemble(y, n, 0, 0.4)
        x, it, _, _ = opcg.pcg(A, b, dg, rtol, 20000)
        assert abs(int(res.iters[m]) - it) <= 1, (m, res.iters[m], it)
        g = float(x @ x)
        assert abs(res.qoi[m] - g) <= 1e-9 * g, (m, res.qoi[m], g)

    # per level: refinement, grouping and E[G^] from the recorded numbers
    start = 0
    for li, rec in enumerate(res.levels):
        here = nodes[start:start + rec.n_samples]
        before = nodes[:start]
        if li == 0:
            assert here == sg.full_grid(d, 1)
            assert rec.groups.tolist() == sg.chunk(list(range(rec.n_samples)), S)
        else:
            new = sg.refine(before, res.qoi[:start], rec.level - 1, tau, budget)
            assert here == new
            groups, pred = sg.group_samples(before, res.iters[:start].astype(float),
                                            res.y[start:start + rec.n_samples], S)
            assert rec.groups.tolist() == groups
            assert np.array_equal(rec.pred, pred)
        upto = nodes[:start + rec.n_samples]
        c = sg.surpluses(upto, res.qoi[:start + rec.n_samples])
        assert rec.qoi_mean == sg.expectation(c)
        start += rec.n_samples
    assert res.qoi_mean == res.levels[-1].qoi_mean
    # the ensemble counts are the max over their members
    for rec in res.levels:
        for g, k in zip(rec.groups, rec.ens_iters):
            assert k == int(rec.iters[g].max())


def test_adaptive_loop_variable_widths_matches_oracle():
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq
    n, d, rtol, tau, budget = 20, 4, 1e-8, 1e-3, 60
    widths, secs = [1, 2, 4, 8, 16], [1.0, 1.3, 1.7, 2.6, 4.5]
    print(f"CASE adaptive-variable n={n} widths={widths}", flush=True)
    prob = E.Problem(n, d, 0, 0.4)
    res = uq.adaptive(prob, 8, budget=budget, max_level=3, tau_rel=tau, strategy="variable",
                      opts=E.SolverOptions(rtol=rtol), widths=widths, iter_seconds=secs)
    nodes = nodes_of(res.level, res.index)
    start = 0
    for rec in res.levels:
        m = rec.n_samples
        if rec.level == 1:
            pred = np.ones(m)
        else:
            _, pred = sg.group_samples(nodes[:start], res.iters[:start].astype(float),
                                       res.y[start:start + m], 1)
        groups, _ = sg.group_variable(pred, widths, secs)
        assert [list(g) for g in rec.groups] == groups
        assert sorted(set(sum(groups, []))) == list(range(m))
        for g, k in zip(rec.groups, rec.ens_iters):
            assert k == int(rec.iters[np.asarray(g)].max())
        start += m
    for mi, nd in enumerate(nodes):
        A, b, dg = oprob.assemble(sg.coords(nd), n, 0, 0.4)
        x, it, _, _ = opcg.pcg(A, b, dg, rtol, 20000)
        assert abs(int(res.iters[mi]) - it) <= 1
        assert abs(res.qoi[mi] - float(x @ x)) <= 1e-9 * float(x @ x)


def test_concurrent_streams_give_the_same_results():
    """Ensembles solved two or three at a time on separate streams: every
    sample's count, G and the grouping are bit for bit those of one at a
    time (each ensemble's arithmetic does not depend on the others)."""
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq
    print("CASE adaptive-streams", flush=True)
    for prob in (E.Problem(20, 4, 0, 0.4), E.Problem(9, 4, dim=3)):
        base = uq.adaptive(prob, 4, budget=40, max_level=3, tau_rel=1e-3,
                           opts=E.SolverOptions(rtol=1e-8))
        for K in (2, 3):
            res = uq.adaptive(prob, 4, budget=40, max_level=3, tau_rel=1e-3,
                              opts=E.SolverOptions(rtol=1e-8), streams=K)
            assert np.array_equal(res.iters, base.iters)
            assert np.array_equal(res.qoi, base.qoi)
            for a, b in zip(res.levels, base.levels):
                assert np.array_equal(np.asarray(a.groups), np.asarray(b.groups))
                assert a.ens_iters == b.ens_iters


@pytest.mark.parametrize("dim", [2, 3])
def test_adaptive_loop_param_strategy(dim):
    """Parameter-based grouping (Section 3.2) in the loop: the library's H
    agrees with the oracle's indicator to 1e-13, and each level's ensembles
    are the (H, generation index) order cut into S (sparse-grid samples share
    coordinates, so exact ties occur and fall back to generation order)."""
    from oracle import fe3d as ofe
    from oracle import problem as oprob2
    from paper_1705_02003_amd import ensemble as E
    from paper_1705_02003_amd import uq
    print(f"CASE adaptive-param dim={dim}", flush=True)
    prob = E.Problem(16, 4, 0, 0.4) if dim == 2 else E.Problem(7, 4, dim=3)
    res = uq.adaptive(prob, 4, budget=45, max_level=3, tau_rel=1e-3, strategy="param",
                      opts=E.SolverOptions(rtol=1e-8))
    start = 0
    for rec in res.levels:
        ys = res.y[start:start + rec.n_samples]
        h = np.array([oprob2.param_indicator(y, 0) if dim == 2 else ofe.param_indicator(y, prob.n)
                      for y in ys])
        np.testing.assert_allclose(res.hind[start:start + rec.n_samples], h, rtol=1e-13)
        want = sg.chunk(sorted(range(rec.n_samples), key=lambda i: (res.hind[start + i], i)), 4)
        assert rec.groups.tolist() == want
        start += rec.n_samples
