"""The C ABI without a GPU: loading, exported symbols, host-side sparse-grid
calls bit-exact with the oracle, and argument validation (no device work)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import sparse_grid as sg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1705_02003_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1705_02003_amd import build
        build.build()
    _lib.lib()
    return _lib


def header_symbols():
    src = open(os.path.join(ROOT, "include", "ens.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ens_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(L):
    syms = header_symbols()
    assert len(syms) >= 14
    cdll = C.CDLL(L.LIB_PATH)
    for s in syms:
        assert hasattr(cdll, s), s
        assert s in L.SIGNATURES, s
    assert set(L.SIGNATURES) == set(syms)
    assert L.lib().ens_version() >= 100
    assert L.lib().ens_strerror(-1) == b"invalid argument"


def nodes_to_arrays(nodes):
    lv = np.array([[l for l, _ in nd] for nd in nodes], np.int32)
    ix = np.array([[k for _, k in nd] for nd in nodes], np.int32)
    return lv, ix


def adaptive_like_grid(d, L_, keep, seed):
    """A full grid with a random subset of its top levels removed (keeps
    every node's ancestors only partially, like an adaptive grid)."""
    rng = np.random.default_rng(seed)
    g = sg.full_grid(d, L_)
    return [nd for nd in g if sg.total_level(nd) <= 1 or rng.random() < keep]


@pytest.mark.parametrize("d,Lv,S,seed", [(2, 5, 8, 0), (4, 4, 16, 1), (4, 5, 32, 2), (8, 2, 32, 3), (3, 3, 4, 4)])
def test_group_samples_bit_exact_with_oracle(L, d, Lv, S, seed):
    from paper_1705_02003_amd import grouping
    rng = np.random.default_rng(seed)
    nodes = adaptive_like_grid(d, Lv, 0.7, seed)
    vals = rng.integers(50, 3000, len(nodes)).astype(float)      # iteration counts
    y_new = rng.uniform(-1, 1, (123, d))
    g_o, p_o = sg.group_samples(nodes, vals, y_new, S)
    lv, ix = nodes_to_arrays(nodes)
    g_c, p_c = grouping.group_samples(lv, ix, vals, y_new, S)
    assert np.array_equal(np.asarray(g_o), g_c)
    assert np.array_equal(p_o, p_c)        # bitwise
    # non-integer node values too (fixed evaluation order on both sides)
    vals2 = rng.standard_normal(len(nodes)) * 1e3
    g_o2, p_o2 = sg.group_samples(nodes, vals2, y_new, S)
    g_c2, p_c2 = grouping.group_samples(lv, ix, vals2, y_new, S)
    assert np.array_equal(np.asarray(g_o2), g_c2) and np.array_equal(p_o2, p_c2)


def test_group_samples_natural_order_and_padding(L):
    from paper_1705_02003_amd import grouping
    g, p = grouping.group_samples(None, None, None, np.zeros((9, 4)), 4)
    assert g.tolist() == [[0, 1, 2, 3], [4, 5, 6, 7], [8, 8, 8, 8]] and not p.any()


@pytest.mark.parametrize("d,Lv,seed", [(2, 5, 0), (4, 5, 1), (8, 2, 2)])
def test_surpluses_and_coords_bit_exact(L, d, Lv, seed):
    from paper_1705_02003_amd import grouping
    rng = np.random.default_rng(seed)
    nodes = adaptive_like_grid(d, Lv, 0.6, seed)
    perm = rng.permutation(len(nodes))
    nodes = [nodes[i] for i in perm]                  # any input order
    vals = rng.standard_normal(len(nodes))
    lv, ix = nodes_to_arrays(nodes)
    c = grouping.surpluses(lv, ix, vals)
    co = sg.surpluses(nodes, vals)
    assert np.array_equal(c, np.array([co[nd] for nd in nodes]))
    assert np.array_equal(grouping.coords(lv, ix), np.array([sg.coords(nd) for nd in nodes]))


@pytest.mark.parametrize("d,seed,tau,budget", [(2, 0, 1e-3, 10**6), (4, 1, 1e-3, 60), (4, 2, 0.05, 10**6), (3, 3, 0.0, 40)])
def test_refine_matches_oracle(L, d, seed, tau, budget):
    from paper_1705_02003_amd import grouping
    rng = np.random.default_rng(seed)
    nodes = sg.full_grid(d, 1)
    level = 1
    for _ in range(3):
        vals = [1.0 + float(np.sin(3 * sg.coords(nd)).sum()) + 0.1 * rng.random() for nd in nodes]
        new_o = sg.refine(nodes, vals, level, tau, budget)
        lv, ix = nodes_to_arrays(nodes)
        nl, ni = grouping.refine(lv, ix, vals, level, tau, budget)
        assert [tuple(zip(a, b)) for a, b in zip(nl.tolist(), ni.tolist())] == \
               [tuple(nd) for nd in new_o]
        if not new_o:
            break
        nodes = nodes + new_o
        level += 1


def test_initial_grid(L):
    from paper_1705_02003_amd import grouping
    lv, ix = grouping.initial_grid(4)
    assert len(lv) == 9
    got = sorted(tuple(zip(a, b)) for a, b in zip(lv.tolist(), ix.tolist()))
    assert got == sorted(tuple(nd) for nd in sg.full_grid(4, 1))


def test_cost_ratio_matches_oracle(L):
    from paper_1705_02003_amd import grouping
    rng = np.random.default_rng(3)
    its = rng.integers(10, 900, 37)
    for S in (4, 8, 16, 32):
        g = grouping.chunk(list(rng.permutation(37)), S)
        assert grouping.cost_ratio(g, its, S) == sg.ratio_R(g.tolist(), list(its), S)


def test_argument_validation_without_gpu(L):
    lib = L.lib()
    lvl = np.array([[3, 0]], np.int32)
    idx = np.array([[9, 0]], np.int32)                 # level 3 has indices 0..3
    out = np.zeros(2)
    rc = lib.ens_sg_coords(2, 1, lvl.ctypes.data_as(L.i32p), idx.ctypes.data_as(L.i32p),
                           out.ctypes.data_as(L.f64p))
    assert rc == L.ENS_EINVAL
    dup_l = np.zeros((2, 2), np.int32)
    rc = lib.ens_sg_surpluses(2, 2, dup_l.ctypes.data_as(L.i32p), dup_l.ctypes.data_as(L.i32p),
                              np.ones(2).ctypes.data_as(L.f64p), np.zeros(2).ctypes.data_as(L.f64p))
    assert rc == L.ENS_EINVAL
    prob = L.ens_problem(64, 2, 0, 0, 0.0)
    opts = L.ens_opts()
    for S in (0, -1, 65, 128):                                                      # S outside [1, 64]
        assert lib.ens_pcg_workspace_bytes(C.byref(prob), C.byref(opts), S) == 0
    for S in (3, 20, 24, 48, 64):                                                   # any width in [1, 64]
        assert lib.ens_pcg_workspace_bytes(C.byref(prob), C.byref(opts), S) > 64 * 64 * S * 8 * 5
    assert lib.ens_pcg_workspace_bytes(C.byref(prob), C.byref(opts), 32) > 64 * 64 * 32 * 8 * 5
    bad = L.ens_problem(1, 2, 0, 0, 0.0)
    assert lib.ens_pcg_workspace_bytes(C.byref(bad), C.byref(opts), 8) == 0
    # null pointers and bad sizes are rejected before any device call
    rc = lib.ens_pcg_solve(C.byref(prob), C.byref(opts), 8, None, None, None, None, None, None,
                           None, None, None, 0, None)
    assert rc == L.ENS_EINVAL
    rc = lib.ens_assemble_ensemble(C.byref(prob), 6, None, C.c_void_p(16), C.c_void_p(16), None)
    assert rc == L.ENS_EINVAL
    rc = lib.ens_assemble_ensemble(C.byref(prob), 65, np.zeros((65, 2)).ctypes.data_as(L.f64p),
                                   C.c_void_p(16), C.c_void_p(16), None)
    assert rc == L.ENS_EINVAL
    opts_bad = L.ens_opts(5, 0, 0.0, 0.0, 0, 0, 0, 0, 0, 0)
    assert lib.ens_pcg_workspace_bytes(C.byref(prob), C.byref(opts_bad), 8) == 0
    # a too-small workspace is ENS_ENOMEM, still before any device work
    rc = lib.ens_pcg_solve(C.byref(prob), C.byref(opts), 8, C.c_void_p(256), C.c_void_p(256),
                           C.c_void_p(256), None, None, None, None, None, C.c_void_p(256), 1024, None)
    assert rc == L.ENS_ENOMEM


def test_grouping_strategies_on_recorded_counts(L):
    """The strategy comparison of the benchmark works from recorded counts:
    'its' is optimal (no grouping has fewer ensemble iterations), 'param'
    orders by the indicator H, every strategy covers every sample, and regrouping at
    another width reproduces the host surrogate grouping (Section 3.1)."""
    from paper_1705_02003_amd import grouping, uq
    rng = np.random.default_rng(11)
    res = uq.UQResult()
    lv1, ix1 = grouping.initial_grid(4)
    y1 = grouping.coords(lv1, ix1)
    # later levels: any distinct dyadic nodes will do for the bookkeeping
    lv2, ix2 = grouping.full_grid(4, 2)
    keep = np.array([i for i in range(len(lv2)) if lv2[i].sum() == 2])
    lv2, ix2 = lv2[keep], ix2[keep]
    y2 = grouping.coords(lv2, ix2)
    it1 = rng.integers(100, 900, len(y1))
    it2 = rng.integers(100, 900, len(y2))
    res.level = np.vstack([lv1, lv2]).astype(np.int32)
    res.index = np.vstack([ix1, ix2]).astype(np.int32)
    res.y = np.vstack([y1, y2])
    res.iters = np.concatenate([it1, it2])
    res.hind = 10.0 ** (1.0 + res.y[:, 0])        # the 2-D model's H = 1 / eps(y_1)
    g32, _ = grouping.group_samples(lv1, ix1, it1, y2, 32)
    res.levels = [uq.LevelRecord(1, len(y1), grouping.chunk(list(range(len(y1))), 32), [], it1,
                                 np.zeros(len(y1)), np.zeros(len(y1)), 0.0),
                  uq.LevelRecord(2, len(y2), g32, [], it2, np.zeros(len(y2)), np.zeros(len(y2)), 0.0)]
    for S in (32, 8):
        per = uq.strategy_groups(res, S)
        costs = uq.grouping_costs(res, S)
        for k, lst in per.items():
            for r, g in zip(res.levels, lst):
                assert g.shape[1] == S
                assert sorted(set(g.reshape(-1).tolist())) == list(range(r.n_samples))
            assert costs["its"]["sum_ensemble_iters"] <= costs[k]["sum_ensemble_iters"]
        order = per["param"][1].reshape(-1)
        h2 = res.hind[len(y1):]
        assert np.all(np.diff(h2[order[:len(y2)]]) >= 0)
        expect, _ = grouping.group_samples(lv1, ix1, it1, y2, S)
        assert np.array_equal(per["surrogate"][1], expect)


def test_layout_and_new_entry_points_without_gpu(L):
    """Slot stride, batch sizing and triad / batch argument checks (no device
    work: every call below fails validation first)."""
    lib = L.lib()
    prob = L.ens_problem(512, 4, 0, 0, 0.4)
    # the slot stride pads N_r S to a multiple of 32 plus 512 elements
    for n, S in ((512, 32), (1024, 32), (64, 8), (33, 1), (27, 2)):
        p = L.ens_problem(n, 4, 0, 0, 0.4)
        Ls = lib.ens_matrix_slot_stride(C.byref(p), S)
        nr_s = n * n * S
        assert Ls == ((nr_s + 31) // 32) * 32 + 512
        assert Ls % 32 == 0 and Ls - nr_s >= 512
    assert lib.ens_matrix_slot_stride(C.byref(prob), 65) == 0
    assert lib.ens_matrix_slot_stride(C.byref(prob), 48) == ((512 * 512 * 48 + 31) // 32) * 32 + 512
    assert lib.ens_batch_workspace_bytes(0) == 0
    assert lib.ens_batch_workspace_bytes(1025) == 0
    assert lib.ens_batch_workspace_bytes(64) > 0
    # triad: null, misaligned, empty, non-finite scalar
    a = C.c_void_p(4096)
    assert lib.ens_stream_triad(None, a, a, 1.0, 8, None) == L.ENS_EINVAL
    assert lib.ens_stream_triad(a, C.c_void_p(4104), a, 1.0, 8, None) == L.ENS_EINVAL
    assert lib.ens_stream_triad(a, a, a, 1.0, 0, None) == L.ENS_EINVAL
    assert lib.ens_stream_triad(a, a, a, float("nan"), 8, None) == L.ENS_EINVAL
    # stream mix: odd or zero n, stride below n, misaligned, an unsupported mix
    assert lib.ens_stream_mix(a, a, 16, 7, 8, 3, None) == L.ENS_EINVAL
    assert lib.ens_stream_mix(a, a, 16, 0, 8, 3, None) == L.ENS_EINVAL
    assert lib.ens_stream_mix(a, a, 8, 16, 8, 3, None) == L.ENS_EINVAL
    assert lib.ens_stream_mix(C.c_void_p(4104), a, 16, 16, 8, 3, None) == L.ENS_EINVAL
    assert lib.ens_stream_mix(a, a, 16, 16, 4, 4, None) == L.ENS_ENOTSUP
    # batch: no items, too many items, a bad width, a too-small item workspace
    bws = C.c_void_p(4096)
    nb = lib.ens_batch_workspace_bytes(1)
    items = (L.ens_batch_item * 1)()
    assert lib.ens_batch_solve(None, 0, items, bws, nb, None) == L.ENS_EINVAL
    assert lib.ens_batch_solve(None, 1, items, bws, nb - 1, None) == L.ENS_ENOMEM
    it = items[0]
    it.prob = prob
    it.S = 65
    it.V_dev = it.b_dev = it.x_dev = it.ws_dev = 4096
    it.ws_bytes = 1 << 40
    assert lib.ens_batch_solve(None, 1, items, bws, nb, None) == L.ENS_EINVAL
    it.S = 24                     # valid width, but the batched solver takes powers of two
    assert lib.ens_batch_solve(None, 1, items, bws, nb, None) == L.ENS_ENOTSUP
    it.S = 32
    it.ws_bytes = 1024
    assert lib.ens_batch_solve(None, 1, items, bws, nb, None) == L.ENS_ENOMEM
    opts = L.ens_opts()
    opts.precond = L.PRECOND_CHEBYSHEV
    it.ws_bytes = 1 << 40
    assert lib.ens_batch_solve(C.byref(opts), 1, items, bws, nb, None) == L.ENS_ENOTSUP


@pytest.mark.parametrize("d,Lv,seed", [(2, 5, 0), (4, 5, 1), (8, 2, 2), (1, 6, 3)])
def test_expectation_bit_exact_with_oracle(L, d, Lv, seed):
    from paper_1705_02003_amd import grouping
    rng = np.random.default_rng(seed)
    nodes = adaptive_like_grid(d, Lv, 0.6, seed)
    nodes = [nodes[i] for i in rng.permutation(len(nodes))]
    lv, ix = nodes_to_arrays(nodes)
    for vals in (rng.integers(50, 3000, len(nodes)).astype(float), rng.standard_normal(len(nodes))):
        assert grouping.expectation(lv, ix, vals) == sg.expectation(sg.surpluses(nodes, vals))


def test_expectation_rejects_bad_arguments(L):
    lib = L.lib()
    lv = np.zeros((1, 2), np.int32)
    out = np.zeros(1)
    v = np.array([np.nan])
    args = (lv.ctypes.data_as(L.i32p), lv.ctypes.data_as(L.i32p))
    assert lib.ens_sg_expectation(2, 1, *args, v.ctypes.data_as(L.f64p), out.ctypes.data_as(L.f64p)) < 0
    v[0] = 2.0
    assert lib.ens_sg_expectation(2, 0, *args, v.ctypes.data_as(L.f64p), out.ctypes.data_as(L.f64p)) < 0
    assert lib.ens_sg_expectation(2, 1, *args, v.ctypes.data_as(L.f64p), None) < 0
    assert lib.ens_sg_expectation(2, 1, *args, v.ctypes.data_as(L.f64p), out.ctypes.data_as(L.f64p)) == 0
    assert out[0] == 2.0


@pytest.mark.parametrize("M,seed", [(1, 0), (7, 1), (100, 2), (515, 3), (1000, 4)])
def test_group_variable_bit_exact_with_oracle(L, M, seed):
    from paper_1705_02003_amd import grouping
    rng = np.random.default_rng(seed)
    widths = [1, 2, 4, 8, 16, 32, 64]
    ts = [1.0 / su for su in (1.0, 1.55, 2.36, 3.27, 4.01, 4.17, 3.59)]
    ts = [w * t for w, t in zip(widths, ts)]
    for pred in (rng.integers(30, 3000, M).astype(float), rng.normal(500, 300, M)):
        g_o, c_o = sg.group_variable(pred, widths, ts)
        g_c, c_c = grouping.group_variable(pred, widths, ts)
        assert [list(g) for g in g_c] == g_o
        assert c_c == c_o
    sub = [4, 16, 64]
    g_o, c_o = sg.group_variable(pred, sub, [ts[2], ts[4], ts[6]])
    g_c, c_c = grouping.group_variable(pred, sub, [ts[2], ts[4], ts[6]])
    assert [list(g) for g in g_c] == g_o and c_c == c_o
    # any widths the solver takes (not only powers of two), up to all 64
    for wl in ([3, 5, 20, 48], list(range(1, 65))):
        tw = [w / (1.0 + 3.5 * (1.0 - np.exp(-w / 12.0))) for w in wl]
        g_o, c_o = sg.group_variable(pred, wl, tw)
        g_c, c_c = grouping.group_variable(pred, wl, tw)
        assert [list(g) for g in g_c] == g_o and c_c == c_o


def test_group_variable_rejects_bad_arguments(L):
    from paper_1705_02003_amd import grouping
    pred = np.ones(5)
    for widths, ts in (([0], [1.0]), ([4, 2], [1.0, 1.0]), ([128], [1.0]), ([65], [1.0]),
                       ([1], [0.0]), ([1], [np.inf]), ([1, 1], [1.0, 1.0]), ([], [])):
        with pytest.raises(RuntimeError):
            grouping.group_variable(pred, widths, ts)
    with pytest.raises(RuntimeError):
        grouping.group_variable(np.array([1.0, np.nan]), [1], [1.0])
    with pytest.raises(RuntimeError):
        grouping.group_variable(np.zeros(0), [1], [1.0])


def test_3d_model_descriptor_without_gpu(L):
    """dim = 3: slot stride and workspace over n^3 rows, descriptor limits,
    argument checks, and the batched solver's refusal of the 3-D model (no
    device work: every call below fails validation first)."""
    lib = L.lib()
    o = L.ens_opts()
    for n, S in ((31, 32), (10, 1), (64, 16)):
        p = L.ens_problem(n, 4, 0, 3, 0.0)
        Ls = lib.ens_matrix_slot_stride(C.byref(p), S)
        assert Ls == ((n ** 3 * S + 31) // 32) * 32 + 512
        ws = lib.ens_pcg_workspace_bytes(C.byref(p), C.byref(o), S)
        p2 = L.ens_problem(n, 4, 0, 2, 0.0)
        ws2 = lib.ens_pcg_workspace_bytes(C.byref(p2), C.byref(o), S)
        # five vectors of the slot stride beyond the same header
        assert ws - ws2 == 5 * 8 * (Ls - lib.ens_matrix_slot_stride(C.byref(p2), S))
    assert lib.ens_matrix_slot_stride(C.byref(L.ens_problem(31, 4, 1, 3, 0.0)), 8) > 0   # Test 2
    for bad in (L.ens_problem(31, 4, 2, 3, 0.0), L.ens_problem(31, 4, 0, 3, 0.4),
                L.ens_problem(31, 0, 0, 3, 0.0), L.ens_problem(31, 17, 0, 3, 0.0),
                L.ens_problem(1, 4, 0, 3, 0.0), L.ens_problem(1025, 4, 0, 3, 0.0),
                L.ens_problem(31, 4, 0, 4, 0.0), L.ens_problem(31, 4, 0, 1, 0.0)):
        assert lib.ens_matrix_slot_stride(C.byref(bad), 8) == 0
        assert lib.ens_pcg_workspace_bytes(C.byref(bad), C.byref(o), 8) == 0
    # 1 <= d is allowed in 3-D (the 2-D model needs d >= 2)
    assert lib.ens_matrix_slot_stride(C.byref(L.ens_problem(31, 1, 0, 3, 0.0)), 8) > 0
    assert lib.ens_matrix_slot_stride(C.byref(L.ens_problem(31, 1, 0, 2, 0.0)), 8) == 0
    p = L.ens_problem(8, 4, 0, 3, 0.0)
    a = C.c_void_p(4096)
    g = np.zeros(64)
    assert lib.ens_assemble_ensemble(C.byref(p), 8, None, a, a, None) == L.ENS_EINVAL
    yh = np.zeros((8, 4)).ctypes.data_as(L.f64p)
    assert lib.ens_dqdy(C.byref(p), 8, yh, a, None, g.ctypes.data_as(L.f64p), a, 1 << 30,
                        None) == L.ENS_EINVAL
    assert lib.ens_dqdy(C.byref(p), 8, yh, a, a, g.ctypes.data_as(L.f64p), a, 16, None) == L.ENS_ENOMEM
    nb = lib.ens_batch_workspace_bytes(1)
    items = (L.ens_batch_item * 1)()
    it = items[0]
    it.prob = p
    it.S = 8
    it.V_dev = it.b_dev = it.x_dev = it.ws_dev = 4096
    it.ws_bytes = 1 << 40
    assert lib.ens_batch_solve(None, 1, items, C.c_void_p(4096), nb, None) == L.ENS_ENOTSUP


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_non_finite_parameters_rejected_before_device_work(L, bad):
    """A non-finite parameter value is ENS_EINVAL from every entry point that
    takes parameters, checked on the host before any device call (the device
    pointers below are never dereferenced)."""
    lib = L.lib()
    dev = C.c_void_p(256)
    for prob in (L.ens_problem(16, 4, 0, 2, 0.4), L.ens_problem(7, 3, 0, 3, 0.0)):
        for S in (1, 5, 20):
            y = np.zeros((S, prob.d))
            y[S - 1, prob.d - 1] = bad
            yp = y.ctypes.data_as(L.f64p)
            assert lib.ens_assemble_ensemble(C.byref(prob), S, yp, dev, dev, None) == L.ENS_EINVAL
            h = np.zeros(S)
            assert lib.ens_param_indicator(C.byref(prob), S, yp, h.ctypes.data_as(L.f64p), dev,
                                           1 << 30, None) == L.ENS_EINVAL
            g = np.zeros((S, prob.d))
            assert lib.ens_dqdy(C.byref(prob), S, yp, dev, dev, g.ctypes.data_as(L.f64p), dev,
                                1 << 30, None) == L.ENS_EINVAL
            it = np.zeros(S, np.int32)
            assert lib.ens_adjoint_grad(C.byref(prob), None, S, yp, dev, dev, dev, dev,
                                        g.ctypes.data_as(L.f64p), it.ctypes.data_as(L.i32p),
                                        it.ctypes.data_as(L.i32p), dev, 1 << 40, None) == L.ENS_EINVAL
    assert lib.ens_qoi_weights(C.byref(L.ens_problem(16, 4, 0, 2, 0.4)), None, None) == L.ENS_EINVAL
    # n = 2: no interior node lies in [0.4, 0.6] (5 i in [6, 9] has no solution)
    assert lib.ens_qoi_weights(C.byref(L.ens_problem(2, 4, 0, 2, 0.4)), C.c_void_p(256),
                               None) == L.ENS_EINVAL


def test_multigrid_descriptor_without_gpu(L):
    """ENS_PRECOND_MULTIGRID: the workspace adds the coarse levels (a header of
    per-level smoother coefficients, then per level 27 matrix slots and four
    vectors of the level's slot stride, and for levels of at most 7 nodes per
    direction a member-major copy of the 27 slots); the 2-D model and grids
    with n + 1 not a power of two are refused before any device work."""
    lib = L.lib()
    o = L.ens_opts()
    o.precond = L.PRECOND_MULTIGRID
    oc = L.ens_opts()
    oc.precond = L.PRECOND_CHEBYSHEV

    def stride(m, S):
        return ((m ** 3 * S + 31) // 32) * 32 + 512

    for n, S in ((15, 8), (31, 32), (3, 1), (63, 64)):
        p = L.ens_problem(n, 4, 0, 3, 0.0)
        ws = lib.ens_pcg_workspace_bytes(C.byref(p), C.byref(o), S)
        wc = lib.ens_pcg_workspace_bytes(C.byref(p), C.byref(oc), S)
        levels, m = [], n
        while m > 1:
            m = (m - 1) // 2
            levels.append(m)
        head = ((8 * 12 * 64 * (2 * 8 + 2 + 1) + 255) // 256) * 256
        copy = sum(((8 * 27 * m ** 3 * S + 255) // 256) * 256 for m in levels if m <= 7)
        assert ws - wc == head + sum(8 * 31 * stride(m, S) for m in levels) + copy, (n, S)
    a = C.c_void_p(4096)
    for bad in (L.ens_problem(10, 4, 0, 3, 0.0), L.ens_problem(31, 4, 0, 2, 0.4),
                L.ens_problem(16, 4, 0, 3, 0.0)):
        assert lib.ens_pcg_workspace_bytes(C.byref(bad), C.byref(o), 8) == 0
        assert lib.ens_pcg_solve(C.byref(bad), C.byref(o), 8, a, a, a, None, None, None, None, None,
                                 a, 1 << 40, None) == L.ENS_ENOTSUP
        assert lib.ens_pcg_solve_noalloc(C.byref(bad), C.byref(o), 8, a, a, a, None, None, None, None,
                                         None) == L.ENS_ENOTSUP
        assert lib.ens_mg_apply(C.byref(bad), None, 8, a, a, a, None, a, 1 << 40, None) == L.ENS_ENOTSUP
    p = L.ens_problem(15, 4, 0, 3, 0.0)
    assert lib.ens_mg_apply(C.byref(p), None, 8, a, a, a, None, a, 16, None) == L.ENS_ENOMEM
    assert lib.ens_mg_apply(C.byref(p), None, 65, a, a, a, None, a, 1 << 40, None) == L.ENS_EINVAL
    # the batched solver is Jacobi-only
    items = (L.ens_batch_item * 1)()
    it = items[0]
    it.prob = L.ens_problem(16, 4, 0, 2, 0.4)
    it.S = 8
    it.V_dev = it.b_dev = it.x_dev = it.ws_dev = 4096
    it.ws_bytes = 1 << 40
    nb = lib.ens_batch_workspace_bytes(1)
    assert lib.ens_batch_solve(C.byref(o), 1, items, a, nb, None) == L.ENS_ENOTSUP
