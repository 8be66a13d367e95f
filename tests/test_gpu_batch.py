"""GPU parity of the batched solver (ens_batch_solve, graph-replayed steps).

Each ensemble of a mixed batch must reproduce its single-ensemble solve:
same iteration counts (+-1) and, at equal counts, solutions within 1e-9; the
oracle's true residual within 2 rtol; replays of the graph with eager work
in between are bit-for-bit identical; retired and zero-rhs ensembles do not
disturb the others.
"""
import numpy as np
import pytest
import torch

from oracle import problem as oprob

pytestmark = pytest.mark.gpu

MIX = [(48, 4), (64, 16), (33, 32), (80, 8), (40, 64), (27, 2), (96, 32)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on an MI355X")
    yield


def make_batch(seed=0, mix=MIX, d=8, member_tiles=False):
    from paper_1705_02003_amd import ensemble as E
    rng = np.random.default_rng(seed)
    items, ys = [], []
    for k, (n, S) in enumerate(mix):
        prob = E.Problem(n, d, 1, 0.45)
        y = rng.uniform(-1, 1, (S, d))
        V, b = E.assemble(prob, torch.tensor(y, dtype=torch.float64, device="cuda"))
        it = {"prob": prob, "V": V, "b": b, "tile_lines": (0, 4, 16)[k % 3]}
        if member_tiles and S >= 8:
            it["member_tile"] = S // 2
        items.append(it)
        ys.append(y)
    return items, ys


@pytest.mark.parametrize("member_tiles", [False, True])
def test_batch_matches_single_solves_and_oracle(member_tiles):
    from paper_1705_02003_amd import ensemble as E
    items, ys = make_batch(member_tiles=member_tiles)
    print("CASE batch mix", MIX, flush=True)
    res = E.batch_solve(items, E.SolverOptions(rtol=1e-8))
    for it, y, r in zip(items, ys, res):
        single = E.solve(it["prob"], it["V"], it["b"], E.SolverOptions(rtol=1e-8))
        assert np.all(r.status == 0) and np.all(single.status == 0)
        assert np.all(np.abs(r.iters - single.iters) <= 1)
        assert r.ens_iters == int(r.iters.max())
        assert r.seconds > 0.0
        same = r.iters == single.iters
        num = torch.linalg.norm(r.x - single.x, dim=0).cpu().numpy()
        den = torch.linalg.norm(single.x, dim=0).cpu().numpy()
        assert np.all((num / den)[same] <= 1e-9)
        n = it["prob"].n
        x = r.x.cpu().numpy()
        for s in range(0, x.shape[1], max(1, x.shape[1] // 4)):
            A, b, _ = oprob.assemble(y[s], n, 1, 0.45)
            assert np.linalg.norm(b - A @ x[:, s]) <= 2e-8 * np.linalg.norm(b)


def test_batch_replays_are_deterministic():
    from paper_1705_02003_amd import ensemble as E
    items, _ = make_batch(seed=1)
    r1 = E.batch_solve(items, E.SolverOptions(rtol=1e-8))
    # eager work of the program between the two graph runs
    E.solve(items[0]["prob"], items[0]["V"], items[0]["b"])
    torch.cuda.synchronize()
    r2 = E.batch_solve(items, E.SolverOptions(rtol=1e-8))
    for a, b in zip(r1, r2):
        assert np.array_equal(a.iters, b.iters)
        assert torch.equal(a.x, b.x)


def test_batch_with_retired_and_capped_ensembles():
    from paper_1705_02003_amd import ensemble as E
    items, _ = make_batch(seed=2, mix=[(40, 8), (32, 4), (56, 16)])
    items[1]["b"].zero_()                       # every member has b = 0
    res = E.batch_solve(items, E.SolverOptions(rtol=1e-8))
    assert np.all(res[1].status == 3) and res[1].ens_iters == 0
    assert torch.count_nonzero(res[1].x).item() == 0
    for k in (0, 2):
        single = E.solve(items[k]["prob"], items[k]["V"], items[k]["b"])
        assert np.all(np.abs(res[k].iters - single.iters) <= 1)
    capped = E.batch_solve(items, E.SolverOptions(rtol=1e-8, max_iter=5))
    for k in (0, 2):
        assert np.all(capped[k].status == 1) and np.all(capped[k].iters == 5)


def test_batch_symmetric_sweep_bitwise():
    """The batched step's five-value symmetric sweep equals its nine-value
    sweep bit for bit."""
    from paper_1705_02003_amd import ensemble as E
    items, _ = make_batch(seed=3, member_tiles=True)
    r1 = E.batch_solve(items, E.SolverOptions(rtol=1e-8))
    r2 = E.batch_solve(items, E.SolverOptions(rtol=1e-8, full_stencil=True))
    for a, b in zip(r1, r2):
        assert np.array_equal(a.iters, b.iters)
        assert torch.equal(a.x, b.x)


def test_batch_in_waves_matches_single_solves():
    """Smallest-first waves (max_wave_bytes): every ensemble still reproduces
    its single solve, results come back in item order, and each ensemble's
    retirement time counts from the first wave's start."""
    from paper_1705_02003_amd import ensemble as E
    items, _ = make_batch(seed=2)
    print("CASE batch waves", MIX, flush=True)
    cost = [120 * it["prob"].rows * int(it["b"].shape[1]) for it in items]
    res = E.batch_solve(items, E.SolverOptions(rtol=1e-8), max_wave_bytes=2.5 * min(cost))
    assert len(res) == len(items)
    for it, r in zip(items, res):
        single = E.solve(it["prob"], it["V"], it["b"], E.SolverOptions(rtol=1e-8))
        assert r.x.shape == single.x.shape
        assert np.all(r.status == 0)
        assert np.all(np.abs(r.iters - single.iters) <= 1)
        same = r.iters == single.iters
        num = torch.linalg.norm(r.x - single.x, dim=0).cpu().numpy()
        den = torch.linalg.norm(single.x, dim=0).cpu().numpy()
        assert np.all((num / den)[same] <= 1e-9)
    # the smallest ensemble is in the first wave, the largest in the last
    assert res[int(np.argmin(cost))].seconds <= res[int(np.argmax(cost))].seconds


@pytest.mark.parametrize("wave_gb", [None, 0.002])
def test_batch_default_waves_bitwise(wave_gb):
    """Smallest-first waves (the autotuner's size, and a size small enough
    to leave several ensembles alone in their waves): an ensemble in a wave
    of several gives the same bits as in one batch (its partial sums land in
    rows fixed by its own unit indices, whatever else is in the batch), and
    an ensemble alone in its wave the bits of its single solve."""
    from paper_1705_02003_amd import autotune
    from paper_1705_02003_amd import ensemble as E
    wave = autotune.tune_wave()
    print("CASE batch auto waves", wave, wave_gb, flush=True)
    assert wave["wave_bytes"] > 0 and wave["ensembles"] >= 1
    items, _ = make_batch(seed=4)
    opts = E.SolverOptions(rtol=1e-8)
    wb = wave["wave_bytes"] if wave_gb is None else wave_gb * 1e9
    waves = E.plan_waves(items, wb)
    assert sorted(i for w in waves for i in w) == list(range(len(items)))
    r_auto = E.batch_solve(items, opts, max_wave_bytes="auto" if wave_gb is None else wb)
    r_one = E.batch_solve(items, opts, max_wave_bytes=None)
    alone = {w[0] for w in waves if len(w) == 1}
    if wave_gb is not None:
        assert len(alone) >= 2 and any(len(w) > 1 for w in waves)
    for i, (a, b) in enumerate(zip(r_auto, r_one)):
        if i in alone:
            from dataclasses import replace
            o = replace(opts, tile_lines=items[i]["tile_lines"],
                        member_tile=items[i].get("member_tile", 0))
            b = E.solve(items[i]["prob"], items[i]["V"], items[i]["b"], o)
        assert np.array_equal(a.iters, b.iters) and np.array_equal(a.status, b.status)
        assert torch.equal(a.x, b.x)
