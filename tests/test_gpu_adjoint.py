"""GPU parity of the differentiation path (EnsembleQoI through the C ABI).

Q_s = w^T u_s, u_s = A(y_s)^-1 1; dQ/dy from the adjoint ensemble PCG and the
dQ/dy kernel.  References: the oracle's direct-solve adjoint gradient
(pinned against a complex-step derivative) and central differences of the
GPU forward map with tight solves.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on an MI355X")
    yield


def rel_err(g, ref):
    scale = np.maximum(np.abs(ref), 1e-2 * np.abs(ref).max(axis=-1, keepdims=True))
    return float(np.max(np.abs(g - ref) / scale))


@pytest.mark.parametrize("n,S,d,eps_model,amp", [(64, 8, 6, 0, 0.4), (40, 4, 8, 1, 0.45)])
def test_autograd_matches_oracle_adjoint(n, S, d, eps_model, amp):
    print("CASE autograd", n, S, d, flush=True)
    from paper_1705_02003_amd import autograd as A
    from paper_1705_02003_amd import ensemble as E
    prob = E.Problem(n, d, eps_model, amp)
    ys = np.random.default_rng(40 + n).uniform(-1, 1, (S, d))
    y = torch.tensor(ys, dtype=torch.float64, device="cuda", requires_grad=True)
    opts = E.SolverOptions(rtol=1e-12)
    Q = A.EnsembleQoI.apply(y, prob, opts)
    Q.sum().backward()
    g = y.grad.cpu().numpy()
    for s in range(S):
        Qo, go, _, _ = oadj.qoi_and_grad(ys[s], n, eps_model, amp)
        assert Q[s].item() == pytest.approx(Qo, rel=1e-10)
        assert rel_err(g[s], go) <= 1e-8


def test_autograd_weighted_backward():
    """The incoming gradient scales each member's row."""
    from paper_1705_02003_amd import autograd as A
    from paper_1705_02003_amd import ensemble as E
    prob = E.Problem(32, 4, 0, 0.4)
    ys = np.random.default_rng(3).uniform(-1, 1, (4, 4))
    y = torch.tensor(ys, dtype=torch.float64, device="cuda", requires_grad=True)
    Q = A.EnsembleQoI.apply(y, prob, E.SolverOptions(rtol=1e-12))
    wts = torch.tensor([1.0, -2.0, 0.5, 0.0], dtype=torch.float64, device="cuda")
    (Q * wts).sum().backward()
    g1 = y.grad.clone()
    y.grad = None
    Q = A.EnsembleQoI.apply(y, prob, E.SolverOptions(rtol=1e-12))
    Q.sum().backward()
    torch.testing.assert_close(g1, y.grad * wts[:, None], rtol=1e-12, atol=1e-18)


def test_adjoint_gradient_matches_central_differences():
    """Adjoint gradient vs central differences (h = 1e-6) of the GPU forward
    map solved to rtol 1e-13 (FD at rtol 1e-8 would be noise-limited at
    ~rtol / h).  Measured per member norm-wise (max_j |g_j - fd_j| / max_j
    |fd_j|): ~3e-8 at both rtol 1e-8 and 1e-10, i.e. the FD noise floor at
    h = 1e-6 (about 1e-14 relative noise in Q divided by 2h), not the adjoint
    solve.  Component-wise against max(|g_j|, 1e-2 ||g||) that floor reads as
    ~3e-6 for the smallest components.  The adjoint gradient itself is pinned
    component-wise against the oracle in test_autograd_matches_oracle_adjoint."""
    from paper_1705_02003_amd import autograd as A
    from paper_1705_02003_amd import ensemble as E
    n, S, d = 96, 16, 6
    prob = E.Problem(n, d, 0, 0.4)
    ys = np.random.default_rng(4).uniform(-1, 1, (S, d))
    fd = A.central_difference(prob, torch.tensor(ys, dtype=torch.float64, device="cuda"), 1e-6,
                              E.SolverOptions(rtol=1e-13))
    errs = {}
    for rtol in (1e-8, 1e-10):
        y = torch.tensor(ys, dtype=torch.float64, device="cuda", requires_grad=True)
        A.EnsembleQoI.apply(y, prob, E.SolverOptions(rtol=rtol)).sum().backward()
        g = y.grad.cpu().numpy()
        errs[rtol] = (rel_err(g, fd), float(np.max(np.abs(g - fd)) / np.abs(fd).max()))
        print(f"adjoint at rtol {rtol:g} vs FD: component-wise {errs[rtol][0]:.3e}, "
              f"norm-wise {errs[rtol][1]:.3e}", flush=True)
    for rtol in errs:
        assert errs[rtol][1] <= 1e-6
        assert errs[rtol][0] <= 1e-5


def test_adjoint_gradient_matches_extrapolated_differences():
    """Component-wise pin of the adjoint gradient against differences whose
    own error is below 1e-6: Richardson-extrapolated central differences
    (4 D(h) - D(2h)) / 3 at h = 1e-3 (truncation O(h^4), about 1e-12 here;
    rounding about 1e-14 |Q| / h), forward map solved to rtol 1e-13.
    Component-wise against max(|fd_j|, 1e-3 max_j |fd_j|), at the adjoint
    solve's rtol 1e-8 and 1e-10."""
    from paper_1705_02003_amd import autograd as A
    from paper_1705_02003_amd import ensemble as E
    n, S, d = 96, 16, 6
    prob = E.Problem(n, d, 0, 0.4)
    ys = np.random.default_rng(4).uniform(-1, 1, (S, d))
    yt = torch.tensor(ys, dtype=torch.float64, device="cuda")
    fo = E.SolverOptions(rtol=1e-13)
    h = 1e-3
    fd = (4 * A.central_difference(prob, yt, h, fo) - A.central_difference(prob, yt, 2 * h, fo)) / 3
    for rtol in (1e-8, 1e-10):
        y = torch.tensor(ys, dtype=torch.float64, device="cuda", requires_grad=True)
        A.EnsembleQoI.apply(y, prob, E.SolverOptions(rtol=rtol)).sum().backward()
        g = y.grad.cpu().numpy()
        scale = np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max(axis=-1, keepdims=True))
        err = float(np.max(np.abs(g - fd) / scale))
        print(f"adjoint at rtol {rtol:g} vs extrapolated differences: component-wise {err:.3e}",
              flush=True)
        assert err <= 1e-6
