"""The no-allocation solve (ens_pcg_solve_noalloc) against ens_pcg_solve.

Both run the same kernels with the same launch shapes; only the workspace
(the library's per-device array instead of the caller's) and the way the
host checks the done flag differ, and neither changes the arithmetic.  So
iterations, status, relative residuals and x must be the same bits.  Two
calls in a row, the second on a smaller input (the array keeps the first
call's contents), both preconditioners; a request beyond the array's size
is refused with ENS_ENOMEM before any work.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests must run on an MI355X")
    yield


def log_case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _case(n, S, d, precond, seed):
    from paper_1705_02003_amd import ensemble as E
    prob = E.Problem(n, d, 1 if precond == "chebyshev" else 0, 0.45 if precond == "chebyshev" else 0.4)
    ys = workloads.uniform_samples(seed, S, d)
    V, b = E.assemble(prob, torch.tensor(ys, dtype=torch.float64, device="cuda"))
    return prob, V, b


@pytest.mark.parametrize("precond", ["jacobi", "chebyshev"])
def test_noalloc_matches_solve_twice_then_smaller(precond):
    from paper_1705_02003_amd import ensemble as E
    opts = E.SolverOptions(precond=precond, rtol=1e-8)
    for n, S, seed in ((160, 32, 1), (70, 8, 2)):
        log_case(test="noalloc", precond=precond, n=n, S=S)
        prob, V, b = _case(n, S, 8 if precond == "chebyshev" else 4, precond, seed)
        ref = E.solve(prob, V, b, opts)
        x = torch.full_like(b, float("nan"))
        got = E.solve_noalloc(prob, V, b, opts, x=x)
        assert got.x.data_ptr() == x.data_ptr()
        assert np.array_equal(got.iters, ref.iters)
        assert np.array_equal(got.status, ref.status)
        assert np.array_equal(got.relres, ref.relres)
        assert got.ens_iters == ref.ens_iters
        assert torch.equal(got.x, ref.x)
        assert np.all(ref.status == 0)


def test_noalloc_rejects_oversized_requests():
    from paper_1705_02003_amd import _lib as L
    from paper_1705_02003_amd import ensemble as E
    prob = E.Problem(512, 4, 0, 0.4)
    S = 32                      # 512^2 x 32 member-rows: far beyond the array
    need = E.workspace_bytes(prob, S)
    assert need > L.NOALLOC_SCRATCH_BYTES
    V = E.empty_matrix(prob, 1)  # never read: the size check comes first
    b = torch.zeros((prob.rows, S), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    it = np.zeros(S, np.int32)
    st = np.zeros(S, np.int32)
    rr = np.zeros(S, np.float64)
    ei = C.c_int32(0)
    pc, oc = prob.c(), E.SolverOptions().c()
    rc = L.lib().ens_pcg_solve_noalloc(C.byref(pc), C.byref(oc), S, C.c_void_p(V.data_ptr()),
                                       C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                       it.ctypes.data_as(L.i32p), st.ctypes.data_as(L.i32p),
                                       rr.ctypes.data_as(L.f64p), C.byref(ei),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.ENS_ENOMEM
    assert torch.count_nonzero(x).item() == 0
