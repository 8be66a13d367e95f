"""Model problem: -div(a(x) K(y) grad u) = 1 on the unit square, u = 0 on the boundary.

Paper, Section 2.1, eq. (elliptic-SPDE): a linear elliptic SPDE with a
parameter-dependent diffusivity tensor; the paper's own instance is 3-D with
A = diag(a, a_y, a_z) (eq. diff-coeff).  This oracle implements the 2-D
rotated-anisotropy instance used by the workloads:

  K(y) = R(theta) diag(1, eps) R(theta)^T,
  eps  = 10^-(1 + y1)              (eps_model 0, eps >= 1e-2)
       = 10^-(1.5 + 1.5 y1)        (eps_model 1, eps >= 1e-3)
  theta = (pi/4)(1 + y2)
  a(x) = 1 + amp * sum_{k=1}^{d-2} y_{k+2} sin(k pi x1) sin(k pi x2) / k^2

Discretisation (the paper is silent here; it used trilinear FE): a
conservative, symmetric nine-point scheme on the (n+2)^2 node grid,
h = 1/(n+1), unknowns at interior nodes, row r = (j-1) n + (i-1) with x1
(index i) fastest.  Face means carry the diagonal terms, central differences
carry the mixed term:

  -d1(a k11 d1 u) - d2(a k22 d2 u) - D0_1(b D0_2 u) - D0_2(b D0_1 u),  b = k12 a.

Couplings to boundary nodes are dropped (zero Dirichlet data).  The matrix
stores A (the 1/h^2 is included); the right-hand side is f = 1.

Stencil slot order (shared with the HIP library only as a documented format,
not as code): slot = 3 (dj + 1) + (di + 1), i.e. SW, S, SE, W, C, E, NW, N, NE,
which is also the column order of a CSR row.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

SLOT_OFFSETS = [(di, dj) for dj in (-1, 0, 1) for di in (-1, 0, 1)]  # (di, dj)
CENTER = 4


def anisotropy(y, eps_model):
    """eps, theta and the tensor entries (k11, k22, k12) of R diag(1, eps) R^T."""
    y1, y2 = y[0], y[1]
    if eps_model == 0:
        eps = 10.0 ** (-(1.0 + y1))
    elif eps_model == 1:
        eps = 10.0 ** (-(1.5 + 1.5 * y1))
    else:
        raise ValueError("eps_model must be 0 or 1")
    theta = (np.pi / 4.0) * (1.0 + y2)
    c = np.cos(theta)
    s = np.sin(theta)
    k11 = c * c + eps * (s * s)
    k22 = s * s + eps * (c * c)
    k12 = (1.0 - eps) * (s * c)
    return eps, theta, k11, k22, k12


def node_coords(n):
    """x_i = i / (n + 1) for i = 0..n+1 (boundary nodes included)."""
    return np.arange(n + 2, dtype=np.float64) / float(n + 1)


def mode_table(n, n_modes):
    """sin(k pi x_i) for k = 1..n_modes, shape (n_modes, n+2)."""
    x = node_coords(n)
    return np.array([np.sin(k * np.pi * x) for k in range(1, n_modes + 1)])


def diffusivity(y, n, amp):
    """a at every node of the (n+2)^2 grid, indexed [j, i]; a = 1 on the boundary."""
    d = len(y)
    n_modes = d - 2
    a = np.ones((n + 2, n + 2), dtype=np.result_type(np.asarray(y), np.float64))
    if n_modes <= 0:
        return a
    tab = mode_table(n, n_modes)
    for k in range(1, n_modes + 1):
        s = tab[k - 1]
        a = a + amp * (y[k + 1] * np.outer(s, s) / float(k * k))
    return a


def stencil_values(y, n, eps_model, amp):
    """The nine stencil coefficients of A for every interior row, shape (9, n*n).

    Slot entries that couple to boundary nodes are zero (dropped couplings).
    """
    _, _, k11, k22, k12 = anisotropy(y, eps_model)
    a = diffusivity(y, n, amp)                     # [j, i], 0..n+1
    b = k12 * a
    I = slice(1, n + 1)
    Ip, Im = slice(2, n + 2), slice(0, n)
    aE = (a[I, I] + a[I, Ip]) / 2.0
    aW = (a[I, I] + a[I, Im]) / 2.0
    aN = (a[I, I] + a[Ip, I]) / 2.0
    aS = (a[I, I] + a[Im, I]) / 2.0
    bE, bW, bN, bS = b[I, Ip], b[I, Im], b[Ip, I], b[Im, I]
    h2 = np.zeros((9, n, n), dtype=aE.dtype)       # entries of h^2 A, [slot, j, i]
    h2[4] = k11 * (aE + aW) + k22 * (aN + aS)
    h2[5] = -k11 * aE
    h2[3] = -k11 * aW
    h2[7] = -k22 * aN
    h2[1] = -k22 * aS
    h2[8] = -(bE + bN) / 4.0
    h2[0] = -(bW + bS) / 4.0
    h2[6] = (bW + bN) / 4.0
    h2[2] = (bE + bS) / 4.0
    # drop couplings to boundary nodes
    h2[[0, 3, 6], :, 0] = 0.0
    h2[[2, 5, 8], :, n - 1] = 0.0
    h2[[0, 1, 2], 0, :] = 0.0
    h2[[6, 7, 8], n - 1, :] = 0.0
    inv_h2 = float((n + 1) * (n + 1))
    return (h2 * inv_h2).reshape(9, n * n)


def to_csr(vals, n):
    """CSR matrix from the (9, n*n) slot values; dropped couplings are absent."""
    rows, cols, data = [], [], []
    jj, ii = np.divmod(np.arange(n * n), n)
    for slot, (di, dj) in enumerate(SLOT_OFFSETS):
        ok = (ii + di >= 0) & (ii + di < n) & (jj + dj >= 0) & (jj + dj < n)
        r = np.nonzero(ok)[0]
        rows.append(r)
        cols.append(r + dj * n + di)
        data.append(vals[slot, r])
    A = sp.csr_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n * n, n * n))
    A.sort_indices()
    return A


def rhs(n):
    """f = 1 at every interior node."""
    return np.ones(n * n)


def assemble(y, n, eps_model, amp):
    """(A as CSR, b, diag(A)) for one sample."""
    vals = stencil_values(np.asarray(y), n, eps_model, amp)
    A = to_csr(vals, n)
    return A, rhs(n), vals[CENTER].copy()


def qoi_weights(n):
    """w with w_r = 1/|B| on the interior nodes of [0.4, 0.6]^2, else 0.

    A node index i (1-based) is inside when 0.4 <= i/(n+1) <= 0.6, decided in
    integers as 2(n+1) <= 5i <= 3(n+1), the same for j.  The QoI is the mean
    of u over those nodes (paper, Section 2.1, "Quantity of interest": a
    spatial average of u).
    """
    i = np.arange(1, n + 1)
    inside = (5 * i >= 2 * (n + 1)) & (5 * i <= 3 * (n + 1))
    mask = np.outer(inside, inside).reshape(-1)
    w = np.zeros(n * n)
    w[mask] = 1.0 / float(mask.sum())
    return w


def param_indicator(y, eps_model) -> float:
    """Section 3.2, eq. (pb-indicator): the supremum over the domain of
    lambda_max / lambda_min of a(x) K(y).  K = R diag(1, eps) R^T and a > 0
    scales both eigenvalues, so the ratio is 1 / eps at every x."""
    eps = anisotropy(np.asarray(y), eps_model)[0]
    return 1.0 / eps
