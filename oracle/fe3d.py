"""3-D model problem of the paper's numerical tests: trilinear finite elements.

Paper, Section 2.1, eqs. (elliptic-SPDE) and (diff-coeff): on D = [0, 1]^3,
-div(A(x, y) grad u) = f with u = 0 on the boundary and the anisotropic
diffusivity A = diag(a(x, y), a_y, a_z),

  a(x, y) = a_min + a_hat exp( sum_{n=1}^N sqrt(lambda_n) b_n(x) y_n ),

where (lambda_n, b_n) are the N largest eigenpairs of the covariance
cov(x, x') = sigma_0 exp(-||x - x'||_1 / delta).  Section 4: sigma_0 =
sqrt(300), delta = 1/4, 32^3 cells, trilinear elements, N = 4.

Readings (the paper leaves them open):
  * a_min = 0.1, a_y = a_z = 1; a_hat = 1 (Test 1), or Test 2's a_hat(y)
    (Section 4, Test 2 equation): 1 for r(y) < d/4, 100 for
    d/4 <= r(y) < d/2, 10 for r(y) >= d/2, with d = sqrt(3) and
    r(y) = ||y||_2 -- decided on r^2 = sum_i y_i^2 (products and sums each
    rounded, in index order) against the exact d^2/16 = 3/16 and
    d^2/4 = 3/4, so sparse-grid nodes on a band edge (dyadic coordinates,
    exact squares) fall as the inequalities say;
  * a is evaluated at each element's centroid and held constant on the
    element; the element matrices are then integrated exactly;
  * f = 1 (the load vector entry of an interior node is h^3);
  * the L1-norm covariance is a product of 1-D kernels exp(-|s - t| / delta),
    so its eigenpairs are products of 1-D ones; the 1-D pairs on [0, 1] are
    the classical closed forms for the exponential kernel (even: cos, odd:
    sin about the midpoint, frequencies from transcendental equations); the
    3-D terms are ordered by decreasing eigenvalue, ties by the 1-D mode
    indices (x, y, z) lexicographically, with each product formed over the
    three factors in ascending 1-D mode order so that ties are exact.

Unknowns: the m^3 interior nodes of the (m + 1)^3-cell mesh, h = 1 / (m + 1),
row r = (k m + j) m + i for node (i + 1, j + 1, k + 1), x fastest.  Stencil
slot of the neighbour at offset (di, dj, dk): 9 (dk + 1) + 3 (dj + 1) +
(di + 1), so 13 is the diagonal and slot order is column order.
"""
from __future__ import annotations

import itertools
import math
from typing import List, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.optimize import brentq

SIGMA0 = math.sqrt(300.0)
DELTA = 0.25
A_MIN, A_HAT, A_Y, A_Z = 0.1, 1.0, 1.0, 1.0
CENTER = 13
SLOT_OFFSETS = [(di, dj, dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)]


# ------------------------------------------------------------ KL modes
def kl_1d(count: int, delta: float = DELTA) -> List[Tuple[int, float, float, float]]:
    """The `count` largest eigenpairs of k(s, t) = exp(-|s - t| / delta) on
    [0, 1] as (kind, omega, lambda, norm): kind 0 is cos(omega (s - 1/2)),
    kind 1 is sin(omega (s - 1/2)), each times norm (unit L2 norm), with
    lambda = 2c / (omega^2 + c^2), c = 1 / delta.  With half-length a = 1/2 the
    even frequencies solve c cos(omega a) = omega sin(omega a) on
    (j pi, j pi + pi/2) / a and the odd ones solve omega cos(omega a) +
    c sin(omega a) = 0 on (j pi + pi/2, (j + 1) pi) / a."""
    c, a = 1.0 / delta, 0.5
    out = []
    for j in range(count):
        lo, hi = j * math.pi / a, (j * math.pi + math.pi / 2) / a
        w = brentq(lambda w: c * math.cos(w * a) - w * math.sin(w * a), lo + 1e-12, hi - 1e-12,
                   xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500)
        out.append((0, w, 2 * c / (w * w + c * c), 1.0 / math.sqrt(a + math.sin(2 * w * a) / (2 * w))))
        lo, hi = (j * math.pi + math.pi / 2) / a, (j + 1) * math.pi / a
        w = brentq(lambda w: w * math.cos(w * a) + c * math.sin(w * a), lo + 1e-12, hi - 1e-12,
                   xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500)
        out.append((1, w, 2 * c / (w * w + c * c), 1.0 / math.sqrt(a - math.sin(2 * w * a) / (2 * w))))
    out.sort(key=lambda t: -t[2])
    return out[:count]


def phi_1d(mode, s):
    kind, w, _, norm = mode
    return norm * (np.cos(w * (s - 0.5)) if kind == 0 else np.sin(w * (s - 0.5)))


def kl_3d(N: int):
    """The N largest 3-D terms: (sqrt(lambda), (p, q, r)) with
    lambda = sigma_0 lambda_p lambda_q lambda_r."""
    K = 8
    m1 = kl_1d(K)
    terms = []
    for p, q, r in itertools.product(range(K), repeat=3):
        a_, b_, c_ = sorted((p, q, r))
        lam = SIGMA0 * (m1[a_][2] * m1[b_][2] * m1[c_][2])
        terms.append((lam, (p, q, r)))
    terms.sort(key=lambda t: (-t[0], t[1]))
    return [(math.sqrt(lam), idx) for lam, idx in terms[:N]], m1


def a_hat(y, test: int = 1) -> float:
    """The factor a_hat of eq. (diff-coeff): 1 in Test 1; in Test 2 the
    banded value of the Test 2 equation by r(y) (the real part of a complex
    y: a_hat is piecewise constant, so its complex-step derivative is 0)."""
    if test == 1:
        return A_HAT
    r2 = 0.0
    for v in np.real(np.asarray(y)).tolist():
        r2 = r2 + v * v
    if r2 < 3.0 / 16.0:
        return 1.0
    if r2 < 3.0 / 4.0:
        return 100.0
    return 10.0


def element_coefficients(y, m: int, test: int = 1) -> np.ndarray:
    """a at the centroid of every cell, shape (m+1, m+1, m+1) indexed [ez, ey, ex]
    (complex y gives complex a, for complex-step derivatives); `test` 1 or 2
    selects a_hat."""
    ah = a_hat(y, test)
    y = np.asarray(y)
    if not np.iscomplexobj(y):
        y = y.astype(np.float64)
    terms, m1 = kl_3d(len(y))
    h = 1.0 / (m + 1)
    xc = (np.arange(m + 1) + 0.5) * h
    g = np.zeros((m + 1, m + 1, m + 1), dtype=y.dtype)
    for (sq, (p, q, r)), yn in zip(terms, y):
        bx, by, bz = phi_1d(m1[p], xc), phi_1d(m1[q], xc), phi_1d(m1[r], xc)
        g = g + sq * yn * (bz[:, None, None] * by[None, :, None] * bx[None, None, :])
    return A_MIN + ah * np.exp(g)


# ------------------------------------------------------------ assembly
def element_matrix(ae: float, ay: float, az: float, h: float) -> np.ndarray:
    """8 x 8 stiffness of diag(ae, ay, az) on one cube cell, exact: with the
    1-D linear-element stiffness K1 = [[1, -1], [-1, 1]] / h and mass
    M1 = [[2, 1], [1, 2]] h / 6, the cell matrix is
    ae Kx My Mz + ay Mx Ky Mz + az Mx My Kz (tensor products).  Local node
    (lx, ly, lz) in {0, 1}^3 has index lx + 2 ly + 4 lz."""
    K1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    Ke = np.zeros((8, 8), dtype=np.result_type(ae, ay, az, 1.0))
    for a_, b_ in itertools.product(range(8), repeat=2):
        ax, ay_, az_ = a_ & 1, (a_ >> 1) & 1, a_ >> 2
        bx, by, bz = b_ & 1, (b_ >> 1) & 1, b_ >> 2
        Ke[a_, b_] = (ae * K1[ax, bx] * M1[ay_, by] * M1[az_, bz]
                      + ay * M1[ax, bx] * K1[ay_, by] * M1[az_, bz]
                      + az * M1[ax, bx] * M1[ay_, by] * K1[az_, bz])
    return Ke


def assemble_from_cells(acell: np.ndarray, m: int, ay: float = A_Y, az: float = A_Z):
    """Global matrix (CSR, interior nodes only) from per-cell a values
    acell[ez, ey, ex]: every cell adds its matrix, cells taken in (ez, ey, ex)
    order with ex fastest, each entry summed in that order (so A[i, j] and
    A[j, i] are the same sum); rows and columns of boundary nodes are dropped
    (zero Dirichlet data)."""
    h = 1.0 / (m + 1)
    acc = {}

    def idx(i, j, k):   # mesh node -> unknown index, or -1 on the boundary
        if 1 <= i <= m and 1 <= j <= m and 1 <= k <= m:
            return ((k - 1) * m + (j - 1)) * m + (i - 1)
        return -1

    for ez, ey, ex in itertools.product(range(m + 1), repeat=3):
        Ke = element_matrix(acell[ez, ey, ex], ay, az, h)
        ids = [idx(ex + (l & 1), ey + ((l >> 1) & 1), ez + (l >> 2)) for l in range(8)]
        for a_, b_ in itertools.product(range(8), repeat=2):
            if ids[a_] >= 0 and ids[b_] >= 0:
                key = (ids[a_], ids[b_])
                acc[key] = acc[key] + Ke[a_, b_] if key in acc else Ke[a_, b_]
    N = m ** 3
    rows = np.array([k[0] for k in acc], dtype=np.int64)
    cols = np.array([k[1] for k in acc], dtype=np.int64)
    vals = np.array(list(acc.values()))
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N), dtype=vals.dtype)


def rhs(m: int) -> np.ndarray:
    """Load vector of f = 1: each interior hat integrates to h^3."""
    h = 1.0 / (m + 1)
    return np.full(m ** 3, h ** 3)


def assemble(y, m: int, test: int = 1):
    """(A as CSR, b, diag(A)) for one sample (Test 1 or Test 2 coefficient)."""
    A = assemble_from_cells(element_coefficients(y, m, test), m)
    return A, rhs(m), A.diagonal().copy()


def slot_values(A, m: int) -> np.ndarray:
    """The 27 stencil values of every row, [27][m^3] (0 where the neighbour
    is outside the grid)."""
    N = m ** 3
    out = np.zeros((27, N))
    C = A.tocoo()
    r, c = C.row, C.col
    di = c % m - r % m
    dj = (c // m) % m - (r // m) % m
    dk = c // (m * m) - r // (m * m)
    assert np.all(np.abs(di) <= 1) and np.all(np.abs(dj) <= 1) and np.all(np.abs(dk) <= 1)
    out[9 * (dk + 1) + 3 * (dj + 1) + (di + 1), r] = C.data
    return out


def param_indicator(y, m: int, test: int = 1) -> float:
    """Section 3.2, eq. (pb-indicator): the supremum over the domain of
    lambda_max / lambda_min of A = diag(a, a_y, a_z), a held on each cube."""
    ac = element_coefficients(y, m, test)
    hi = np.maximum(np.maximum(ac, A_Y), A_Z)
    lo = np.minimum(np.minimum(ac, A_Y), A_Z)
    return float(np.max(hi / lo))


# ------------------------------------------------------------ adjoint
def qoi_weights(m: int) -> np.ndarray:
    """w with w_r = 1/|B| on the interior nodes of [0.4, 0.6]^3, else 0; a
    node index i (1-based) is inside when 2(m+1) <= 5i <= 3(m+1), decided in
    integers, the same in every direction (Section 2.1: a spatial mean of u)."""
    i = np.arange(1, m + 1)
    inside = (5 * i >= 2 * (m + 1)) & (5 * i <= 3 * (m + 1))
    mask = (inside[:, None, None] & inside[None, :, None] & inside[None, None, :]).reshape(-1)
    w = np.zeros(m ** 3)
    w[mask] = 1.0 / float(mask.sum())
    return w


def dA_bilinear(lam, u, y, m: int, test: int = 1) -> np.ndarray:
    """lambda^T (dA/dy_j) u for j = 0..d-1.  Only a depends on y; on cube c,
    da_c/dy_j = a_hat exp(g_c) sqrt(lambda_j) b_j(x_c) = (a_c - a_min)
    sqrt(lambda_j) b_j(x_c), and the part of the cube matrix that a
    multiplies is Kx My Mz, so the form is the sum over cubes of that
    derivative times lambda_c^T (Kx My Mz) u_c (nodal values, 0 on the
    boundary)."""
    y = np.asarray(y, dtype=np.float64)
    terms, m1 = kl_3d(len(y))
    h = 1.0 / (m + 1)
    xc = (np.arange(m + 1) + 0.5) * h
    eg = element_coefficients(y, m, test) - A_MIN
    Kc = element_matrix(1.0, 0.0, 0.0, h)
    Lp = np.zeros((m + 2,) * 3)
    Up = np.zeros((m + 2,) * 3)
    Lp[1:-1, 1:-1, 1:-1] = np.asarray(lam).reshape(m, m, m)
    Up[1:-1, 1:-1, 1:-1] = np.asarray(u).reshape(m, m, m)
    # the eight local nodal values of every cube, local index lx + 2 ly + 4 lz
    loc = lambda P, l: P[(l >> 2):(l >> 2) + m + 1, ((l >> 1) & 1):((l >> 1) & 1) + m + 1, (l & 1):(l & 1) + m + 1]
    B = np.zeros((m + 1,) * 3)
    for a_, b_ in itertools.product(range(8), repeat=2):
        B = B + loc(Lp, a_) * Kc[a_, b_] * loc(Up, b_)
    out = np.zeros(len(y))
    for j, (sq, (p, q, r)) in enumerate(terms):
        bj = phi_1d(m1[r], xc)[:, None, None] * phi_1d(m1[q], xc)[None, :, None] * phi_1d(m1[p], xc)[None, None, :]
        out[j] = float(np.sum(eg * sq * bj * B))
    return out


def qoi_and_grad(y, m: int, test: int = 1):
    """(Q, dQ/dy, u, lambda) with direct sparse solves (exact to round-off)."""
    A, b, _ = assemble(y, m, test)
    w = qoi_weights(m)
    lu = spla.splu(A.tocsc())
    u = lu.solve(b)
    lam = lu.solve(w)
    return float(w @ u), -dA_bilinear(lam, u, y, m, test), u, lam


def qoi_complex_step(y, m: int, j: int, h: float = 1e-30, test: int = 1) -> float:
    """dQ/dy_j = Im Q(y + i h e_j) / h with a complex sparse direct solve."""
    yc = np.asarray(y, dtype=np.complex128).copy()
    yc[j] += 1j * h
    A = assemble_from_cells(element_coefficients(yc, m, test), m)
    u = spla.splu(A.tocsc()).solve(rhs(m).astype(np.complex128))
    return float(np.imag(qoi_weights(m) @ u)) / h
