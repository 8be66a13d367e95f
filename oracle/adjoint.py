"""QoI, adjoint solve and the gradient dQ/dy = -lambda^T (dA/dy) u.

The paper's quantity of interest is a spatial mean of u (Section 2.1,
"Quantity of interest").  Here Q(y) = w^T u(y) with w the mean over the
interior nodes of [0.4, 0.6]^2.  Since A is symmetric and b does not depend on
y, dQ/dy_j = -lambda^T (dA/dy_j) u with A lambda = w.

lambda^T A u written as an energy form over faces and nodes of the
(n+2)^2 grid (lambda = u = 0 on boundary nodes), with D+ the forward
difference across a face and D0 the central difference at a node:

  h^2 lambda^T A u = sum_{x-faces} k11 a_f (D+ lambda)(D+ u)
                   + sum_{y-faces} k22 a_f (D+ lambda)(D+ u)
                   + sum_{nodes} (k12 a / 4) [(D0_1 lambda)(D0_2 u) + (D0_2 lambda)(D0_1 u)]

(D0 here is the undivided difference u_{+1} - u_{-1}).  Differentiating the
coefficients: d eps/d y1 = -c ln 10 eps (c = 1 or 1.5 by model),
d(k11, k22, k12)/d eps = (s^2, c^2, -s c), d theta/d y2 = pi/4,
d(k11, k22, k12)/d theta = (1 - eps)(-sin 2theta, sin 2theta, cos 2theta),
d a/d y_{k+2} = amp sin(k pi x1) sin(k pi x2) / k^2.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from . import problem


def _pad(v, n):
    """Interior vector (n*n) -> node field (n+2, n+2) with zero boundary, [j, i]."""
    F = np.zeros((n + 2, n + 2), dtype=v.dtype)
    F[1:n + 1, 1:n + 1] = v.reshape(n, n)
    return F


def energy_terms(lam, u, n):
    """The three face/node sums of h^2 lambda^T A u with unit coefficients.

    Returns (Ex, Ey, Em) where
      Ex[j, i] = (lam[j,i+1]-lam[j,i]) (u[j,i+1]-u[j,i])       x-face (i -> i+1), i = 0..n
      Ey[j, i] = (lam[j+1,i]-lam[j,i]) (u[j+1,i]-u[j,i])       y-face (j -> j+1), j = 0..n
      Em[j, i] = (D0_1 lam)(D0_2 u) + (D0_2 lam)(D0_1 u)       interior nodes
    so that h^2 lambda^T A u = sum k11 a_xface Ex + sum k22 a_yface Ey + sum (k12 a / 4) Em.
    """
    L, U = _pad(lam, n), _pad(u, n)
    Ex = (L[:, 1:] - L[:, :-1]) * (U[:, 1:] - U[:, :-1])          # (n+2, n+1)
    Ey = (L[1:, :] - L[:-1, :]) * (U[1:, :] - U[:-1, :])          # (n+1, n+2)
    I = slice(1, n + 1)
    d1L = L[I, 2:] - L[I, :-2]
    d2L = L[2:, I] - L[:-2, I]
    d1U = U[I, 2:] - U[I, :-2]
    d2U = U[2:, I] - U[:-2, I]
    Em = d1L * d2U + d2L * d1U                                     # (n, n)
    return Ex, Ey, Em


def bilinear(lam, u, y, n, eps_model, amp):
    """lambda^T A(y) u from the face/node form (independent of the CSR matrix)."""
    _, _, k11, k22, k12 = problem.anisotropy(y, eps_model)
    a = problem.diffusivity(y, n, amp)
    Ex, Ey, Em = energy_terms(lam, u, n)
    ax = (a[:, 1:] + a[:, :-1]) / 2.0
    ay = (a[1:, :] + a[:-1, :]) / 2.0
    I = slice(1, n + 1)
    tot = k11 * np.sum(ax * Ex) + k22 * np.sum(ay * Ey) + k12 * np.sum(a[I, I] * Em) / 4.0
    return tot * float((n + 1) ** 2)


def dA_bilinear(lam, u, y, n, eps_model, amp):
    """lambda^T (dA/dy_j) u for j = 0..d-1 (vector of length d)."""
    d = len(y)
    eps, theta, k11, k22, k12 = problem.anisotropy(y, eps_model)
    a = problem.diffusivity(y, n, amp)
    Ex, Ey, Em = energy_terms(lam, u, n)
    I = slice(1, n + 1)
    inv_h2 = float((n + 1) ** 2)

    def form(a_field, c11, c22, c12):
        ax = (a_field[:, 1:] + a_field[:, :-1]) / 2.0
        ay = (a_field[1:, :] + a_field[:-1, :]) / 2.0
        return (c11 * np.sum(ax * Ex) + c22 * np.sum(ay * Ey)
                + c12 * np.sum(a_field[I, I] * Em) / 4.0) * inv_h2

    c, s = math.cos(theta), math.sin(theta)
    g = np.zeros(d)
    deps = -(1.0 if eps_model == 0 else 1.5) * math.log(10.0) * eps
    g[0] = form(a, s * s * deps, c * c * deps, -s * c * deps)
    dth = math.pi / 4.0
    g[1] = form(a, -(1.0 - eps) * math.sin(2 * theta) * dth,
                (1.0 - eps) * math.sin(2 * theta) * dth,
                (1.0 - eps) * math.cos(2 * theta) * dth)
    if d > 2:
        tab = problem.mode_table(n, d - 2)
        for k in range(1, d - 1):
            da = amp * np.outer(tab[k - 1], tab[k - 1]) / float(k * k)
            g[k + 1] = form(da, k11, k22, k12)
    return g


def qoi_and_grad(y, n, eps_model, amp, solve=None):
    """(Q, dQ/dy, u, lambda) with direct sparse solves (exact to round-off)."""
    A, b, _ = problem.assemble(y, n, eps_model, amp)
    w = problem.qoi_weights(n)
    lu = spla.splu(A.tocsc())
    u = lu.solve(b)
    lam = lu.solve(w)
    Q = float(w @ u)
    g = -dA_bilinear(lam, u, y, n, eps_model, amp)
    return Q, g, u, lam


def qoi_complex_step(y, n, eps_model, amp, j, h=1e-30):
    """dQ/dy_j = Im Q(y + i h e_j) / h with a complex sparse direct solve."""
    yc = np.asarray(y, dtype=np.complex128).copy()
    yc[j] += 1j * h
    vals = problem.stencil_values(yc, n, eps_model, amp)
    A = problem.to_csr(vals, n)
    u = spla.splu(A.tocsc()).solve(problem.rhs(n).astype(np.complex128))
    return float(np.imag(problem.qoi_weights(n) @ u)) / h


def qoi_direct(y, n, eps_model, amp):
    A, b, _ = problem.assemble(y, n, eps_model, amp)
    u = spla.splu(A.tocsc()).solve(b)
    return float(problem.qoi_weights(n) @ u)
