"""torch.autograd.Function for the ensemble QoI and its adjoint gradient.

Q_s(y_s) = w^T u_s with A(y_s) u_s = f and w the mean over the interior
nodes of [0.4, 0.6]^2 (3-D model: [0.4, 0.6]^3; the paper's QoI is a
spatial mean of u, Section 2.1).
Forward: ensemble assembly + ensemble PCG + per-member dot.  Backward: the
adjoint ensemble PCG A lambda = w (A is symmetric) on the same matrix values,
then dQ/dy_j = -lambda^T (dA/dy_j) u from the dQ/dy kernel.  All of it runs in
libens; this module only wires tensors.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import ensemble as E


class EnsembleQoI(torch.autograd.Function):
    """Q = EnsembleQoI.apply(y, problem, options) for y of shape (S, d)."""

    @staticmethod
    def forward(ctx, y: torch.Tensor, prob: E.Problem, opts: Optional[E.SolverOptions] = None):
        opts = opts or E.SolverOptions()
        y = y.detach().contiguous()
        V, b = E.assemble(prob, y)
        ws = E.workspace(prob, int(y.shape[0]), opts, y.device)
        res = E.solve(prob, V, b, opts, ws=ws)
        if np.any(res.status != 0):
            raise RuntimeError(f"forward solve did not converge: status {res.status.tolist()}")
        w = E.qoi_weights(prob.n, device=y.device, dim=prob.dim)
        Q = E.member_dot(res.x, w, ws=ws)
        ctx.save_for_backward(y)
        ctx.cache = (prob, opts, V, res.x, w, ws)
        ctx.forward_iters = res.iters
        return torch.tensor(Q, dtype=torch.float64, device=y.device)

    @staticmethod
    def backward(ctx, gQ: torch.Tensor):
        (y,) = ctx.saved_tensors
        prob, opts, V, u, w, ws = ctx.cache
        _, g, iters, status = E.adjoint_grad(prob, y, V, u, w, opts, ws=ws)
        if np.any(status != 0):
            raise RuntimeError(f"adjoint solve did not converge: status {status.tolist()}")
        ctx.adjoint_iters = iters
        grad = torch.tensor(g, dtype=torch.float64, device=y.device)
        return gQ.reshape(-1, 1).to(torch.float64) * grad, None, None


def qoi(prob: E.Problem, y: torch.Tensor, opts: Optional[E.SolverOptions] = None) -> np.ndarray:
    """Q per member without building a graph (used for finite differences)."""
    with torch.no_grad():
        return EnsembleQoI.apply(y, prob, opts).cpu().numpy()


def central_difference(prob: E.Problem, y: torch.Tensor, h: float = 1e-6,
                       opts: Optional[E.SolverOptions] = None) -> np.ndarray:
    """dQ/dy by central differences; each direction perturbs all S members at
    once, so the whole ensemble costs 2 d ensemble solves."""
    S, d = int(y.shape[0]), int(y.shape[1])
    g = np.zeros((S, d))
    for j in range(d):
        e = torch.zeros_like(y)
        e[:, j] = h
        g[:, j] = (qoi(prob, y + e, opts) - qoi(prob, y - e, opts)) / (2 * h)
    return g
