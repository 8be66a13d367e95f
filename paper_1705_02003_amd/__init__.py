"""MI355X-native ensemble preconditioned CG for many anisotropic-diffusion
samples at once, with surrogate-based grouping of samples into ensembles.

Compute runs in libens.so (hand-written HIP kernels for gfx950 behind the C
ABI in include/ens.h).  Modules:

  ensemble  assemble / solve / spmv / cheb_apply / member_dot / dqdy /
            adjoint_grad on torch CUDA tensors
  grouping  sparse-grid surrogate, grouping, refinement and the cost ratio R
  autograd  EnsembleQoI, a torch.autograd.Function over forward + adjoint
  uq        the adaptive level loop (solve, surrogate, refine, group)
  build     compiles libens.so in-tree
"""
from ._lib import EnsError, lib  # noqa: F401

__all__ = ["EnsError", "lib"]
