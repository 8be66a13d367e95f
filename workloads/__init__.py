"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds random draws and workload shapes only.  It contains none of
the method's arithmetic (no coefficients, no assembly, no solver, no sparse
grid): every quantity computed from a sample lives either in ``oracle/`` or in
the HIP library, which never import each other.

Sampling follows one fixed recipe: ``numpy.random.default_rng(seed)`` and
``uniform(-1, 1, (M, d))`` -- the parameter space of the model problem is the
hypercube [-1, 1]^d (paper, Section 4: Gamma = [-1, 1]^N).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

# Coefficient models: eps(y1) = 10^-(1 + y1) (down to 1e-2) or
# eps(y1) = 10^-(1.5 + 1.5 y1) (down to 1e-3); theta(y2) = (pi/4)(1 + y2).
EPS_MODEL_MILD = 0
EPS_MODEL_STRONG = 1

PRECOND_JACOBI = 0
PRECOND_CHEBYSHEV = 1


@dataclass(frozen=True)
class Workload:
    """Shape of one synthetic workload of the anisotropic-diffusion family."""

    name: str
    n: int                 # interior grid points per dimension (N_r = n*n rows)
    d: int                 # parameter dimension (y1: anisotropy, y2: angle, rest: modes)
    eps_model: int         # EPS_MODEL_MILD or EPS_MODEL_STRONG
    amp: float             # amplitude of the a(x) modes (0 when d == 2)
    S: Tuple[int, ...]     # ensemble widths exercised
    precond: int           # PRECOND_JACOBI or PRECOND_CHEBYSHEV
    rtol: float
    max_iter: int
    seed: int
    n_samples: int
    note: str = ""


# The five synthetic workloads.  They stand in for the paper's Section 4
# experiments (3-D trilinear FE with AMG on a CPU node), whose constants are
# not all stated; these are 2-D nine-point finite-difference instances of the
# same anisotropic diffusion family.
SMALL = Workload("small-64x64-d2", 64, 2, EPS_MODEL_MILD, 0.0, (8,),
                 PRECOND_JACOBI, 1e-8, 5000, 0, 32,
                 "32 uniform samples grouped by a sparse-grid iteration surrogate")
ADAPTIVE_512 = Workload("adaptive-sg-512x512-d4", 512, 4, EPS_MODEL_MILD, 0.4,
                        (16, 32), PRECOND_JACOBI, 1e-8, 20000, 1, 1024,
                        "1024 adaptive sparse-grid nodes, levels 1-5")
CHEB_1024 = Workload("uniform-1024x1024-d8-cheb4", 1024, 8, EPS_MODEL_STRONG, 0.45,
                     (32, 64), PRECOND_CHEBYSHEV, 1e-8, 20000, 2, 4096,
                     "4096 uniform samples, degree-4 Jacobi-Chebyshev")
BATCHED = Workload("batched-64-ensembles-d8", 0, 8, EPS_MODEL_STRONG, 0.45,
                   (4, 8, 16, 32, 64), PRECOND_JACOBI, 1e-8, 20000, 3, 0,
                   "64 ensembles of mixed width and grid in one launch")
ADJOINT_512 = Workload("adjoint-512x512-d6", 512, 6, EPS_MODEL_MILD, 0.4, (32,),
                       PRECOND_JACOBI, 1e-8, 20000, 4, 512,
                       "QoI = mean of u over [0.4,0.6]^2, gradient by adjoint")

# The paper's own test problem (Section 4): 3-D, trilinear finite elements
# on 32^3 cells (n = 31 interior nodes per dimension), N = 4 parameters,
# solver tolerance 1e-7; 512 uniform samples grouped by a surrogate trained
# on the level-2 sparse grid.  eps_model and amp do not apply (0).
FE3D_32 = Workload("fe3d-32cube-d4", 31, 4, EPS_MODEL_MILD, 0.0, (32,),
                   PRECOND_CHEBYSHEV, 1e-7, 20000, 5, 512,
                   "3-D trilinear FE, log-normal KL diffusivity, Jacobi and Chebyshev-4")

# The paper's Test 2 (Section 4): the same problem with the discontinuous
# factor a_hat(y) in {1, 100, 10} banded by |y| (selected by eps_model 1 in
# the 3-D model).
FE3D_32_TEST2 = Workload("fe3d-32cube-d4-test2", 31, 4, 1, 0.0, (32,),
                         PRECOND_CHEBYSHEV, 1e-7, 20000, 5, 512,
                         "3-D trilinear FE, Test 2: a_hat(y) banded by |y|")

ALL = (SMALL, ADAPTIVE_512, CHEB_1024, BATCHED, ADJOINT_512, FE3D_32, FE3D_32_TEST2)


def uniform_samples(seed: int, M: int, d: int) -> np.ndarray:
    """M samples drawn uniformly from [-1, 1]^d, shape (M, d), float64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (M, d))


def random_permutations(seed: int, sizes: List[int]) -> List[np.ndarray]:
    """One permutation per level, drawn in level order from one generator.

    Used for the random-grouping comparator: level ``l`` gets
    ``rng.permutation(sizes[l])``.
    """
    rng = np.random.default_rng(seed)
    return [rng.permutation(m) for m in sizes]


@dataclass
class BatchedDraw:
    widths: List[int] = field(default_factory=list)
    grids: List[int] = field(default_factory=list)
    samples: List[np.ndarray] = field(default_factory=list)


def batched_draw(seed: int = 3, n_ens: int = 64,
                 widths=(4, 8, 16, 32, 64), grids=(256, 512, 1024),
                 d: int = 8) -> BatchedDraw:
    """Mixed-ensemble draw: widths first, then grids, then y per ensemble."""
    rng = np.random.default_rng(seed)
    w = [int(v) for v in rng.choice(np.asarray(widths), size=n_ens)]
    g = [int(v) for v in rng.choice(np.asarray(grids), size=n_ens)]
    ys = [rng.uniform(-1.0, 1.0, (s, d)) for s in w]
    return BatchedDraw(w, g, ys)


def identical_samples(y: np.ndarray, S: int) -> np.ndarray:
    """S copies of one sample (perfect grouping: every member does the same work)."""
    y = np.asarray(y, dtype=np.float64).reshape(1, -1)
    return np.repeat(y, S, axis=0)
