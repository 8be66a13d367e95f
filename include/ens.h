/*
 * ens.h -- C ABI of the MI355X ensemble-PCG library (libens.so).
 *
 * The library solves S discretised anisotropic-diffusion systems L_m U_m = F_m
 * at once.  All members share one sparsity pattern (a nine-point stencil on
 * an n x n grid of interior points); each member has its own matrix values.
 * Paper: Section 2.3, eqs. (discrete-sys), (discrete-ensemble-sys) and
 * (discrete-comm-kron-sys); the ensemble matrix stores each nonzero as a
 * length-S array, and inner products and norms are computed per member so
 * that each member converges at its own rate (Section 2.3, last paragraphs;
 * Section 4, the paragraphs on the convergence test and on the A-norm guard).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Real data are IEEE double (FP64); counts and indices are int32_t.
 *  - N_r = n * n rows; row r = j * n + i with i (x1 direction) fastest,
 *    i, j in [0, n).
 *  - Ensemble layout (member index innermost, the commuted Kronecker ordering
 *    of eq. (discrete-comm-kron-sys)):
 *        vector X      : X[r * S + s]                      ([N_r][S])
 *        matrix values : V[k * L + r * S + s]              ([9][L], L >= N_r S)
 *    with L = ens_matrix_slot_stride(prob, S): each slot holds its N_r * S
 *    values at its start and is followed by a few KiB of padding, so that
 *    the nine slots do not sit a large power of two apart (they stream
 *    together; see ens_matrix_slot_stride).  A V buffer has 9 * L doubles.
 *    Stencil slot k = 3 (dj + 1) + (di + 1) couples row (i, j) to column
 *    (i + di, j + dj): k = 0 SW, 1 S, 2 SE, 3 W, 4 C (diagonal), 5 E, 6 NW,
 *    7 N, 8 NE -- the column order of a CSR row.  Slots that would couple to
 *    a boundary node hold 0 (zero Dirichlet data).
 *  - Any ensemble width 1 <= S <= 64 (the paper's typical widths are 4 to
 *    32, Section 2.3; its Table 1 uses 20).  Inside the kernels a point's
 *    members are handled by a power-of-two group of lanes, so a width that
 *    is not a power of two leaves some lanes idle but moves only the S
 *    members' bytes.  (The batched solver, ens_batch_solve, takes widths
 *    that are powers of two, at least 2.)
 *  - "_dev" pointers are device memory of the current HIP device, "_host"
 *    pointers are host memory.  The caller owns every buffer; the library
 *    allocates no device memory, keeps no pointer after a call returns, and
 *    holds no state between calls.  Device buffers must be 16-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *    Device work is enqueued on that stream.  Calls documented as blocking
 *    synchronise that stream before returning.
 *  - Every entry point returns ENS_OK (0) or a negative error code.  Arguments
 *    are validated before any work is enqueued; on error nothing is written.
 *    ENS_EHIP means a HIP call failed; ens_last_hip_error() returns its code.
 *    A member that does not converge is NOT an error: see the status codes.
 */
#ifndef ENS_H
#define ENS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define ENS_OK 0
#define ENS_EINVAL (-1)   /* bad argument (size, pointer, non-finite parameter) */
#define ENS_ENOMEM (-2)   /* caller's workspace smaller than required            */
#define ENS_EHIP (-3)     /* a HIP runtime call failed                           */
#define ENS_ENOTSUP (-4)  /* valid but unsupported combination                   */

/* per-member solver status */
#define ENS_CONVERGED 0   /* ||r_k||_2 <= rtol ||b||_2 reached; iters = k          */
#define ENS_MAX_ITER 1    /* max_iter reached without convergence                 */
#define ENS_BREAKDOWN 2   /* p^T A p not a positive finite number: update replaced
                             by zero and the member frozen (the paper's guard)     */
#define ENS_ZERO_RHS 3    /* b = 0: x = 0, iters = 0                               */

#define ENS_PRECOND_JACOBI 0
#define ENS_PRECOND_CHEBYSHEV 1
#define ENS_PRECOND_MULTIGRID 2   /* 3-D model, n + 1 a power of two (ENS_ENOTSUP otherwise) */

/* Problem descriptor.
 *
 * dim = 0 or 2 (the 2-D model): -div(a(x) K(y) grad u) = f on the unit
 * square, u = 0 on the boundary, discretised by the conservative nine-point
 * scheme.
 *   K = R(theta) diag(1, eps) R(theta)^T,  theta = (pi/4)(1 + y1'),
 *   eps = 10^-(1 + y0')            (eps_model 0)
 *       = 10^-(1.5 + 1.5 y0')      (eps_model 1)
 *   a(x) = 1 + amp * sum_{k=1}^{d-2} y'_{k+1} sin(k pi x1) sin(k pi x2) / k^2
 * where y' = (y'_0 .. y'_{d-1}) is one member's parameter vector (0-based).
 * N_r = n^2 rows, nine matrix slots (SW, S, SE, W, C, E, NW, N, NE).
 *
 * dim = 3 (the paper's test problem, Section 2.1, eqs. (elliptic-SPDE) and
 * (diff-coeff), Section 4): -div(diag(a, a_y, a_z) grad u) = 1 on the unit
 * cube, u = 0 on the boundary, trilinear finite elements on (n+1)^3 cubes,
 *   a(x, y) = a_min + a_hat exp(sum_{k<d} sqrt(lambda_k) b_k(x) y'_k),
 * (lambda_k, b_k) the d largest eigenpairs of the covariance
 * sigma_0 exp(-|x - x'|_1 / delta), sigma_0 = sqrt(300), delta = 1/4, with
 * a_min = 0.1, a_y = a_z = 1; a is taken at each cube's centre.  a_hat:
 * eps_model 0 = the paper's Test 1, a_hat = 1; eps_model 1 = its Test 2
 * (Section 4, Test 2 equation), a_hat(y') = 1, 100 or 10 as |y'|_2 lies
 * below sqrt(3)/4, in [sqrt(3)/4, sqrt(3)/2), or at or above sqrt(3)/2,
 * decided on sum_k y'_k^2 (rounded products and sums, in index order)
 * against 3/16 and 3/4.
 * The eigenpairs are products of 1-D ones (cos / sin about 1/2, frequencies
 * from the exponential kernel's transcendental equations), ordered by
 * decreasing lambda, ties by their 1-D mode indices (x, y, z).
 * N_r = n^3 rows (x fastest), 27 matrix slots 9 (dz+1) + 3 (dy+1) + (dx+1)
 * (13 = diagonal); eps_model 0 or 1 (the a_hat above), amp 0, 1 <= d <= 16.
 * The batched solver takes the 2-D model only. */
typedef struct {
  int32_t n;          /* interior points per dimension, 2 <= n            */
  int32_t d;          /* parameters per member, 2 <= d <= 16 (3-D: 1..16) */
  int32_t eps_model;  /* 0 or 1 (3-D: 0 Test 1, 1 Test 2)                  */
  int32_t dim;        /* 0 or 2: the 2-D model; 3: the 3-D model          */
  double amp;         /* amplitude of the a(x) modes (finite, |amp| < 1; 3-D: 0) */
} ens_problem;

/* Solver options.  Zero-initialise, then set what you need; fields left 0
 * take the documented default. */
typedef struct {
  int32_t precond;      /* ENS_PRECOND_JACOBI (default), _CHEBYSHEV, _MULTIGRID */
  int32_t cheb_degree;  /* Chebyshev residual-polynomial degree, 2..8 (4)     */
  double cheb_ratio;    /* lambda_max / lambda_min of the Chebyshev interval (30) */
  double rtol;          /* relative residual tolerance (1e-8)                 */
  int32_t max_iter;     /* iteration cap (20000)                              */
  int32_t poll_every;   /* iterations between the host's checks of the device
                           done flag; 0 = adaptive: 16, or for an ensemble of
                           at least 2^19 member-rows the largest power of two
                           <= sqrt(iterations so far), between 4 and 16 (a
                           solve overruns its last iteration by up to two
                           such intervals of early-exit launches)            */
  int32_t tile_lines;   /* stencil tile height in grid lines, 0 = heuristic   */
  int32_t max_groups;   /* workgroups of the stencil/update kernels, 0 = heuristic */
  int32_t flags;        /* ENS_FLAG_* bits below                              */
  int32_t member_tile;  /* members per stencil tile: a power of two (a wide
                           ensemble is swept in tiles of this many members,
                           the last tile holding the rest); 0 or >= S: S */
} ens_opts;

/* Time the fused SpMV kernel with HIP events (ens_stats.spmv_ms). */
#define ENS_FLAG_TIME_SPMV 1
/* Solves and Chebyshev applications: read all nine stored matrix values of
   every row.  By default they use the symmetry that CG requires of A and read
   only the centre, E, N, NE and NW values, taking W, S, SW, SE of row (i, j)
   from E(i-1, j), N(i, j-1), NE(i-1, j-1), NW(i+1, j-1); both give the same
   bits on the bitwise-symmetric matrices ens_assemble_ensemble writes.  The
   full read is kept for verification and for matrices stored otherwise.
   ens_spmv always reads all nine values.  3-D model: by default the 14
   values of slots 13..26 are read per row and slot s < 13 of row P is taken
   as slot 26 - s of the neighbour row P + offset(s); with the flag all 27. */
#define ENS_FLAG_FULL_STENCIL 2
/* Multigrid: run every level of the V-cycle with its own kernel launches.
   By default the coarse levels of at most 7^3 nodes run as one launch, one
   workgroup per member holding those levels in LDS; both give the same
   bits.  The per-level form is kept for verification. */
#define ENS_FLAG_MG_LEVELWISE 4

/* Optional statistics of one solve. */
typedef struct {
  int32_t ens_iters;          /* iterations the ensemble ran = max_i iters_i  */
  int32_t spmv_timed;         /* fused-SpMV launches timed with HIP events    */
  double spmv_ms;             /* their summed duration (ms)                   */
  int32_t spmv_groups;        /* workgroups per fused-SpMV launch             */
  int32_t tile_lines;         /* tile height used                             */
} ens_stats;

/* ------------------------------------------------------------ assembly */
/* Assemble the ensemble matrix and right-hand side for S members.
 * Paper: Section 2.3 (each nonzero stored as a length-S array; mesh and graph
 * are sample independent and shared: the tables of the a(x) modes at the grid
 * nodes are computed once per tile for all members).  y_host: [S][d]
 * parameters (host memory; read before the call returns -- they travel with
 * the kernel launches -- so the array may be reused at once).
 * Outputs V_dev [9][L] (A, with the 1/h^2 included; L the slot stride, the
 * padding is not written) and b_dev [N_r][S]
 * (f = 1).  3-D model: V_dev [27][L], the finite-element stiffness matrix
 * (each cube's matrix integrated exactly with a held at the cube's centre),
 * b = h^3 (the load of f = 1).  Asynchronous on `stream`.
 * Errors (before any device work): ENS_EINVAL for a NULL pointer, a
 * non-finite parameter value, n < 2, d outside [2,16], eps_model outside
 * {0,1}, S outside [1,64], or non-finite amp (3-D: the limits of the
 * descriptor above; n <= 1024). */
int ens_assemble_ensemble(const ens_problem* prob, int32_t S, const double* y_host,
                          double* V_dev, double* b_dev, void* stream);

/* Elements L from the start of one matrix slot to the next in every V_dev
 * argument: N_r * S rounded up to a multiple of 32, plus 512 (4 KiB).  When
 * N_r * S * 8 bytes is a large power of two, unpadded slots would stream at
 * about 80 % of the bandwidth of padded ones on MI355X.  0 if the arguments
 * are invalid. */
size_t ens_matrix_slot_stride(const ens_problem* prob, int32_t S);

/* ------------------------------------------------------------- solver */
/* Bytes of device workspace ens_pcg_solve / ens_adjoint_grad need, or 0 if
 * the arguments are invalid. */
size_t ens_pcg_workspace_bytes(const ens_problem* prob, const ens_opts* opts, int32_t S);

/* Ensemble preconditioned CG for A_s x_s = b_s, s = 0..S-1, x_0 = 0.
 * Paper: Section 2.3 (per-member inner products; the ensemble iterates until
 * every member has converged) and Section 4 (each member's own convergence
 * iteration is recorded; when p^T A p is numerically zero the member's update
 * is replaced by zero and its x stops changing).  Each member follows the
 * Hestenes-Stiefel PCG recurrence; a member that has converged is frozen (its
 * x and r no longer change) while the others continue.  Preconditioner:
 * Jacobi (diagonal = slot 4 of V; 3-D: slot 13) or a Chebyshev polynomial in
 * D^-1 A over [lambda_max / cheb_ratio, lambda_max], lambda_max the member's
 * Gershgorin bound max_i sum_j |a_ij| / a_ii, or (3-D model only) one
 * geometric multigrid V-cycle per application (see ens_mg_apply).  Both
 * models; the 3-D model ignores tile_lines and member_tile.
 * In:  V_dev [9][L] (3-D: [27][L]; symmetric positive definite per member),
 *      b_dev [N_r][S].
 * Out: x_dev [N_r][S] (overwritten); iters_host[S], status_host[S],
 *      relres_host[S] (= ||r|| / ||b|| of the recurrence residual at exit, 0
 *      for ENS_ZERO_RHS), *ens_iters_host = max_s iters_s; stats may be NULL.
 * ws_dev / ws_bytes: caller-owned workspace of at least
 * ens_pcg_workspace_bytes() bytes (ENS_ENOMEM otherwise).
 * Blocking: synchronises `stream` before returning. */
int ens_pcg_solve(const ens_problem* prob, const ens_opts* opts, int32_t S,
                  const double* V_dev, const double* b_dev, double* x_dev,
                  int32_t* iters_host, int32_t* status_host, double* relres_host,
                  int32_t* ens_iters_host, ens_stats* stats,
                  void* ws_dev, size_t ws_bytes, void* stream);

/* The solve of ens_pcg_solve, for callers that cannot allocate memory (code
 * under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results, but the workspace is the
 * library's own device array of ENS_NOALLOC_SCRATCH_BYTES bytes (one per
 * device, held until the process ends) and the call allocates nothing --
 * no device or pinned memory, no events: it checks the done flag by copying
 * it to the host and synchronising `stream` once per poll interval.
 * Arguments and outputs as ens_pcg_solve (without stats).
 * Errors: as ens_pcg_solve; ENS_ENOMEM when ens_pcg_workspace_bytes(prob,
 * opts, S) exceeds ENS_NOALLOC_SCRATCH_BYTES (Jacobi: up to about 1.5e6
 * member-rows N_r * S; Chebyshev: about 1.1e6; multigrid, whose coarse
 * levels add about 4.2 vectors: about 0.68e6, e.g. 31^3 nodes at S = 23).
 * Every call on one device uses that device's array and leaves its contents
 * behind (the solve clears what must start at zero): calls that overlap on
 * one device, from several threads or streams, race and give wrong results.
 * Blocking: synchronises `stream` before returning. */
#define ENS_NOALLOC_SCRATCH_BYTES (64u << 20)
int ens_pcg_solve_noalloc(const ens_problem* prob, const ens_opts* opts, int32_t S,
                          const double* V_dev, const double* b_dev, double* x_dev,
                          int32_t* iters_host, int32_t* status_host, double* relres_host,
                          int32_t* ens_iters_host, void* stream);

/* One ensemble matrix-vector product q = A p (the operation the solver's fused
 * kernel performs each iteration, without the fused updates).
 * In: V_dev [9][L] (3-D: [27][L]), p_dev [N_r][S]; out: q_dev [N_r][S].
 * Asynchronous. */
int ens_spmv(const ens_problem* prob, int32_t S, const double* V_dev,
             const double* p_dev, double* q_dev, void* stream);

/* Apply the Chebyshev preconditioner once: z = M^-1 r per member, with the
 * polynomial of ens_pcg_solve (degree opts->cheb_degree, ratio opts->cheb_ratio).
 * In: V_dev [9][L] (3-D: [27][L]), r_dev [N_r][S]; out: z_dev [N_r][S]; lmax_host[S] (may be NULL)
 * receives each member's Gershgorin bound.  Blocking (reads back lmax). */
int ens_cheb_apply(const ens_problem* prob, const ens_opts* opts, int32_t S,
                   const double* V_dev, const double* r_dev, double* z_dev,
                   double* lmax_host, void* ws_dev, size_t ws_bytes, void* stream);

/* Apply the multigrid preconditioner once: z = V(r) per member, one V-cycle
 * (paper, Section 4: CG preconditioned by a multigrid hierarchy with a
 * degree-2 Chebyshev smoother on every level and a direct solve on the
 * coarsest; here its geometric form on the 3-D model's structured mesh).
 * Levels: n interior nodes per direction (n + 1 = 2^k cells, k >= 2), then
 * (n - 1) / 2, ..., 1; prolongation P is trilinear interpolation, restriction
 * P^T, the coarse operators the Galerkin products P^T A P (formed per member
 * on the device, in the workspace).  Each level above the coarsest smooths
 * its correction equation A x = b from x = 0 with the degree-2 Chebyshev
 * polynomial in D^-1 A on [lambda_max / cheb_ratio, lambda_max] (lambda_max
 * the level's Gershgorin bound), restricts the residual, adds the
 * prolongated coarse correction and smooths the new residual with the same
 * polynomial; the one-node coarsest level is solved exactly.  The V-cycle is
 * symmetric positive definite, so it may precondition CG.
 * opts: cheb_ratio (30 by default); precond and cheb_degree are ignored.
 * In: V_dev [27][L] (3-D model; symmetric positive definite per member),
 *     r_dev [N_r][S]; out: z_dev [N_r][S]; lmax_host[S] (may be NULL)
 *     receives each member's fine-level Gershgorin bound.
 * ws_dev / ws_bytes: at least ens_pcg_workspace_bytes() bytes for
 * opts with precond = ENS_PRECOND_MULTIGRID (ENS_ENOMEM otherwise).
 * Errors: ENS_ENOTSUP for the 2-D model or n + 1 not a power of two.
 * Blocking (reads back lmax). */
int ens_mg_apply(const ens_problem* prob, const ens_opts* opts, int32_t S,
                 const double* V_dev, const double* r_dev, double* z_dev,
                 double* lmax_host, void* ws_dev, size_t ws_bytes, void* stream);

/* Per-member dot products out_host[s] = sum_r a[r][s] * b[r][s].  With
 * b_broadcast != 0, b_dev is a single vector [N_r] shared by all members.
 * The reduction order is fixed, independent of the member index.
 * Blocking.  Uses the first ens_pcg_workspace_bytes(...) bytes of ws. */
int ens_member_dot(int32_t N_r, int32_t S, const double* a_dev, const double* b_dev,
                   int32_t b_broadcast, double* out_host,
                   void* ws_dev, size_t ws_bytes, void* stream);

/* Parameter-based grouping indicator (paper, Section 3.2, eq.
 * (pb-indicator)): per member, H = the supremum over the domain of
 * lambda_max / lambda_min of the diffusion tensor.  2-D model: a(x) K(y) has
 * eigenvalues a and a eps, so H = 1 / eps(y'_0).  3-D model: diag(a, a_y,
 * a_z) with a held on each cube, so H = the largest max(a, a_y, a_z) /
 * min(a, a_y, a_z) over the cubes.  In: y_host [S][d] (host; copied into the
 * workspace).  Out: h_host [S].  Uses the first ens_pcg_workspace_bytes(...)
 * bytes of ws.  Blocking.  Errors: as ens_assemble_ensemble; ENS_ENOMEM for
 * a too-small workspace. */
int ens_param_indicator(const ens_problem* prob, int32_t S, const double* y_host,
                        double* h_host, void* ws_dev, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------- adjoint */
/* dQ/dy for Q_s = w^T u_s, with A_s u_s = b (A symmetric, b independent of y):
 *   solve A_s lambda_s = w by the same ensemble PCG, then
 *   dQ_s/dy_j = -lambda_s^T (dA_s/dy_j) u_s,
 * the bilinear form evaluated face by face and node by node from the
 * coefficient derivatives (not from a differentiated matrix).
 * In: y_host [S][d] (host; finite, else ENS_EINVAL; copied into the
 * workspace), V_dev (assembled for y), u_dev [N_r][S] (forward solution),
 * w_dev [N_r] (shared QoI weights, e.g. ens_qoi_weights).  Out: lambda_dev [N_r][S],
 * grad_host [S][d], iters_host[S], status_host[S] of the adjoint solve.
 * 3-D model: only a depends on y; on cube c, da_c/dy_j = a_hat exp(g_c)
 * sqrt(lambda_j) b_j(x_c), and the form is the sum over cubes of that
 * derivative times lambda_c^T (Kx My Mz) u_c.  Blocking. */
int ens_adjoint_grad(const ens_problem* prob, const ens_opts* opts, int32_t S,
                     const double* y_host, const double* V_dev, const double* u_dev,
                     const double* w_dev, double* lambda_dev, double* grad_host,
                     int32_t* iters_host, int32_t* status_host,
                     void* ws_dev, size_t ws_bytes, void* stream);

/* The weights of the quantity of interest Q = w^T u, the mean of u over the
 * interior nodes in the box [0.4, 0.6]^dim (paper, Section 2.1: the output of
 * interest is a spatial functional of the solution; the box mean is this
 * model's choice).  w_dev [N_r]: 1 / count at the nodes inside, 0 elsewhere;
 * node index i in [1, n] is inside when 2 (n + 1) <= 5 i <= 3 (n + 1), decided
 * in integers.  Asynchronous on `stream`.  Errors: as the problem descriptor;
 * ENS_EINVAL for a NULL pointer or when no node lies in the box (n = 2). */
int ens_qoi_weights(const ens_problem* prob, double* w_dev, void* stream);

/* The dQ/dy kernel alone: grad_host[s][j] = -lambda_s^T (dA_s/dy_j) u_s for
 * given u and lambda (both models); y_host [S][d] as in ens_adjoint_grad.
 * Blocking. */
int ens_dqdy(const ens_problem* prob, int32_t S, const double* y_host,
             const double* u_dev, const double* lambda_dev, double* grad_host,
             void* ws_dev, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------- batching */
/* One ensemble of a batch.  The caller assembles it (ens_assemble_ensemble)
 * and gives it its own ens_pcg_solve workspace (Jacobi layout). */
typedef struct {
  ens_problem prob;        /* grid size n (the coefficient model is not used here) */
  int32_t S;               /* ensemble width, a power of two in [2, 64]            */
  int32_t tile_lines;      /* stencil tile height, 0 = heuristic                   */
  const double* V_dev;     /* [9][L], L = ens_matrix_slot_stride(&prob, S)         */
  const double* b_dev;     /* [N_r][S]                                             */
  double* x_dev;           /* [N_r][S], overwritten                                */
  void* ws_dev;            /* >= ens_pcg_workspace_bytes(&prob, Jacobi, S) bytes   */
  size_t ws_bytes;
  int32_t* iters_host;     /* [S] out, may be NULL                                 */
  int32_t* status_host;    /* [S] out, may be NULL                                 */
  double* relres_host;     /* [S] out, may be NULL                                 */
  int32_t ens_iters;       /* out: max over members                                */
  int32_t member_tile;     /* members per stencil tile (power of two <= S), 0 = S  */
  double seconds;          /* out: device time from the batch start until this
                              ensemble's last member stopped                       */
} ens_batch_item;

/* Bytes of the batch workspace for n_items ensembles (descriptor table,
 * unit prefixes, retirement flags and clocks), 0 if n_items is invalid. */
size_t ens_batch_workspace_bytes(int32_t n_items);

/* Solve n_items ensembles of different width, grid and iteration count
 * together (Jacobi-PCG, the semantics of ens_pcg_solve for each).  One CG
 * step for all ensembles is a graph of four kernels (fused stencil, finish,
 * update, finish) whose stencil and update kernels stride over the work of
 * every unfinished ensemble; the graph is replayed until every ensemble has
 * retired.  Paper: Section 5 names ensembles of varying size as future work;
 * each ensemble here still runs max over its members iterations (eqs. (Rl),
 * (R)).  opts: Jacobi only (ENS_ENOTSUP otherwise); max_groups sets the grid
 * of the strided kernels (default 512, a multiple of 8).  Blocking.
 * Errors: ENS_EINVAL (bad item), ENS_ENOMEM (a workspace too small),
 * ENS_ENOTSUP (an item of the 3-D model). */
int ens_batch_solve(const ens_opts* opts, int32_t n_items, ens_batch_item* items,
                    void* batch_ws, size_t batch_ws_bytes, void* stream);

/* --------------------------------------------------- sparse grid (host) */
/* Nodes of the centre-rooted piecewise-linear hierarchy (paper, Section 2.2):
 * one (level, index) pair per dimension.  1-D coordinates:
 *   level 0: index 0 -> 0;  level 1: index 0 -> -1, index 1 -> +1;
 *   level l >= 2: index k in [0, 2^(l-1)) -> -1 + (2k+1) 2^(1-l).
 * node_level / node_index are [M][d] row-major.  All sparse-grid calls are
 * host-only, synchronous and deterministic; floating-point evaluation uses a
 * fixed order (nodes in canonical order: total level, then level vector, then
 * index vector, lexicographic; each term c, then multiplied by the 1-D hat
 * values for dimensions 0..d-1, then added), so results are bit-for-bit
 * reproducible. */

/* Surrogate-based grouping (paper, Section 3.1, eq. SGSiterations and the
 * rule after it): build the surrogate I^ of node_value (e.g. iteration
 * counts) over the M nodes by hierarchical surpluses, evaluate it at the
 * M_new samples y_new [M_new][d], order them by increasing (I^, sample id)
 * and cut the order into ensembles of S.  The last ensemble is padded by
 * repeating its last sample (Section 4, Test 1 footnote).  With M == 0 the
 * samples keep their generation order and pred_out is all zero.
 * Out: groups_out [ceil(M_new/S)][S] sample ids, pred_out [M_new].
 * Errors: ENS_EINVAL for bad sizes, a NULL pointer, an invalid node, a
 * duplicate node, or a non-finite value / sample outside [-1,1]. */
int ens_group_samples(int32_t d, int32_t M, const int32_t* node_level,
                      const int32_t* node_index, const double* node_value,
                      int32_t M_new, const double* y_new, int32_t S,
                      int32_t* groups_out, double* pred_out);

/* Hierarchical surpluses of node_value over the nodes (paper, Section 2.2,
 * eq. hierSGint): c_m = v_m - sum over nodes j of lower total level of
 * c_j psi_j(y_m).  Out: surplus_out [M] in input order. */
int ens_sg_surpluses(int32_t d, int32_t M, const int32_t* node_level,
                     const int32_t* node_index, const double* node_value,
                     double* surplus_out);

/* Mean of the sparse-grid interpolant of node_value under the uniform density
 * 2^-d on [-1,1]^d (paper, Section 2.1: the quantity of interest is the
 * expectation of G(y); Section 2.2: the interpolant sum_m c_m psi_m integrates
 * term by term).  A 1-D basis function of level l integrates to 1 (l = 0),
 * 1/4 (l = 1) or 2^-l (l >= 2) against the density 1/2; the sum runs over the
 * nodes in canonical order, each term c_m times the d weights in dimension
 * order.  Host only and synchronous.  Out: *mean_out.
 * Errors: ENS_EINVAL for M = 0, a NULL pointer, an invalid or duplicate node,
 * or a non-finite value. */
int ens_sg_expectation(int32_t d, int32_t M, const int32_t* node_level,
                       const int32_t* node_index, const double* node_value,
                       double* mean_out);

/* Ensembles of varying width (paper, Section 5: choose ensemble sizes by a
 * combinatorial optimisation from a per-size performance model and the cost
 * surrogate).  Input: pred [M], the predicted iteration count of each sample
 * (a prediction below 1 counts as 1); the allowed widths [n_widths]
 * (ascending, distinct, in [1, 64]: any ensemble width the solver takes) and
 * iter_seconds [n_widths], the time of one ensemble iteration at each width.
 * The samples are ordered by ascending (pred, id) and the order is cut into
 * consecutive groups; group g has a width w_g and holds 1..w_g real samples
 * (padded to w_g by repeating its last one) and costs
 * iter_seconds[w_g] * (its largest prediction).  The cut with the least total
 * cost is found exactly (dynamic programming over the order; ties keep the
 * smaller width, then the fewer samples in the last group).  Ordering first
 * loses nothing: exchanging samples between two groups so that the one with
 * the smaller maximum holds the smaller samples never raises a group's
 * maximum.  Host only and synchronous.
 * Out: order_out [M] sample ids; group_width_out, group_count_out [M]
 * (the first *n_groups_out entries are used; group g takes the next
 * group_count_out[g] ids of the order); *cost_out, the least total cost.
 * Errors: ENS_EINVAL for M < 1, a NULL pointer, a bad width list, a
 * non-positive or non-finite iter_seconds, or a non-finite prediction. */
int ens_group_variable(int32_t M, const double* pred, int32_t n_widths,
                       const int32_t* widths, const double* iter_seconds,
                       int32_t* order_out, int32_t* group_width_out,
                       int32_t* group_count_out, int32_t* n_groups_out,
                       double* cost_out);

/* Coordinates of nodes: y_out [M][d]. */
int ens_sg_coords(int32_t d, int32_t M, const int32_t* node_level,
                  const int32_t* node_index, double* y_out);

/* Classic surplus-based refinement (paper, Section 2.2, "Adaptivity"): every
 * node of total level `newest_level` whose |surplus| >= tau_rel * |value of
 * the centre node| contributes its children (one dimension at a time) that
 * are not yet in the grid.  If more candidates exist than budget - M, they are
 * taken in decreasing order of the largest |surplus| among their refined
 * parents, ties in canonical order.  The accepted nodes are written in
 * canonical order to new_level_out / new_index_out ([max_new][d]) and their
 * count to *n_new_out.  ENS_EINVAL if max_new is too small for the result. */
int ens_sg_refine(int32_t d, int32_t M, const int32_t* node_level,
                  const int32_t* node_index, const double* node_value,
                  int32_t newest_level, double tau_rel, int32_t budget,
                  int32_t max_new, int32_t* new_level_out, int32_t* new_index_out,
                  int32_t* n_new_out);

/* ------------------------------------------------------------- misc */
const char* ens_strerror(int code);
int ens_last_hip_error(void);   /* hipError_t of the last ENS_EHIP, 0 if none */
int ens_version(void);          /* library ABI version (major * 100 + minor)  */

/* ------------------------------------------------------- calibration */
/* STREAM triad c = a + scalar * b over n doubles (two reads and one write
 * per element): the achievable-HBM-bandwidth reference that the solver's
 * kernels are reported against beside the 8 TB/s peak.  Buffers are device
 * memory, 16-byte aligned, and must not overlap.  Asynchronous on `stream`.
 * Errors: ENS_EINVAL for a NULL or misaligned pointer, n = 0 or a
 * non-finite scalar. */
int ens_stream_triad(const double* a_dev, const double* b_dev, double* c_dev, double scalar,
                     size_t n, void* stream);

/* STREAM-style streaming with the read/write mix of a solver kernel: for
 * e < n, dst[w * stride + e] = sum_{k < nread} src[k * stride + e] for every
 * w < nwrite.  The arrays sit `stride` doubles apart (use a stride a few KiB
 * past n, as ens_matrix_slot_stride does, so the streams are not a large
 * power of two apart).  Supported (nread, nwrite): (8, 3) -- the fused
 * solver step's eight reads and three writes per member-row -- (3, 1),
 * (2, 1) and (1, 1).  Asynchronous on `stream`.  Errors: ENS_EINVAL for a
 * NULL or misaligned pointer, odd or zero n, or stride < n; ENS_ENOTSUP for
 * another mix. */
int ens_stream_mix(const double* src_dev, double* dst_dev, size_t stride, size_t n,
                   int32_t nread, int32_t nwrite, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ENS_H */
