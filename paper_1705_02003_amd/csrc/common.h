// Internal definitions shared by the HIP translation units of libens.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ens.h"

namespace ens {

constexpr int kNT = 256;          // threads per workgroup (4 wave64s)
constexpr int kWaves = kNT / 64;
constexpr int kFinNT = 256;       // threads of a one-workgroup finishing kernel
constexpr int kMaxS = 64;
constexpr int kMaxGroups = 2048;  // cap on workgroups of reducing kernels
constexpr int kRing = 2 * kNT + 2 * kMaxS;  // doubles per LDS ring line (tile + halo)
constexpr int kMaxCheb = 8;       // maximum Chebyshev degree
constexpr int kChebCoef = 2 * kMaxCheb + 2;

// control words (int32) in the workspace
enum Ctl : int {
  CTL_DONE = 0,   // 1 when no member is active
  CTL_K = 1,      // completed iterations
  CTL_MAXIT = 6,  // iteration cap (copied from the options)
  CTL_COUNT = 16
};

// Per-member state of one ensemble solve (device arrays of length S).
struct Members {
  double* rho;         // r^T z
  double* alpha;       // step of the current iteration (0 if inactive)
  double* alpha_prev;  // step still to be applied to x (deferred update)
  double* beta;        // direction update coefficient (0 if inactive)
  double* bnorm;       // ||b||
  double* relres;      // ||r|| / ||b|| of the latest residual
  double* lmax;        // Gershgorin bound of D^-1 A
  double* cheb;        // [S][kChebCoef] Chebyshev coefficients
  double* result;      // [S][16] scratch results of member reductions
  int* active;
  int* iters;
  int* status;
  int* ctl;            // control words
};

struct Workspace {
  double* y;      // [S][d] parameters staged from the host (kMaxS * 16 doubles)
  double* p[2];   // search directions (ping-pong)
  double* q;      // A p
  double* r;      // residual
  double* z[2];   // preconditioned residual (Chebyshev ping-pong)
  double* aux;    // one extra vector (adjoint right-hand side)
  double* partial;  // [3][kMaxGroups][S]
  Members m;
};

// Member lanes.  A grid point's S members are contiguous (row stride S, any
// S in [1, 64]); VEC = 2 members per thread when S is even, else 1.  The
// threads of one point form a power-of-two group of tpp lanes, so a point
// has Sp = tpp * VEC >= S member slots; slots s >= S are idle lanes that load
// a valid address, compute, and neither store nor add to any sum.  Partial
// sums and per-member state are indexed by slot (stride Sp).
struct Geometry {
  int n, S, Sp, vec, tpp;    // tpp: threads per grid point of the flat kernels
  int sw, swp, nstile, stpp; // member tile: sw members per stencil tile (the last
                             // may hold fewer), swp = stpp * vec slots, ceil(S / sw) tiles
  int tx, ty;                // tile: points per line chunk, lines per band
  int nchunk, nband, ntiles, groups;   // ntiles counts spatial tiles (per member tile)
  size_t nr, nelem;          // rows, rows * S
  size_t vstride;            // elements from one matrix slot to the next (slot_stride)
  int full;                  // 1: the sweep reads all nine matrix values per row
  int dim;                   // 2: nine-point grid n x n; 3: 27-point grid n x n x n
  int nslot, cslot;          // matrix slots per row and the diagonal's slot
  int np;                    // 3-D product: x-neighbouring points per thread (1 or 2)
};


// ------------------------------------------------------------ kernel args
// Assembly takes the parameters by value, kAsmY doubles per launch (the
// members m0 .. m0 + mc - 1 of the ensemble), so the caller's host array is
// copied at launch and no device buffer is needed; a wide ensemble with
// many parameters is assembled in several launches.
constexpr int kAsmY = 128;
constexpr int kAsmTX = 32, kAsmTY = 8;   // grid points per assembly tile (x, y)
constexpr int kMaxModes = 14;            // sine modes of a(x): d - 2 <= 14

struct AsmArgs {
  double y[kAsmY];  // [mc][d]: members m0 .. m0 + mc - 1
  double* V;        // [9][vstride], slot k holds [N_r][S]
  double* b;        // [N_r][S]
  int n, S, d, eps_model;
  int m0, mc, mcp;  // first member, members, threads per point (power of two >= mc)
  int ntx;          // tiles per grid line
  double amp;
  size_t vstride;
};

// M_CHEB1: the residual update r -= alpha q fused with the first Chebyshev
// step (the ring holds z_0 = D^-1 r / theta formed from r, q and the
// diagonal; r is written to a second buffer, since neighbouring tiles still
// read the old one).  M_RESID (3-D): q = r - A src, and with cheb_init the
// smoother start zout = D^-1 q / theta.  M_CHEBX (3-D): the Chebyshev step
// of a multigrid post-smoother, its result added to the level's x in place
// (x += src + d, d = c1 src + c2 D^-1 (r - A src); nothing else stored),
// with dotv the partial sums of dotv^T x.
enum Mode { M_SPMV = 0, M_PCG_J = 1, M_PCG_Z = 2, M_CHEB = 3, M_CHEB1 = 4, M_RESID = 5, M_CHEBX = 6 };

struct StencilArgs {
  const double* V;
  const double* r;
  const double* src;   // ring source: p (SPMV), z (PCG_Z direction source, CHEB)
  const double* pold;  // previous direction (PCG)
  double* pnew;        // new direction (PCG)
  double* q;           // A p (PCG, SPMV)
  double* x;           // solution, deferred update (PCG)
  double* zout;        // Chebyshev output z
  const double* zprev; // Chebyshev step k >= 3: z_{k-2}, read at the own point (may be zout)
  const double* q_in;  // M_CHEB1: A p of the current step
  double* r_out;       // M_CHEB1: the updated residual
  double* partial;     // [groups][Sp]; M_CHEB1: [2][groups][Sp] (r^T z on a last step, r^T r)
  Members m;
  Geometry g;
  int cheb_step;       // Chebyshev step 1..deg-1
  int cheb_last;       // 1 on the final step of a preconditioner application
  int cheb_init;       // 1 when the application yields the initial rho
  const double* dotv;  // M_CHEBX: partial sums of dotv^T x (none if null)
};

struct UpdateArgs {
  const double* V;
  double* r;
  const double* q;
  double* z;        // Chebyshev: z_0 = D^-1 r / theta
  double* partial;  // [2][groups][Sp]: r^T z (Jacobi), r^T r
  Members m;
  Geometry g;
  double rtol;
};

struct InitArgs {
  const double* V;
  const double* b;
  int b_broadcast;   // b is one vector [N_r] shared by all members
  double* x;
  double* p0;
  double* r;
  double* partial;   // [3][groups][Sp]: r^T z, b^T b, Gershgorin max
  Members m;
  Geometry g;
  int max_iter;
  int cheb;          // 1: Chebyshev preconditioner (Gershgorin bound, coefficients)
  int cheb_degree;
  double cheb_ratio;
};

struct DqdyArgs {
  const double* y;   // [S][d]
  const double* u;   // [N_r][S]
  const double* lam; // [N_r][S]
  double* partial;   // [d][groups][Sp]
  Geometry g;
  int d, eps_model;
  int ntx, ntiles;   // assembly-shaped tiles (kAsmTX x kAsmTY points)
  double amp;
};

enum Finish { F_ALPHA = 0, F_UPDATE_J = 1, F_UPDATE_C = 2, F_CHEB = 3, F_INIT = 4, F_DOT = 5, F_SUMS = 6,
              F_MAX = 7 };

struct FinishArgs {
  const double* partial;  // consecutive arrays of G * Sp partials
  int G;                  // workgroups of the producer kernel
  int kind;               // Finish
  Members m;
  Geometry g;
  double rtol;
  int cheb;               // F_INIT: Chebyshev (Gershgorin bound, coefficients)
  int cheb_init;          // F_CHEB: the application that yields the initial rho
  int cheb_degree;
  double cheb_ratio;
  int max_iter;
  int nsum;               // F_DOT / F_SUMS: number of partial arrays
  double scale;           // F_DOT / F_SUMS: factor applied to each sum
};

// ------------------------------------------------------------ launchers
void launch_assemble(const AsmArgs& a, hipStream_t s);
template <int MODE>
void launch_stencil(const StencilArgs& a, hipStream_t s);
void launch_update(const UpdateArgs& a, bool cheb, int groups, hipStream_t s);
void launch_init(const InitArgs& a, int groups, hipStream_t s);
void launch_cheb_start(const double* V, const double* r, double* z, const Members& m,
                       const Geometry& g, int groups, hipStream_t s);
void launch_final(double* x, const double* p0, const double* p1, const Members& m,
                  const Geometry& g, int groups, hipStream_t s);
void launch_triad(const double* a, const double* b, double* c, double s, size_t n, hipStream_t st);
int launch_stream_mix(const double* src, double* dst, size_t stride, size_t n, int nread, int nwrite,
                      hipStream_t st);
void launch_dot(const double* x, const double* y, int y_bcast, double* partial, const Geometry& g,
                int groups, hipStream_t s);
void launch_finish(const FinishArgs& a, hipStream_t s);
void launch_dqdy(const DqdyArgs& a, int groups, hipStream_t s);

size_t workspace_bytes(size_t nr, int S, bool cheb);
Workspace carve_workspace(void* base, size_t nr, int S, bool cheb);
int init_groups(const Geometry& g);   // workgroups of the element-wise kernels
Geometry make_geometry(int n, int S, int tile_lines, int max_groups, int member_tile = 0);
Geometry make_geometry3(int m, int S);

// the 3-D model's stencil step of every mode (fe3d.hip; launch_stencil
// forwards dim = 3 geometries to it); its other kernels are in fe3d.h
template <int MODE>
void launch_fe3d(const StencilArgs& a, hipStream_t s);
// Elements from the start of one matrix slot (or workspace vector) to the
// next: the slot's N_r * S elements plus 4 KiB.  Arrays that stream together
// must not sit a large power of two apart: at 2^28 bytes eleven such streams
// reach only about 80 % of the bandwidth they reach when offset by 4 KiB.
inline size_t slot_stride(size_t nelem) { return ((nelem + 31) & ~(size_t)31) + 512; }
int set_hip_error(hipError_t e);
int valid_S(int S);
inline int pow2ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

}  // namespace ens
