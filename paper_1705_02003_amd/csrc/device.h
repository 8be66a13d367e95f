// Device code shared by the single-ensemble kernels (kernels.hip) and the
// batched kernels (batch.hip): vector loads, the fixed-tree member
// reductions, the fused tile sweep and the finish logic.
#pragma once

#include "common.h"

namespace ens {

typedef double d2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------ load/store
// Every buffer of this library is in global memory.  The helpers below
// access it through global-address-space pointers: a pointer loaded from
// memory (rather than passed as a kernel argument) is otherwise generic to
// the compiler, which then emits flat instructions, and flat loads also count
// against the LDS wait counter, so every LDS wait of the tile sweep would
// stall on them.
#define ENS_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const ENS_GLOBAL T*)p;
}

template <class T>
struct same_type {
  using type = T;
};

template <class T>
__device__ __forceinline__ void gstore(T* p, typename same_type<T>::type v) {
  *(ENS_GLOBAL T*)p = v;
}

template <int VEC>
__device__ __forceinline__ void ld(double (&v)[VEC], const double* p) {
  if constexpr (VEC == 2) {
    const d2 t = *(const ENS_GLOBAL d2*)p;
    v[0] = t.x;
    v[1] = t.y;
  } else {
    v[0] = *(const ENS_GLOBAL double*)p;
  }
}

// matrix values are streamed once per iteration: non-temporal loads keep the
// vectors' lines in the caches
template <int VEC>
__device__ __forceinline__ void ld_stream(double (&v)[VEC], const double* p) {
  if constexpr (VEC == 2) {
    const d2 t = __builtin_nontemporal_load((const ENS_GLOBAL d2*)p);
    v[0] = t.x;
    v[1] = t.y;
  } else {
    v[0] = __builtin_nontemporal_load((const ENS_GLOBAL double*)p);
  }
}

template <int VEC>
__device__ __forceinline__ void st(double* p, const double (&v)[VEC]) {
  if constexpr (VEC == 2) {
    d2 t;
    t.x = v[0];
    t.y = v[1];
    *(ENS_GLOBAL d2*)p = t;
  } else {
    *(ENS_GLOBAL double*)p = v[0];
  }
}

// ------------------------------------------------------------ reductions
// Sum v over the threads of the workgroup holding the same members (t % tpp
// equal).  Result for members (t % tpp) * VEC + c is left in v of threads
// t < tpp.  `lds` holds kWaves * 64 * VEC doubles.
template <int VEC>
__device__ __forceinline__ void group_reduce(double (&v)[VEC], int tpp, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = tpp; off < 64; off <<= 1)
#pragma unroll
    for (int c = 0; c < VEC; ++c) v[c] += __shfl_xor(v[c], off);
  __syncthreads();
  if (lane < tpp) {
#pragma unroll
    for (int c = 0; c < VEC; ++c) lds[(wave * 64 + lane) * VEC + c] = v[c];
  }
  __syncthreads();
  if ((int)threadIdx.x < tpp) {
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      double a = lds[threadIdx.x * VEC + c];
      for (int w = 1; w < kWaves; ++w) a += lds[(w * 64 + threadIdx.x) * VEC + c];
      v[c] = a;
    }
  }
}

template <int VEC>
__device__ __forceinline__ void group_max(double (&v)[VEC], int tpp, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = tpp; off < 64; off <<= 1)
#pragma unroll
    for (int c = 0; c < VEC; ++c) v[c] = fmax(v[c], __shfl_xor(v[c], off));
  __syncthreads();
  if (lane < tpp) {
#pragma unroll
    for (int c = 0; c < VEC; ++c) lds[(wave * 64 + lane) * VEC + c] = v[c];
  }
  __syncthreads();
  if ((int)threadIdx.x < tpp) {
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      double a = lds[threadIdx.x * VEC + c];
      for (int w = 1; w < kWaves; ++w) a = fmax(a, lds[(w * 64 + threadIdx.x) * VEC + c]);
      v[c] = a;
    }
  }
}

// write this workgroup's partial [Sp] (member slots s0 .. s0 + tpp VEC - 1,
// threads t < tpp); a finish kernel launched after this one reads them (the
// kernel boundary makes them visible across XCDs, so no in-kernel
// device-scope fence is needed)
template <int VEC>
__device__ __forceinline__ void put_partial(double* partial, int Sp, int tpp, const double (&v)[VEC],
                                            int s0 = 0) {
  if ((int)threadIdx.x < tpp) {
#pragma unroll
    for (int c = 0; c < VEC; ++c) partial[(size_t)blockIdx.x * Sp + s0 + threadIdx.x * VEC + c] = v[c];
  }
}

// Member sums of NARR partial arrays P[a][g][s] (s < S, S here the slot
// count Sp, a power of two) over the workgroups g < G, returned for slot
// s = threadIdx.x (t < S), in a block of kFinNT threads.  Thread t loads
// VEC members per row (16-byte loads when VEC = 2); the
// R = kFinNT * VEC / S row sets are k, k + R, k + 2R, ... with
// k = t / (S / VEC), summed in that order with up to 32 loads in flight,
// then a fixed halving tree over k.  The order does not depend on the
// member.  `lds` holds NARR * kFinNT * VEC doubles.
template <int VEC, int NARR>
__device__ __forceinline__ void final_sums(const double* const (&P)[NARR], int G, int S,
                                           double* lds, double (&out)[NARR]) {
  const int t = threadIdx.x;
  const int W = S / VEC, R = kFinNT / W;
  const int pr = t % W, k = t / W;
  const int col = pr * VEC;
  constexpr int B = 32 / NARR;
  double acc[NARR][VEC];
#pragma unroll
  for (int a = 0; a < NARR; ++a)
#pragma unroll
    for (int c = 0; c < VEC; ++c) acc[a][c] = 0.0;
  // rows k, k + R, k + 2R, ... in increasing order, B of them in flight;
  // rows past G contribute +0
  for (int g = k; g < G; g += B * R) {
    double v[NARR][B][VEC];
#pragma unroll
    for (int a = 0; a < NARR; ++a)
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if (g + u * R < G) {
          ld<VEC>(v[a][u], P[a] + (size_t)(g + u * R) * S + col);
        } else {
#pragma unroll
          for (int c = 0; c < VEC; ++c) v[a][u][c] = 0.0;
        }
      }
#pragma unroll
    for (int a = 0; a < NARR; ++a)
#pragma unroll
      for (int u = 0; u < B; ++u)
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[a][c] += v[a][u][c];
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NARR; ++a)
#pragma unroll
    for (int c = 0; c < VEC; ++c) lds[a * kFinNT * VEC + k * S + col + c] = acc[a][c];
  __syncthreads();
  for (int stride = (R / 2) * S; stride >= S; stride >>= 1) {
#pragma unroll
    for (int a = 0; a < NARR; ++a)
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        const int i = t * VEC + c;
        if (i < stride) lds[a * kFinNT * VEC + i] += lds[a * kFinNT * VEC + i + stride];
      }
    __syncthreads();
  }
  const int s = t & (S - 1);
#pragma unroll
  for (int a = 0; a < NARR; ++a) out[a] = lds[a * kFinNT * VEC + s];
}

template <int VEC>
__device__ __forceinline__ double final_sum(const double* partial, int G, int S, double* lds) {
  const double* const P[1] = {partial};
  double out[1];
  final_sums<VEC, 1>(P, G, S, lds, out);
  return out[0];
}

__device__ __forceinline__ double final_max(const double* partial, int G, int S, double* lds) {
  const int t = threadIdx.x, s = t & (S - 1), k = t / S, T = kFinNT / S;
  double acc = 0.0;
  for (int g = k; g < G; g += T) acc = fmax(acc, gload(&partial[(size_t)g * S + s]));
  __syncthreads();
  lds[t] = acc;
  __syncthreads();
  for (int stride = kFinNT / 2; stride >= S; stride >>= 1) {
    if (t < stride) lds[t] = fmax(lds[t], lds[t + stride]);
    __syncthreads();
  }
  return lds[s];
}

// ------------------------------------------------------------ tiles
// Tile range of this workgroup: the tiles are split into eight contiguous
// ranges, one per XCD (consecutive workgroup ids are dispatched round-robin
// over the eight XCDs), so neighbouring tiles -- whose halos overlap -- run
// on the same XCD and share its L2.
__device__ __forceinline__ void tile_range(const Geometry& g, int& first, int& step, int& end) {
  const int G = gridDim.x, b = blockIdx.x;
  if (G >= 8 && (G & 7) == 0) {
    const int x = b & 7, w = b >> 3;
    const int lo = (int)(((long long)x * g.ntiles) >> 3);
    const int hi = (int)(((long long)(x + 1) * g.ntiles) >> 3);
    first = lo + w;
    step = G >> 3;
    end = hi;
  } else {
    first = b;
    step = G;
    end = g.ntiles;
  }
}

// What one tile sweep reads and writes: one ensemble's buffers and geometry.
struct TileView {
  const double* V;
  const double* r;
  const double* src;
  const double* pold;
  double* pnew;
  double* q;
  double* x;
  double* zout;
  const double* zprev;  // M_CHEB from the third step on: z_{k-2} (may be zout)
  const double* q_in;   // M_CHEB1
  double* r_out;        // M_CHEB1
  int n, S;        // grid size, ensemble width (row stride of every vector)
  int sw, s0;      // members this tile covers: s0 .. s0 + sw - 1
  int swp;         // member slots per point (tpp * VEC >= sw): the LDS point stride
  int tpp;         // threads per grid point (a power of two)
  int tx, ty, nchunk;
  size_t nelem, vstride;   // elements per vector; from one matrix slot to the next
  int cheb_step, cheb_last;
};

// One tile of the fused sweep: tx grid points of one line chunk times ty
// lines.  The tile is swept line by line; the values the stencil reads
// (M_PCG_J: the new direction p = r / diag + beta p_old; M_PCG_Z: p = z +
// beta p_old; M_SPMV: p; M_CHEB: z) are formed once per point, including a
// one-point halo, into a four-line LDS ring, so each line needs one barrier
// (a ring slot is rewritten only after every thread has passed the barrier
// that follows its last reader).  Then, per point and member, the nine-point
// product is taken from the ring and the mode's fused updates follow:
//   M_PCG_*: store p and q = A p, accumulate p^T q, apply the deferred
//            x += alpha_prev p_old;
//   M_CHEB:  one Chebyshev step z_k = z_{k-1} + d_k with
//            d_k = c1 d_{k-1} + c2 D^-1 (r - A z_{k-1}), and on the last step
//            accumulate r^T z_k.  The increment is not stored: d_0 = z_0 is
//            the ring value itself, d_1 = z_1 - z_0 with z_0 = D^-1 r / theta
//            formed again from r and the diagonal the step reads anyway, and
//            from the third step on d_{k-1} = z_{k-1} - z_{k-2} with z_{k-2}
//            read at the own point (ZPREV; z_k may overwrite it in place).
//            `aprev` carries theta;
//   M_CHEB1: the residual update and the first Chebyshev step in one sweep:
//            the ring value is z_0 = (r - alpha q) / diag / theta, and per own
//            point r' = r - alpha q is stored (to r_out), r'^T r' accumulated,
//            d_1 = c1 z_0 + c2 D^-1 (r' - A z_0), z_1 = z_0 + d_1 stored (and
//            r'^T z_1 accumulated into acc2 when it is the last step).
//            `beta` carries alpha of active members (else 0), `aprev` theta.
//
// SYM: the matrix is symmetric, so only C, E, N, NE, NW are read; the lower
// coefficients of row (i, j) are W = E(i-1, j), S = N(i, j-1), SW = NE(i-1,
// j-1) and SE = NW(i+1, j-1).  Each thread keeps N, NE, NW of its point's
// previous line in registers; E of the current line and NE, NW of the
// previous line are exchanged through `sym` (LDS, 2 x 3 lines of kRing
// doubles).  The products are formed in the same order as the nine-value
// sweep, so on a bitwise-symmetric matrix both give the same bits.
template <int VEC, int MODE, bool SYM, bool ZPREV = false>
__device__ __forceinline__ void stencil_tile(const TileView& a, int tile, double (*ring)[kRing],
                                             double* sym,
                                             const double (&beta)[VEC], const double (&aprev)[VEC],
                                             const double (&c1)[VEC], const double (&c2)[VEC],
                                             double (&acc)[VEC], double (&acc2)[VEC]) {
  constexpr bool PCG = (MODE == M_PCG_J || MODE == M_PCG_Z);
  constexpr bool DIAG_IN_RING = (MODE == M_PCG_J || MODE == M_CHEB1);   // diagonal loaded with the ring line
  const int t = threadIdx.x;
  const int S = a.S, n = a.n, tpp = a.tpp, sw = a.swp;
  const int lp = t / tpp;
  const int cl = (t % tpp) * VEC;   // first member slot of this thread within the tile
  // idle slots (past the tile's members) read the tile's last members and
  // store and sum nothing
  const bool lane_ok = cl < a.sw;
  const int sv = a.s0 + (lane_ok ? cl : a.sw - VEC);   // member whose values this lane loads
  const size_t slot_stride = a.vstride;
  const size_t line_stride = (size_t)n * S;
  const int chunk = tile % a.nchunk, band = tile / a.nchunk;
  const int i0 = chunk * a.tx, j0 = band * a.ty;
  const int j1 = min(j0 + a.ty, n);
  const int i = i0 + lp;
  const bool own_i = i < n;
  const bool own_s = own_i && lane_ok;   // this lane's point and members exist
  // halo duty: threads t < tpp also hold the point left of the chunk,
  // threads tpp <= t < 2 tpp the point right of it
  const bool halo = t < 2 * tpp, left_halo = t < tpp;
  const int hpt = left_halo ? -1 : a.tx;
  const int hi = i0 + hpt;
  const bool halo_i = hi >= 0 && hi < n;
  // Loads are issued by every lane at a point clamped into the grid and the
  // values of lanes without that point are replaced by zero afterwards: a
  // load inside a lane-dependent branch whose value is used after the branch
  // makes the compiler wait for it at the branch's end, before the line's
  // other loads are issued.
  const size_t col = (size_t)min(i, n - 1) * S + sv;
  const size_t hcol = (size_t)min(max(hi, 0), n - 1) * S + sv;
  auto row = [&](int jj) { return (size_t)min(max(jj, 0), n - 1) * line_stride; };

  // retained per own point: previous direction, diagonal, ring value
  double cur_pold[VEC], cur_v4[VEC], cur_val[VEC];
  double nxt_pold[VEC], nxt_v4[VEC], nxt_val[VEC];

  // the inputs of a ring value at element e, and the value itself:
  // M_PCG_J r / diag + beta p_old, M_PCG_Z z + beta p_old, M_CHEB1
  // (r - alpha q) / diag / theta, else the source
  auto fill_load = [&](size_t e, double (&v0)[VEC], double (&v1)[VEC], double (&v2)[VEC]) {
    if constexpr (MODE == M_SPMV || MODE == M_CHEB) {
      ld<VEC>(v0, a.src + e);
    } else if constexpr (MODE == M_CHEB1) {
      ld<VEC>(v0, a.r + e);
      ld<VEC>(v1, a.q_in + e);
      ld<VEC>(v2, a.V + 4 * slot_stride + e);
    } else if constexpr (MODE == M_PCG_J) {
      ld<VEC>(v0, a.r + e);
      ld<VEC>(v1, a.pold + e);
      ld<VEC>(v2, a.V + 4 * slot_stride + e);
    } else {  // M_PCG_Z
      ld<VEC>(v0, a.src + e);
      ld<VEC>(v1, a.pold + e);
    }
  };
  // M_CHEB1: the updated residual r - alpha q of member slot c (alpha 0:
  // unchanged, as in the separate update)
  auto rnew = [&](double r, double qv, int c) { return beta[c] != 0.0 ? fma(-beta[c], qv, r) : r; };
  auto combine = [&](const double (&v0)[VEC], const double (&v1)[VEC], const double (&v2)[VEC],
                     bool ok, double (&out)[VEC]) {
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      double v;
      if constexpr (MODE == M_PCG_J) v = fma(beta[c], v1[c], v0[c] / v2[c]);
      else if constexpr (MODE == M_PCG_Z) v = fma(beta[c], v1[c], v0[c]);
      else if constexpr (MODE == M_CHEB1) v = (rnew(v0[c], v1[c], c) / v2[c]) / aprev[c];
      else v = v0[c];
      out[c] = ok ? v : 0.0;
    }
  };
  // Ring values: the own point of ring line jj (`own` marks a line of this
  // tile, whose new direction is also stored) and, for the halo lanes, the
  // halo point.  The halo branch is entered only after every load of the
  // line has been issued, so its wait is the line's one round trip.
  auto put_own = [&](int jj, bool own, const double (&o0)[VEC], const double (&o1)[VEC],
                     const double (&o2)[VEC], double (&rp)[VEC], double (&rv4)[VEC],
                     double (&rval)[VEC]) {
    double* line = ring[(jj - j0 + 4) & 3];
    const bool ok = jj >= 0 && jj < n && own_i;
    double val[VEC];
    combine(o0, o1, o2, ok, val);
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      // retained: p_old (PCG) or the updated residual (M_CHEB1), the diagonal
      rp[c] = PCG ? o1[c] : ((MODE == M_CHEB1) ? rnew(o0[c], o1[c], c) : 0.0);
      rv4[c] = DIAG_IN_RING ? o2[c] : 0.0;
      line[(lp + 1) * sw + cl + c] = val[c];
      rval[c] = val[c];
    }
    if constexpr (PCG) {
      if (ok && own && lane_ok) st<VEC>(a.pnew + row(jj) + col, val);
    }
  };
  auto put_halo = [&](int jj, const double (&h0)[VEC], const double (&h1)[VEC],
                      const double (&h2)[VEC]) {
    double hv[VEC];
    combine(h0, h1, h2, jj >= 0 && jj < n && halo_i, hv);
#pragma unroll
    for (int c = 0; c < VEC; ++c) ring[(jj - j0 + 4) & 3][(hpt + 1) * sw + cl + c] = hv[c];
  };

  // symmetric sweep: per line slot (j - j0) & 1, LDS lines of E (line j),
  // NE and NW (line j - 1), each with the one-point halo
  auto symL = [&](int jj, int w) { return sym + (((jj - j0) & 1) * 3 + w) * kRing; };
  double prevN[VEC], prevNE[VEC], prevNW[VEC];   // own point, line j - 1

  __syncthreads();  // the previous tile's readers are done with the ring
  {
    if constexpr (SYM) {
      const size_t ep = row(j0 - 1) + col;
      ld_stream<VEC>(prevN, a.V + 7 * slot_stride + ep);
      ld_stream<VEC>(prevNE, a.V + 8 * slot_stride + ep);
      ld_stream<VEC>(prevNW, a.V + 6 * slot_stride + ep);
    }
    double a0[VEC], a1[VEC], a2[VEC], b0[VEC], b1[VEC], b2[VEC];
    fill_load(row(j0 - 1) + col, a0, a1, a2);
    fill_load(row(j0) + col, b0, b1, b2);
    if (halo) {
      double h0[VEC], h1[VEC], h2[VEC], g0[VEC], g1[VEC], g2[VEC];
      fill_load(row(j0 - 1) + hcol, h0, h1, h2);
      fill_load(row(j0) + hcol, g0, g1, g2);
      put_halo(j0 - 1, h0, h1, h2);
      put_halo(j0, g0, g1, g2);
    }
    double d0[VEC], d1[VEC], d2v[VEC];
    put_own(j0 - 1, false, a0, a1, a2, d0, d1, d2v);
    put_own(j0, true, b0, b1, b2, cur_pold, cur_v4, cur_val);
    if constexpr (SYM) {
      const bool okp = j0 > 0 && own_i;
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        prevN[c] = okp ? prevN[c] : 0.0;
        prevNE[c] = okp ? prevNE[c] : 0.0;
        prevNW[c] = okp ? prevNW[c] : 0.0;
      }
    }
  }
  for (int j = j0; j < j1; ++j) {
    // This line's matrix values (and x, or the Chebyshev r and z_{k-2}), the next
    // ring line's inputs and the halo values are all issued before any is
    // used: the line costs one memory round trip.
    const size_t rj = (size_t)j * line_stride;
    const size_t e = rj + col;
    double vk[9][VEC], xv[VEC], rr[VEC], dd[VEC];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if (SYM && k < 4) continue;                 // lower coefficients: from neighbours
      if (k == 4 && DIAG_IN_RING) continue;       // the diagonal came with the ring line
      ld_stream<VEC>(vk[k], a.V + (size_t)k * slot_stride + e);
    }
    if constexpr (PCG) ld<VEC>(xv, a.x + e);
    if constexpr (MODE == M_CHEB) {
      ld<VEC>(rr, a.r + e);
      if constexpr (ZPREV) ld<VEC>(dd, a.zprev + e);
    }
    double o0[VEC], o1[VEC], o2[VEC];
    fill_load(row(j + 1) + col, o0, o1, o2);
    if (halo) {
      double h0[VEC], h1[VEC], h2[VEC], hE[VEC], hX[VEC];
      fill_load(row(j + 1) + hcol, h0, h1, h2);
      if constexpr (SYM) {
        // E(i0 - 1, j) and NE(i0 - 1, j - 1) left of the chunk,
        // NW(i0 + tx, j - 1) right of it
        ld_stream<VEC>(hE, a.V + 5 * slot_stride + rj + hcol);
        ld_stream<VEC>(hX, a.V + (left_halo ? 8 : 6) * slot_stride + row(j - 1) + hcol);
      }
      put_halo(j + 1, h0, h1, h2);
      if constexpr (SYM) {
        const bool okE = halo_i && left_halo, okX = halo_i && j > 0;
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          if (left_halo) {
            symL(j, 0)[cl + c] = okE ? hE[c] : 0.0;
            symL(j, 1)[cl + c] = okX ? hX[c] : 0.0;
          } else {
            symL(j, 2)[(a.tx + 1) * sw + cl + c] = okX ? hX[c] : 0.0;
          }
        }
      }
    }
    put_own(j + 1, j + 1 < j1, o0, o1, o2, nxt_pold, nxt_v4, nxt_val);
    if constexpr (DIAG_IN_RING) {
#pragma unroll
      for (int c = 0; c < VEC; ++c) vk[4][c] = cur_v4[c];
    }
    if constexpr (SYM) {
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        symL(j, 0)[(lp + 1) * sw + cl + c] = own_i ? vk[5][c] : 0.0;
        symL(j, 1)[(lp + 1) * sw + cl + c] = prevNE[c];
        symL(j, 2)[(lp + 1) * sw + cl + c] = prevNW[c];
      }
    }
    __syncthreads();
    if constexpr (SYM) {
      // lower coefficients of row (i, j): SW = NE(i-1, j-1), S = N(i, j-1),
      // SE = NW(i+1, j-1), W = E(i-1, j)
      const double* pSW = symL(j, 1) + lp * sw + cl;
      const double* pSE = symL(j, 2) + (lp + 2) * sw + cl;
      const double* pW = symL(j, 0) + lp * sw + cl;
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        vk[0][c] = pSW[c];
        vk[1][c] = prevN[c];
        vk[2][c] = pSE[c];
        vk[3][c] = pW[c];
        prevN[c] = own_i ? vk[7][c] : 0.0;
        prevNE[c] = own_i ? vk[8][c] : 0.0;
        prevNW[c] = own_i ? vk[6][c] : 0.0;
      }
    }
    double q[VEC];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int dj = k / 3 - 1, di = k % 3 - 1;
      const double* rp = &ring[(j + dj - j0 + 4) & 3][(lp + 1 + di) * sw + cl];
      double pv[VEC];
      if constexpr (VEC == 2) {
        const d2 tt = *reinterpret_cast<const d2*>(rp);
        pv[0] = tt.x;
        pv[1] = tt.y;
      } else {
        pv[0] = rp[0];
      }
#pragma unroll
      for (int c = 0; c < VEC; ++c) q[c] = (k == 0) ? vk[0][c] * pv[c] : fma(vk[k][c], pv[c], q[c]);
    }
    // lanes without a point (the last chunk of a line) store nothing and
    // add nothing
    if constexpr (MODE == M_SPMV) {
      if (own_s) st<VEC>(a.q + e, q);
    } else if constexpr (PCG) {
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        acc[c] = own_s ? fma(cur_val[c], q[c], acc[c]) : acc[c];
        if (aprev[c] != 0.0) xv[c] = fma(aprev[c], cur_pold[c], xv[c]);
      }
      if (own_s) {
        st<VEC>(a.q + e, q);
        st<VEC>(a.x + e, xv);
      }
    } else if constexpr (MODE == M_CHEB1) {
      // d_0 = z_0 (the ring value), r' retained from the ring fill
      double zn[VEC], dn[VEC];
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        const double rn = cur_pold[c];
        dn[c] = c1[c] * cur_val[c] + c2[c] * ((rn - q[c]) / vk[4][c]);
        zn[c] = cur_val[c] + dn[c];
        acc[c] = own_s ? fma(rn, rn, acc[c]) : acc[c];
        if (a.cheb_last) acc2[c] = own_s ? fma(rn, zn[c], acc2[c]) : acc2[c];
      }
      if (own_s) {
        st<VEC>(a.r_out + e, cur_pold);
        st<VEC>(a.zout + e, zn);
      }
    } else {  // M_CHEB
      double zn[VEC];
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        double dp;   // d_{k-1}
        if constexpr (ZPREV) dp = cur_val[c] - dd[c];
        else if (a.cheb_step == 1) dp = cur_val[c];
        else dp = cur_val[c] - (rr[c] / vk[4][c]) / aprev[c];
        const double dn = c1[c] * dp + c2[c] * ((rr[c] - q[c]) / vk[4][c]);
        zn[c] = cur_val[c] + dn;
        if (a.cheb_last) acc[c] = own_s ? fma(rr[c], zn[c], acc[c]) : acc[c];
      }
      if (own_s) st<VEC>(a.zout + e, zn);
    }
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      cur_pold[c] = nxt_pold[c];
      cur_v4[c] = nxt_v4[c];
      cur_val[c] = nxt_val[c];
    }
  }
}

// Reduce a producer's per-workgroup partials in a fixed order and apply the
// per-member scalar logic of the step (one workgroup of kFinNT threads).
// `fin` holds 2 * kFinNT * 2 doubles.  Returns 1 when this call retired the
// ensemble.
template <int VEC>
__device__ __forceinline__ int finish_body(const FinishArgs& a, double* fin, int& live) {
  const int S = a.g.S, Sp = a.g.Sp, t = threadIdx.x;   // members, member slots
  const Members& m = a.m;
  const size_t ps = (size_t)a.G * Sp;
  switch (a.kind) {
    case F_ALPHA:
    case F_CHEB:
    case F_UPDATE_J:
    case F_UPDATE_C: {
      // A step of a running solve.  The control words and this member's
      // state are loaded before the partials are reduced and before any
      // store, so their latency overlaps the reduction's loads.
      const int done = gload(&m.ctl[CTL_DONE]);
      const int kprev = gload(&m.ctl[CTL_K]);
      const int maxit = gload(&m.ctl[CTL_MAXIT]);
      const bool mine = t < S;
      int act = 0;
      double rho = 0.0, alpha = 0.0, bn = 0.0;
      if (mine) {
        act = gload(&m.active[t]);
        rho = gload(&m.rho[t]);
        alpha = gload(&m.alpha[t]);
        bn = gload(&m.bnorm[t]);
      }
      double s0, s1 = 0.0;
      if (a.kind == F_UPDATE_J) {
        // r^T r and r^T z
        const double* const P[2] = {a.partial + ps, a.partial};
        double o2[2];
        final_sums<VEC, 2>(P, a.G, Sp, fin, o2);
        s0 = o2[0];
        s1 = o2[1];
      } else {
        // p^T A p (F_ALPHA), r^T z (F_CHEB) or r^T r (F_UPDATE_C)
        s0 = final_sum<VEC>(a.partial + (a.kind == F_UPDATE_C ? ps : 0), a.G, Sp, fin);
      }
      if (done) return 0;
      if (a.kind == F_ALPHA) {
        // p^T A p per member -> alpha, or freeze the member (the guard)
        if (mine) {
          double al = 0.0;
          if (act) {
            if (isfinite(s0) && s0 > 0.0) {
              al = rho / s0;
            } else {
              gstore(&m.active[t], 0);
              gstore(&m.status[t], ENS_BREAKDOWN);
              gstore(&m.iters[t], kprev + 1);
            }
          }
          gstore(&m.alpha[t], al);
        }
        return 0;
      }
      if (a.kind == F_CHEB) {
        // r^T z of a fresh preconditioner application -> rho (and beta)
        if (mine) {
          if (a.cheb_init) {
            gstore(&m.rho[t], s0);
            gstore(&m.beta[t], 0.0);
          } else if (act) {
            gstore(&m.beta[t], s0 / rho);
            gstore(&m.rho[t], s0);
          } else {
            gstore(&m.beta[t], 0.0);
          }
        }
        return 0;
      }
      // convergence test ||r_k|| <= rtol ||b||, iteration count, beta
      const int k = kprev + 1;
      if (t == 0) live = 0;
      __syncthreads();
      if (mine) {
        if (act) {
          const double rn = sqrt(s0);
          gstore(&m.relres[t], rn / bn);
          if (rn <= a.rtol * bn) {
            act = 0;
            gstore(&m.status[t], ENS_CONVERGED);
            gstore(&m.iters[t], k);
          } else if (k >= maxit) {
            act = 0;
            gstore(&m.status[t], ENS_MAX_ITER);
            gstore(&m.iters[t], k);
          }
          if (!act) gstore(&m.active[t], 0);
        }
        gstore(&m.alpha_prev[t], alpha);
        if (act) {
          if (a.kind == F_UPDATE_J) {
            gstore(&m.beta[t], s1 / rho);
            gstore(&m.rho[t], s1);
          }
          atomicAdd(&live, 1);
        } else {
          gstore(&m.beta[t], 0.0);
        }
      }
      __syncthreads();
      const int retired = (live == 0) ? 1 : 0;
      if (t == 0) {
        gstore(&m.ctl[CTL_K], k);
        gstore(&m.ctl[CTL_DONE], retired);
      }
      return retired;
    }
    case F_INIT: {
      const double bbs = final_sum<VEC>(a.partial + ps, a.G, Sp, fin);
      double rzs = 0.0, lmax = 0.0;
      if (!a.cheb) rzs = final_sum<VEC>(a.partial, a.G, Sp, fin);
      else lmax = final_max(a.partial + 2 * ps, a.G, Sp, fin);
      if (t == 0) live = 0;
      __syncthreads();
      if (t >= S && t < Sp) {
        // idle slots: inactive, every step zero
        gstore(&m.active[t], 0);
        gstore(&m.alpha[t], 0.0);
        gstore(&m.alpha_prev[t], 0.0);
        gstore(&m.beta[t], 0.0);
        gstore(&m.rho[t], 0.0);
        gstore(&m.bnorm[t], 1.0);
        gstore(&m.cheb[(size_t)t * kChebCoef], 1.0);
        for (int k = 1; k < 2 * kMaxCheb + 1; ++k) gstore(&m.cheb[(size_t)t * kChebCoef + k], 0.0);
      }
      if (t < S) {
        const double bn = sqrt(bbs);
        gstore(&m.bnorm[t], bn);
        gstore(&m.alpha[t], 0.0);
        gstore(&m.alpha_prev[t], 0.0);
        gstore(&m.beta[t], 0.0);
        gstore(&m.rho[t], rzs);
        gstore(&m.iters[t], 0);
        if (bn == 0.0) {
          gstore(&m.active[t], 0);
          gstore(&m.status[t], ENS_ZERO_RHS);
          gstore(&m.relres[t], 0.0);
        } else {
          gstore(&m.active[t], 1);
          gstore(&m.status[t], ENS_MAX_ITER);
          gstore(&m.relres[t], 1.0);
          atomicAdd(&live, 1);
        }
        if (a.cheb) {
          // Chebyshev semi-iteration on [lmax / ratio, lmax]: theta, delta the
          // centre and half-width; step k uses c1 = rho_k rho_{k-1},
          // c2 = 2 rho_k / delta with rho_k = 1 / (2 sigma1 - rho_{k-1}).
          gstore(&m.lmax[t], lmax);
          const double lmin = lmax / a.cheb_ratio;
          const double theta = (lmax + lmin) / 2.0;
          const double delta = (lmax - lmin) / 2.0;
          const double sigma1 = theta / delta;
          double rho0 = 1.0 / sigma1;
          double* cf = m.cheb + (size_t)t * kChebCoef;
          gstore(&cf[0], theta);
          for (int k = 1; k < a.cheb_degree; ++k) {
            const double rho1 = 1.0 / (2.0 * sigma1 - rho0);
            gstore(&cf[2 * k - 1], rho1 * rho0);
            gstore(&cf[2 * k], 2.0 * rho1 / delta);
            rho0 = rho1;
          }
        }
      }
      __syncthreads();
      if (t == 0) {
        gstore(&m.ctl[CTL_K], 0);
        gstore(&m.ctl[CTL_MAXIT], a.max_iter);
        gstore(&m.ctl[CTL_DONE], (live == 0) ? 1 : 0);
      }
      return 0;
    }
    case F_MAX: {
      // per-member maximum of one partial array into result[s][0]
      const double v = final_max(a.partial, a.G, Sp, fin);
      if (t < S) gstore(&m.result[(size_t)t * 16], v);
      return 0;
    }
    case F_DOT:
    case F_SUMS: {
      // nsum member sums, scaled, into result[s][q]
      for (int q = 0; q < a.nsum; ++q) {
        const double v = final_sum<VEC>(a.partial + q * ps, a.G, Sp, fin);
        if (t < S) gstore(&m.result[(size_t)t * 16 + q], a.scale * v);
      }
      return 0;
    }
  }
  return 0;
}

}  // namespace ens
