// Device code shared by the single-ensemble kernels (kernels.hip) and the
// batched kernels (batch.hip): vector loads, the fixed-tree member
// reductions, the fused tile sweep and the finish logic.
#pragma once

#include "common.h"

namespace ens {

typedef double d2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------ load/store
template <int VEC>
__device__ __forceinline__ void ld(double (&v)[VEC], const double* p) {
  if constexpr (VEC == 2) {
    const d2 t = *reinterpret_cast<const d2*>(p);
    v[0] = t.x;
    v[1] = t.y;
  } else {
    v[0] = *p;
  }
}

// matrix values are streamed once per iteration: non-temporal loads keep the
// vectors' lines in the caches
template <int VEC>
__device__ __forceinline__ void ld_stream(double (&v)[VEC], const double* p) {
  if constexpr (VEC == 2) {
    const d2 t = __builtin_nontemporal_load(reinterpret_cast<const d2*>(p));
    v[0] = t.x;
    v[1] = t.y;
  } else {
    v[0] = __builtin_nontemporal_load(p);
  }
}

template <int VEC>
__device__ __forceinline__ void st(double* p, const double (&v)[VEC]) {
  if constexpr (VEC == 2) {
    d2 t;
    t.x = v[0];
    t.y = v[1];
    *reinterpret_cast<d2*>(p) = t;
  } else {
    *p = v[0];
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

// write this workgroup's partial [S] (threads t < tpp); a finish kernel
// launched after this one reads them (the kernel boundary makes them visible
// across XCDs, so no in-kernel device-scope fence is needed)
template <int VEC>
__device__ __forceinline__ void put_partial(double* partial, int S, int tpp, const double (&v)[VEC],
                                            int s0 = 0) {
  if ((int)threadIdx.x < tpp) {
#pragma unroll
    for (int c = 0; c < VEC; ++c) partial[(size_t)blockIdx.x * S + s0 + threadIdx.x * VEC + c] = v[c];
  }
}

// Member sums of NARR partial arrays P[a][g][s] over the workgroups g < G,
// returned for member s = threadIdx.x (t < S).  Thread t loads VEC members
// per row (16-byte loads when VEC = 2); the R = kNT * VEC / S row sets are
// k, k + R, k + 2R, ... with k = t / (S / VEC), summed in that order with up
// to 16 loads in flight, then a fixed halving tree over k.  The order does
// not depend on the member.  `lds` holds NARR * kNT * VEC doubles.
template <int VEC, int NARR>
__device__ __forceinline__ void final_sums(const double* const (&P)[NARR], int G, int S,
                                           double* lds, double (&out)[NARR]) {
  const int t = threadIdx.x;
  const int W = S / VEC, R = kNT / W;
  const int pr = t % W, k = t / W;
  const int col = pr * VEC;
  constexpr int B = 16 / NARR;
  double acc[NARR][VEC];
#pragma unroll
  for (int a = 0; a < NARR; ++a)
#pragma unroll
    for (int c = 0; c < VEC; ++c) acc[a][c] = 0.0;
  int g = k;
  for (; g + (B - 1) * R < G; g += B * R) {
    double v[NARR][B][VEC];
#pragma unroll
    for (int a = 0; a < NARR; ++a)
#pragma unroll
      for (int u = 0; u < B; ++u) ld<VEC>(v[a][u], P[a] + (size_t)(g + u * R) * S + col);
#pragma unroll
    for (int a = 0; a < NARR; ++a)
#pragma unroll
      for (int u = 0; u < B; ++u)
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[a][c] += v[a][u][c];
  }
  for (; g < G; g += R) {
#pragma unroll
    for (int a = 0; a < NARR; ++a) {
      double v[VEC];
      ld<VEC>(v, P[a] + (size_t)g * S + col);
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[a][c] += v[c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NARR; ++a)
#pragma unroll
    for (int c = 0; c < VEC; ++c) lds[a * kNT * VEC + k * S + col + c] = acc[a][c];
  __syncthreads();
  for (int stride = (R / 2) * S; stride >= S; stride >>= 1) {
#pragma unroll
    for (int a = 0; a < NARR; ++a)
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        const int i = t * VEC + c;
        if (i < stride) lds[a * kNT * VEC + i] += lds[a * kNT * VEC + i + stride];
      }
    __syncthreads();
  }
  const int s = t & (S - 1);
#pragma unroll
  for (int a = 0; a < NARR; ++a) out[a] = lds[a * kNT * VEC + s];
}

template <int VEC>
__device__ __forceinline__ double final_sum(const double* partial, int G, int S, double* lds) {
  const double* const P[1] = {partial};
  double out[1];
  final_sums<VEC, 1>(P, G, S, lds, out);
  return out[0];
}

__device__ __forceinline__ double final_max(const double* partial, int G, int S, double* lds) {
  const int t = threadIdx.x, s = t & (S - 1), k = t / S, T = kNT / S;
  double acc = 0.0;
  for (int g = k; g < G; g += T) acc = fmax(acc, partial[(size_t)g * S + s]);
  __syncthreads();
  lds[t] = acc;
  __syncthreads();
  for (int stride = kNT / 2; stride >= S; stride >>= 1) {
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
  double* d;
  double* zout;
  int n, S;        // grid size, ensemble width (row stride of every vector)
  int sw, s0;      // members this tile covers: s0 .. s0 + sw - 1
  int tpp;         // threads per grid point = sw / VEC
  int tx, ty, nchunk;
  size_t nelem;
  int cheb_last;
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
//   M_CHEB:  one Chebyshev step d = c1 d + c2 D^-1 (r - A z), z += d, and
//            on the last step accumulate r^T z.
//
// SYM: the matrix is symmetric, so only C, E, N, NE, NW are read; the lower
// coefficients of row (i, j) are W = E(i-1, j), S = N(i, j-1), SW = NE(i-1,
// j-1) and SE = NW(i+1, j-1).  Each thread keeps N, NE, NW of its point's
// previous line in registers; E of the current line and NE, NW of the
// previous line are exchanged through `sym` (LDS, 2 x 3 lines of kRing
// doubles).  The products are formed in the same order as the nine-value
// sweep, so on a bitwise-symmetric matrix both give the same bits.
template <int VEC, int MODE, bool SYM>
__device__ __forceinline__ void stencil_tile(const TileView& a, int tile, double (*ring)[kRing],
                                             double* sym,
                                             const double (&beta)[VEC], const double (&aprev)[VEC],
                                             const double (&c1)[VEC], const double (&c2)[VEC],
                                             double (&acc)[VEC]) {
  const int t = threadIdx.x;
  const int S = a.S, n = a.n, tpp = a.tpp, sw = a.sw;
  const int lp = t / tpp;
  const int cl = (t % tpp) * VEC;   // first member of this thread within the tile
  const int sv = a.s0 + cl;         // ... within the ensemble
  const size_t slot_stride = a.nelem;
  const int chunk = tile % a.nchunk, band = tile / a.nchunk;
  const int i0 = chunk * a.tx, j0 = band * a.ty;
  const int j1 = min(j0 + a.ty, n);
  const int i = i0 + lp;
  const bool own_i = i < n;

  // retained per own point: previous direction, diagonal, ring value
  double cur_pold[VEC], cur_v4[VEC], cur_val[VEC];
  double nxt_pold[VEC], nxt_v4[VEC], nxt_val[VEC];

  // form the ring values of line jj; `own` marks a line of this tile
  auto fill = [&](int jj, bool own, double (&rp)[VEC], double (&rv4)[VEC], double (&rval)[VEC]) {
    double* line = ring[(jj - j0 + 4) & 3];
    double val[VEC];
    const bool in_line = (jj >= 0 && jj < n);
    if (in_line && own_i) {
      const size_t e = ((size_t)jj * n + i) * S + sv;
      if constexpr (MODE == M_SPMV || MODE == M_CHEB) {
        ld<VEC>(val, a.src + e);
      } else if constexpr (MODE == M_PCG_J) {
        double rr[VEC], pp[VEC], dd[VEC];
        ld<VEC>(rr, a.r + e);
        ld<VEC>(pp, a.pold + e);
        ld<VEC>(dd, a.V + 4 * slot_stride + e);
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          val[c] = fma(beta[c], pp[c], rr[c] / dd[c]);
          rp[c] = pp[c];
          rv4[c] = dd[c];
        }
        if (own) st<VEC>(a.pnew + e, val);
      } else {  // M_PCG_Z
        double zz[VEC], pp[VEC];
        ld<VEC>(zz, a.src + e);
        ld<VEC>(pp, a.pold + e);
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          val[c] = fma(beta[c], pp[c], zz[c]);
          rp[c] = pp[c];
        }
        if (own) st<VEC>(a.pnew + e, val);
      }
    } else {
#pragma unroll
      for (int c = 0; c < VEC; ++c) val[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      line[(lp + 1) * sw + cl + c] = val[c];
      rval[c] = val[c];
    }
    // one-point halo on both sides of the chunk
    if (t < 2 * tpp) {
      const int hp = (t < tpp) ? -1 : a.tx;
      const int hi = i0 + hp;
      double hv[VEC];
      if (in_line && hi >= 0 && hi < n) {
        const size_t he = ((size_t)jj * n + hi) * S + sv;
        if constexpr (MODE == M_SPMV || MODE == M_CHEB) {
          ld<VEC>(hv, a.src + he);
        } else if constexpr (MODE == M_PCG_J) {
          double rr[VEC], pp[VEC], dd[VEC];
          ld<VEC>(rr, a.r + he);
          ld<VEC>(pp, a.pold + he);
          ld<VEC>(dd, a.V + 4 * slot_stride + he);
#pragma unroll
          for (int c = 0; c < VEC; ++c) hv[c] = fma(beta[c], pp[c], rr[c] / dd[c]);
        } else {
          double zz[VEC], pp[VEC];
          ld<VEC>(zz, a.src + he);
          ld<VEC>(pp, a.pold + he);
#pragma unroll
          for (int c = 0; c < VEC; ++c) hv[c] = fma(beta[c], pp[c], zz[c]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < VEC; ++c) hv[c] = 0.0;
      }
#pragma unroll
      for (int c = 0; c < VEC; ++c) line[(hp + 1) * sw + cl + c] = hv[c];
    }
  };

  // symmetric sweep: per line slot (j - j0) & 1, LDS lines of E (line j),
  // NE and NW (line j - 1), each with the one-point halo
  auto symL = [&](int jj, int w) { return sym + (((jj - j0) & 1) * 3 + w) * kRing; };
  const bool left_halo = t < tpp, halo = t < 2 * tpp;
  const int hi = i0 + (left_halo ? -1 : a.tx);   // halo point of this thread
  double prevN[VEC], prevNE[VEC], prevNW[VEC];   // own point, line j - 1
#pragma unroll
  for (int c = 0; c < VEC; ++c) prevN[c] = prevNE[c] = prevNW[c] = 0.0;

  __syncthreads();  // the previous tile's readers are done with the ring
  {
    double d0[VEC], d1[VEC], d2v[VEC];
    fill(j0 - 1, false, d0, d1, d2v);
  }
  if constexpr (SYM) {
    if (j0 > 0 && own_i) {
      const size_t ep = ((size_t)(j0 - 1) * n + i) * S + sv;
      ld_stream<VEC>(prevN, a.V + 7 * slot_stride + ep);
      ld_stream<VEC>(prevNE, a.V + 8 * slot_stride + ep);
      ld_stream<VEC>(prevNW, a.V + 6 * slot_stride + ep);
    }
  }
  fill(j0, true, cur_pold, cur_v4, cur_val);
  for (int j = j0; j < j1; ++j) {
    // Issue this line's matrix values (and x, or the Chebyshev r and d)
    // before forming the next ring line: both sets of loads are then in
    // flight together and the line costs one memory round trip.
    const size_t e = ((size_t)j * n + i) * S + sv;
    double vk[9][VEC], xv[VEC], rr[VEC], dd[VEC], hE[VEC], hX[VEC];
    if constexpr (SYM) {
#pragma unroll
      for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int c = 0; c < VEC; ++c) vk[k][c] = 0.0;
#pragma unroll
      for (int c = 0; c < VEC; ++c) hE[c] = hX[c] = 0.0;
    }
    if (own_i) {
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        if (SYM && k < 4) continue;   // lower coefficients: from neighbours
        if (k == 4 && MODE == M_PCG_J) {
#pragma unroll
          for (int c = 0; c < VEC; ++c) vk[4][c] = cur_v4[c];
        } else {
          ld_stream<VEC>(vk[k], a.V + (size_t)k * slot_stride + e);
        }
      }
      if constexpr (MODE == M_PCG_J || MODE == M_PCG_Z) ld<VEC>(xv, a.x + e);
      if constexpr (MODE == M_CHEB) {
        ld<VEC>(rr, a.r + e);
        ld<VEC>(dd, a.d + e);
      }
    }
    if constexpr (SYM) {
      // halo: E(i0 - 1, j) and NE(i0 - 1, j - 1) left of the chunk,
      // NW(i0 + tx, j - 1) right of it
      if (halo && hi >= 0 && hi < n) {
        const size_t he = ((size_t)j * n + hi) * S + sv;
        if (left_halo) {
          ld_stream<VEC>(hE, a.V + 5 * slot_stride + he);
          if (j > 0) ld_stream<VEC>(hX, a.V + 8 * slot_stride + he - (size_t)n * S);
        } else if (j > 0) {
          ld_stream<VEC>(hX, a.V + 6 * slot_stride + he - (size_t)n * S);
        }
      }
    }
    fill(j + 1, j + 1 < j1, nxt_pold, nxt_v4, nxt_val);
    if constexpr (SYM) {
      double* lE = symL(j, 0);
      double* lNE = symL(j, 1);
      double* lNW = symL(j, 2);
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        lE[(lp + 1) * sw + cl + c] = vk[5][c];
        lNE[(lp + 1) * sw + cl + c] = prevNE[c];
        lNW[(lp + 1) * sw + cl + c] = prevNW[c];
        if (halo) {
          if (left_halo) {
            lE[cl + c] = hE[c];
            lNE[cl + c] = hX[c];
          } else {
            lNW[(a.tx + 1) * sw + cl + c] = hX[c];
          }
        }
      }
    }
    __syncthreads();
    if (own_i) {
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
          prevN[c] = vk[7][c];
          prevNE[c] = vk[8][c];
          prevNW[c] = vk[6][c];
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
      if constexpr (MODE == M_SPMV) {
        st<VEC>(a.q + e, q);
      } else if constexpr (MODE == M_PCG_J || MODE == M_PCG_Z) {
        st<VEC>(a.q + e, q);
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          acc[c] = fma(cur_val[c], q[c], acc[c]);
          if (aprev[c] != 0.0) xv[c] = fma(aprev[c], cur_pold[c], xv[c]);
        }
        st<VEC>(a.x + e, xv);
      } else {  // M_CHEB
        double zn[VEC];
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          dd[c] = c1[c] * dd[c] + c2[c] * ((rr[c] - q[c]) / vk[4][c]);
          zn[c] = cur_val[c] + dd[c];
          if (a.cheb_last) acc[c] = fma(rr[c], zn[c], acc[c]);
        }
        st<VEC>(a.d + e, dd);
        st<VEC>(a.zout + e, zn);
      }
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
// per-member scalar logic of the step (one workgroup).  `fin` holds
// 2 * kNT * 2 doubles.  Returns 1 when this call retired the ensemble.
template <int VEC>
__device__ __forceinline__ int finish_body(const FinishArgs& a, double* fin, int& live) {
  const int S = a.g.S, t = threadIdx.x;
  const Members& m = a.m;
  const size_t ps = (size_t)a.G * S;
  if (a.kind != F_INIT && a.kind != F_DOT && a.kind != F_SUMS) {
    if (m.ctl[CTL_DONE]) return 0;
  }
  switch (a.kind) {
    case F_ALPHA: {
      // p^T A p per member -> alpha, or freeze the member (the guard)
      const double sig = final_sum<VEC>(a.partial, a.G, S, fin);
      if (t < S) {
        double al = 0.0;
        if (m.active[t]) {
          if (isfinite(sig) && sig > 0.0) {
            al = m.rho[t] / sig;
          } else {
            m.active[t] = 0;
            m.status[t] = ENS_BREAKDOWN;
            m.iters[t] = m.ctl[CTL_K] + 1;
          }
        }
        m.alpha[t] = al;
      }
      return 0;
    }
    case F_CHEB: {
      // r^T z of a fresh preconditioner application -> rho (and beta)
      const double rz = final_sum<VEC>(a.partial, a.G, S, fin);
      if (t < S) {
        if (a.cheb_init) {
          m.rho[t] = rz;
          m.beta[t] = 0.0;
        } else if (m.active[t]) {
          m.beta[t] = rz / m.rho[t];
          m.rho[t] = rz;
        } else {
          m.beta[t] = 0.0;
        }
      }
      return 0;
    }
    case F_UPDATE_J:
    case F_UPDATE_C: {
      // convergence test ||r_k|| <= rtol ||b||, iteration count, beta
      double rrs, rzs = 0.0;
      if (a.kind == F_UPDATE_J) {
        const double* const P[2] = {a.partial + ps, a.partial};
        double o2[2];
        final_sums<VEC, 2>(P, a.G, S, fin, o2);
        rrs = o2[0];
        rzs = o2[1];
      } else {
        rrs = final_sum<VEC>(a.partial + ps, a.G, S, fin);
      }
      const int k = m.ctl[CTL_K] + 1;
      if (t == 0) live = 0;
      __syncthreads();
      if (t < S) {
        if (m.active[t]) {
          const double rn = sqrt(rrs);
          m.relres[t] = rn / m.bnorm[t];
          if (rn <= a.rtol * m.bnorm[t]) {
            m.active[t] = 0;
            m.status[t] = ENS_CONVERGED;
            m.iters[t] = k;
          } else if (k >= m.ctl[CTL_MAXIT]) {
            m.active[t] = 0;
            m.status[t] = ENS_MAX_ITER;
            m.iters[t] = k;
          }
        }
        m.alpha_prev[t] = m.alpha[t];
        if (m.active[t]) {
          if (a.kind == F_UPDATE_J) {
            m.beta[t] = rzs / m.rho[t];
            m.rho[t] = rzs;
          }
          atomicAdd(&live, 1);
        } else {
          m.beta[t] = 0.0;
        }
      }
      __syncthreads();
      const int retired = (live == 0) ? 1 : 0;
      if (t == 0) {
        m.ctl[CTL_K] = k;
        m.ctl[CTL_DONE] = retired;
      }
      return retired;
    }
    case F_INIT: {
      const double bbs = final_sum<VEC>(a.partial + ps, a.G, S, fin);
      double rzs = 0.0, lmax = 0.0;
      if (!a.cheb) rzs = final_sum<VEC>(a.partial, a.G, S, fin);
      else lmax = final_max(a.partial + 2 * ps, a.G, S, fin);
      if (t == 0) live = 0;
      __syncthreads();
      if (t < S) {
        const double bn = sqrt(bbs);
        m.bnorm[t] = bn;
        m.alpha[t] = 0.0;
        m.alpha_prev[t] = 0.0;
        m.beta[t] = 0.0;
        m.rho[t] = rzs;
        m.iters[t] = 0;
        if (bn == 0.0) {
          m.active[t] = 0;
          m.status[t] = ENS_ZERO_RHS;
          m.relres[t] = 0.0;
        } else {
          m.active[t] = 1;
          m.status[t] = ENS_MAX_ITER;
          m.relres[t] = 1.0;
          atomicAdd(&live, 1);
        }
        if (a.cheb) {
          // Chebyshev semi-iteration on [lmax / ratio, lmax]: theta, delta the
          // centre and half-width; step k uses c1 = rho_k rho_{k-1},
          // c2 = 2 rho_k / delta with rho_k = 1 / (2 sigma1 - rho_{k-1}).
          m.lmax[t] = lmax;
          const double lmin = lmax / a.cheb_ratio;
          const double theta = (lmax + lmin) / 2.0;
          const double delta = (lmax - lmin) / 2.0;
          const double sigma1 = theta / delta;
          double rho0 = 1.0 / sigma1;
          double* cf = m.cheb + (size_t)t * kChebCoef;
          cf[0] = theta;
          for (int k = 1; k < a.cheb_degree; ++k) {
            const double rho1 = 1.0 / (2.0 * sigma1 - rho0);
            cf[2 * k - 1] = rho1 * rho0;
            cf[2 * k] = 2.0 * rho1 / delta;
            rho0 = rho1;
          }
        }
      }
      __syncthreads();
      if (t == 0) {
        m.ctl[CTL_K] = 0;
        m.ctl[CTL_MAXIT] = a.max_iter;
        m.ctl[CTL_DONE] = (live == 0) ? 1 : 0;
      }
      return 0;
    }
    case F_DOT:
    case F_SUMS: {
      // nsum member sums, scaled, into result[s][q]
      for (int q = 0; q < a.nsum; ++q) {
        const double v = final_sum<VEC>(a.partial + q * ps, a.G, S, fin);
        if (t < S) m.result[(size_t)t * 16 + q] = a.scale * v;
      }
      return 0;
    }
  }
  return 0;
}

}  // namespace ens
