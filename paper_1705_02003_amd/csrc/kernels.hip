// HIP kernels of the ensemble PCG hot path for CDNA4 (gfx950).
//
// Data layout: member index innermost (paper, Section 2.3, commuted Kronecker
// ordering): vectors X[r * S + s], matrix values V[(k * N_r + r) * S + s].
// A grid point's S members are contiguous, so every load and store moves
// whole 8*S-byte runs, and the stencil structure (the shared sparsity
// pattern) is implicit: there is no index array at all, it is "read" once
// per tile for all S members (Section 2.3, reuse of sample-independent data).
//
// Thread mapping: VEC = 2 members per thread (one 16-byte load) when S >= 2,
// VEC = 1 for S = 1.  tpp = S / VEC threads cover one grid point; a wave64
// covers 64 / tpp consecutive points of one grid line.
//
// Reductions: every per-member inner product is reduced in a fixed tree
// (per-thread sequential sums, xor-shuffles across lanes that hold the same
// members, a fixed-order sum across the four waves, then a fixed-order sum
// over workgroup partials in the last workgroup to finish).  The tree does
// not depend on the member index, so results are deterministic and
// permuting members permutes results bit for bit.  No floating-point
// atomics are used.
#include <cmath>

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
__device__ __forceinline__ void put_partial(double* partial, int S, int tpp, const double (&v)[VEC]) {
  if ((int)threadIdx.x < tpp) {
#pragma unroll
    for (int c = 0; c < VEC; ++c) partial[(size_t)blockIdx.x * S + threadIdx.x * VEC + c] = v[c];
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

// ------------------------------------------------------------ assembly
// One thread per (row, member).  Evaluation order of every expression
// follows the scheme's definition term by term; contraction into FMA is off
// so the values are the plainly rounded ones.
__global__ __launch_bounds__(kNT) void assemble_kernel(AsmArgs a) {
#pragma clang fp contract(off)
  const size_t e = (size_t)blockIdx.x * kNT + threadIdx.x;
  if (e >= a.nelem) return;
  const int n = a.n;
  const int s = (int)(e & (size_t)(a.S - 1));
  const size_t row = e >> a.logS;
  const int i = (int)(row % n), j = (int)(row / n);
  const double* y = a.y + (size_t)s * a.d;

  const double eps = (a.eps_model == 0) ? pow(10.0, -(1.0 + y[0])) : pow(10.0, -(1.5 + 1.5 * y[0]));
  const double theta = (M_PI / 4.0) * (1.0 + y[1]);
  const double c = cos(theta), sn = sin(theta);
  const double k11 = c * c + eps * (sn * sn);
  const double k22 = sn * sn + eps * (c * c);
  const double k12 = (1.0 - eps) * (sn * c);

  // a at the node (I, J) = (i + 1, j + 1) and its four neighbours, 1-based
  // node indices on the (n+2)^2 grid, x = index / (n + 1).
  const int I = i + 1, J = j + 1;
  double aC = 1.0, aE = 1.0, aW = 1.0, aN = 1.0, aS = 1.0;
  for (int k = 1; k <= a.d - 2; ++k) {
    const double kp = (double)k * M_PI;
    const double sIm = sin(kp * ((double)(I - 1) / (double)(n + 1)));
    const double sI = sin(kp * ((double)I / (double)(n + 1)));
    const double sIp = sin(kp * ((double)(I + 1) / (double)(n + 1)));
    const double sJm = sin(kp * ((double)(J - 1) / (double)(n + 1)));
    const double sJ = sin(kp * ((double)J / (double)(n + 1)));
    const double sJp = sin(kp * ((double)(J + 1) / (double)(n + 1)));
    const double yk = y[k + 1], kk = (double)(k * k);
    aC = aC + a.amp * ((yk * (sJ * sI)) / kk);
    aE = aE + a.amp * ((yk * (sJ * sIp)) / kk);
    aW = aW + a.amp * ((yk * (sJ * sIm)) / kk);
    aN = aN + a.amp * ((yk * (sJp * sI)) / kk);
    aS = aS + a.amp * ((yk * (sJm * sI)) / kk);
  }
  const double fE = (aC + aE) / 2.0, fW = (aC + aW) / 2.0;
  const double fN = (aC + aN) / 2.0, fS = (aC + aS) / 2.0;
  const double bE = k12 * aE, bW = k12 * aW, bN = k12 * aN, bS = k12 * aS;

  double h2[9];
  h2[4] = k11 * (fE + fW) + k22 * (fN + fS);
  h2[5] = -k11 * fE;
  h2[3] = -k11 * fW;
  h2[7] = -k22 * fN;
  h2[1] = -k22 * fS;
  h2[8] = -(bE + bN) / 4.0;
  h2[0] = -(bW + bS) / 4.0;
  h2[6] = (bW + bN) / 4.0;
  h2[2] = (bE + bS) / 4.0;
  if (i == 0) h2[0] = h2[3] = h2[6] = 0.0;
  if (i == n - 1) h2[2] = h2[5] = h2[8] = 0.0;
  if (j == 0) h2[0] = h2[1] = h2[2] = 0.0;
  if (j == n - 1) h2[6] = h2[7] = h2[8] = 0.0;
  const double inv_h2 = (double)(n + 1) * (double)(n + 1);
#pragma unroll
  for (int k = 0; k < 9; ++k) a.V[(size_t)k * a.nelem + e] = h2[k] * inv_h2;
  a.b[e] = 1.0;
}

// ------------------------------------------------------------ stencil
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

// Fused tile kernel.  A tile is tx grid points of one line chunk times ty
// lines.  The tile is swept line by line; the values the stencil reads
// (M_PCG_J: the new direction p = r / diag + beta p_old; M_PCG_Z: p = z +
// beta p_old; M_SPMV: p; M_CHEB: z) are formed once per point, including a
// one-point halo, into a four-line LDS ring, so each line needs one barrier.
// Then, per point and member, the nine-point product is taken from the ring
// and the mode's fused updates follow:
//   M_PCG_*: store p and q = A p, accumulate p^T q, apply the deferred
//            x += alpha_prev p_old; the last workgroup turns p^T q into alpha
//            (or freezes a member whose p^T A p is not a positive finite
//            number -- the paper's guard).
//   M_CHEB:  one Chebyshev step d = c1 d + c2 D^-1 (r - A z), z += d; the
//            last step accumulates r^T z and the last workgroup forms beta.
template <int VEC, int MODE>
__global__ __launch_bounds__(kNT) void stencil_kernel(StencilArgs a) {
  __shared__ __attribute__((aligned(16))) double ring[4][kRing];
  __shared__ double red[kWaves * 64 * 2];
  const Geometry& g = a.g;
  if constexpr (MODE != M_SPMV) {
    if (a.m.ctl[CTL_DONE]) return;
  }
  const int t = threadIdx.x;
  const int S = g.S, n = g.n, tpp = g.tpp;
  const int lp = t / tpp;
  const int sv = (t % tpp) * VEC;
  const size_t slot_stride = g.nelem;

  double beta[VEC], aprev[VEC], c1[VEC], c2[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) {
    beta[c] = 0.0;
    aprev[c] = 0.0;
    c1[c] = 0.0;
    c2[c] = 0.0;
    if constexpr (MODE == M_PCG_J || MODE == M_PCG_Z) {
      beta[c] = a.m.beta[sv + c];
      aprev[c] = a.m.alpha_prev[sv + c];
    }
    if constexpr (MODE == M_CHEB) {
      c1[c] = a.m.cheb[(size_t)(sv + c) * kChebCoef + 2 * a.cheb_step - 1];
      c2[c] = a.m.cheb[(size_t)(sv + c) * kChebCoef + 2 * a.cheb_step];
    }
  }
  double acc[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) acc[c] = 0.0;

  int tile, tstep, tend;
  tile_range(g, tile, tstep, tend);
  for (; tile < tend; tile += tstep) {
    const int chunk = tile % g.nchunk, band = tile / g.nchunk;
    const int i0 = chunk * g.tx, j0 = band * g.ty;
    const int j1 = min(j0 + g.ty, n);
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
        line[(lp + 1) * S + sv + c] = val[c];
        rval[c] = val[c];
      }
      // one-point halo on both sides of the chunk
      if (t < 2 * tpp) {
        const int hp = (t < tpp) ? -1 : g.tx;
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
        for (int c = 0; c < VEC; ++c) line[(hp + 1) * S + sv + c] = hv[c];
      }
    };

    __syncthreads();  // the previous tile's readers are done with the ring
    {
      double d0[VEC], d1[VEC], d2v[VEC];
      fill(j0 - 1, false, d0, d1, d2v);
    }
    fill(j0, true, cur_pold, cur_v4, cur_val);
    for (int j = j0; j < j1; ++j) {
      // Issue this line's matrix values (and x, or the Chebyshev r and d)
      // before forming the next ring line: both sets of loads are then in
      // flight together and the line costs one memory round trip.
      const size_t e = ((size_t)j * n + i) * S + sv;
      double vk[9][VEC], xv[VEC], rr[VEC], dd[VEC];
      if (own_i) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
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
      fill(j + 1, j + 1 < j1, nxt_pold, nxt_v4, nxt_val);
      __syncthreads();
      if (own_i) {
        double q[VEC];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          const int dj = k / 3 - 1, di = k % 3 - 1;
          const double* rp = &ring[(j + dj - j0 + 4) & 3][(lp + 1 + di) * S + sv];
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

  if constexpr (MODE == M_SPMV) {
    return;
  } else {
    if constexpr (MODE == M_CHEB) {
      if (!a.cheb_last) return;
    }
    group_reduce<VEC>(acc, tpp, red);
    put_partial<VEC>(a.partial, S, tpp, acc);
  }
}

// ------------------------------------------------------------ update
// r -= alpha q for active members; then (Jacobi) z = D^-1 r and partial
// r^T z, r^T r, or (Chebyshev) the first semi-iteration step d = z =
// D^-1 r / theta.  The last workgroup applies the convergence test
// ||r_k|| <= rtol ||b|| per member, records the member's iteration count,
// forms beta (Jacobi) and raises the done flag when no member is active.
template <int VEC, bool CHEB>
__global__ __launch_bounds__(kNT) void update_kernel(UpdateArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  if (a.m.ctl[CTL_DONE]) return;
  const Geometry& g = a.g;
  const int S = g.S, tpp = g.tpp;
  const int t = threadIdx.x;
  const int sv = (t % tpp) * VEC;
  double alpha[VEC], act[VEC], ith[VEC], rz[VEC], rr[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) {
    act[c] = a.m.active[sv + c] ? 1.0 : 0.0;
    alpha[c] = a.m.alpha[sv + c];
    ith[c] = CHEB ? a.m.cheb[(size_t)(sv + c) * kChebCoef] : 0.0;
    rz[c] = 0.0;
    rr[c] = 0.0;
  }
  // grid-stride loop, four strides per pass so 12 loads are in flight
  constexpr int U = 4;
  const size_t stride = (size_t)gridDim.x * kNT * VEC;
  for (size_t e0 = ((size_t)blockIdx.x * kNT + t) * VEC; e0 < g.nelem; e0 += U * stride) {
    double rv[U][VEC], qv[U][VEC], dv[U][VEC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t e = e0 + u * stride;
      if (e < g.nelem) {
        ld<VEC>(rv[u], a.r + e);
        ld<VEC>(qv[u], a.q + e);
        ld<VEC>(dv[u], a.V + 4 * g.nelem + e);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t e = e0 + u * stride;
      if (e >= g.nelem) break;
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        if (act[c] != 0.0 && alpha[c] != 0.0) rv[u][c] = fma(-alpha[c], qv[u][c], rv[u][c]);
        rr[c] = fma(rv[u][c], rv[u][c], rr[c]);
      }
      st<VEC>(a.r + e, rv[u]);
      if constexpr (!CHEB) {
#pragma unroll
        for (int c = 0; c < VEC; ++c) rz[c] = fma(rv[u][c], rv[u][c] / dv[u][c], rz[c]);
      } else {
        double zz[VEC];
#pragma unroll
        for (int c = 0; c < VEC; ++c) zz[c] = (rv[u][c] / dv[u][c]) / ith[c];
        st<VEC>(a.d + e, zz);
        st<VEC>(a.z + e, zz);
      }
    }
  }
  const size_t pstride = (size_t)gridDim.x * S;
  group_reduce<VEC>(rr, tpp, red);
  put_partial<VEC>(a.partial + pstride, S, tpp, rr);
  if constexpr (!CHEB) {
    group_reduce<VEC>(rz, tpp, red);
    put_partial<VEC>(a.partial, S, tpp, rz);
  }
}

// ------------------------------------------------------------ init / final
// x = 0, p_0 = 0, r = b; per member ||b||, r^T D^-1 r (Jacobi) or the
// Gershgorin bound max_i sum_j |a_ij| / a_ii (row sums left to right in
// column order) with the Chebyshev coefficients of the member.
template <int VEC>
__global__ __launch_bounds__(kNT) void init_kernel(InitArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  const Geometry& g = a.g;
  const int S = g.S, tpp = g.tpp, t = threadIdx.x;
  double rz[VEC], bb[VEC], gm[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) rz[c] = bb[c] = gm[c] = 0.0;
  const size_t stride = (size_t)gridDim.x * kNT * VEC;
  for (size_t e = ((size_t)blockIdx.x * kNT + t) * VEC; e < g.nelem; e += stride) {
    double bv[VEC], dv[VEC], zero[VEC];
    if (a.b_broadcast) {
#pragma unroll
      for (int c = 0; c < VEC; ++c) bv[c] = a.b[(e + c) >> g.logS];
    } else {
      ld<VEC>(bv, a.b + e);
    }
    ld<VEC>(dv, a.V + 4 * g.nelem + e);
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      zero[c] = 0.0;
      bb[c] = fma(bv[c], bv[c], bb[c]);
      if (!a.cheb) rz[c] = fma(bv[c], bv[c] / dv[c], rz[c]);
    }
    st<VEC>(a.x + e, zero);
    st<VEC>(a.p0 + e, zero);
    st<VEC>(a.r + e, bv);
    if (a.cheb) {
      double rs[VEC];
#pragma unroll
      for (int c = 0; c < VEC; ++c) rs[c] = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        double vk[VEC];
        ld<VEC>(vk, a.V + (size_t)k * g.nelem + e);
#pragma unroll
        for (int c = 0; c < VEC; ++c) rs[c] = rs[c] + fabs(vk[c]);
      }
#pragma unroll
      for (int c = 0; c < VEC; ++c) gm[c] = fmax(gm[c], rs[c] / dv[c]);
    }
  }
  const size_t ps = (size_t)gridDim.x * S;
  group_reduce<VEC>(bb, tpp, red);
  put_partial<VEC>(a.partial + ps, S, tpp, bb);
  if (!a.cheb) {
    group_reduce<VEC>(rz, tpp, red);
    put_partial<VEC>(a.partial, S, tpp, rz);
  } else {
    group_max<VEC>(gm, tpp, red);
    put_partial<VEC>(a.partial + 2 * ps, S, tpp, gm);
  }
}

// Chebyshev: d = z = D^-1 r / theta for every member (start of an application)
template <int VEC>
__global__ __launch_bounds__(kNT) void cheb_start_kernel(const double* V, const double* r, double* d,
                                                         double* z, Members m, Geometry g) {
  const int t = threadIdx.x, sv = (t % g.tpp) * VEC;
  double ith[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) ith[c] = m.cheb[(size_t)(sv + c) * kChebCoef];
  const size_t stride = (size_t)gridDim.x * kNT * VEC;
  for (size_t e = ((size_t)blockIdx.x * kNT + t) * VEC; e < g.nelem; e += stride) {
    double rv[VEC], dv[VEC], zz[VEC];
    ld<VEC>(rv, r + e);
    ld<VEC>(dv, V + 4 * g.nelem + e);
#pragma unroll
    for (int c = 0; c < VEC; ++c) zz[c] = (rv[c] / dv[c]) / ith[c];
    st<VEC>(d + e, zz);
    st<VEC>(z + e, zz);
  }
}

// the deferred x += alpha p of the last iteration
template <int VEC>
__global__ __launch_bounds__(kNT) void final_kernel(double* x, const double* p0, const double* p1,
                                                    Members m, Geometry g) {
  const int t = threadIdx.x, sv = (t % g.tpp) * VEC;
  const double* p = (m.ctl[CTL_K] & 1) ? p1 : p0;
  double ap[VEC];
  bool any = false;
#pragma unroll
  for (int c = 0; c < VEC; ++c) {
    ap[c] = m.alpha_prev[sv + c];
    any |= (ap[c] != 0.0);
  }
  if (!any) return;
  const size_t stride = (size_t)gridDim.x * kNT * VEC;
  for (size_t e = ((size_t)blockIdx.x * kNT + t) * VEC; e < g.nelem; e += stride) {
    double xv[VEC], pv[VEC];
    ld<VEC>(xv, x + e);
    ld<VEC>(pv, p + e);
#pragma unroll
    for (int c = 0; c < VEC; ++c)
      if (ap[c] != 0.0) xv[c] = fma(ap[c], pv[c], xv[c]);
    st<VEC>(x + e, xv);
  }
}

// per-member dot products (b optionally broadcast over members)
template <int VEC>
__global__ __launch_bounds__(kNT) void dot_kernel(const double* x, const double* y, int y_bcast,
                                                  double* partial, Geometry g) {
  __shared__ double red[kWaves * 64 * 2];
  const int t = threadIdx.x, S = g.S, tpp = g.tpp;
  double acc[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) acc[c] = 0.0;
  const size_t stride = (size_t)gridDim.x * kNT * VEC;
  for (size_t e = ((size_t)blockIdx.x * kNT + t) * VEC; e < g.nelem; e += stride) {
    double xv[VEC], yv[VEC];
    ld<VEC>(xv, x + e);
    if (y_bcast) {
#pragma unroll
      for (int c = 0; c < VEC; ++c) yv[c] = y[(e + c) >> g.logS];
    } else {
      ld<VEC>(yv, y + e);
    }
#pragma unroll
    for (int c = 0; c < VEC; ++c) acc[c] = fma(xv[c], yv[c], acc[c]);
  }
  group_reduce<VEC>(acc, tpp, red);
  put_partial<VEC>(partial, S, tpp, acc);
}


// ------------------------------------------------------------ finish
// One workgroup, launched right after a producer kernel: reduces the
// producer's per-workgroup partials in a fixed order and applies the
// per-member scalar logic of the step.
template <int VEC>
__global__ __launch_bounds__(kNT) void finish_kernel(FinishArgs a) {
  __shared__ double fin[2 * kNT * 2];
  __shared__ int live;
  const int S = a.g.S, t = threadIdx.x;
  const Members& m = a.m;
  const size_t ps = (size_t)a.G * S;
  if (a.kind != F_INIT && a.kind != F_DOT && a.kind != F_SUMS) {
    if (m.ctl[CTL_DONE]) return;
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
      return;
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
      return;
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
      if (t == 0) {
        m.ctl[CTL_K] = k;
        m.ctl[CTL_DONE] = (live == 0) ? 1 : 0;
      }
      return;
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
      return;
    }
    case F_DOT:
    case F_SUMS: {
      // nsum member sums, scaled, into result[s][q]
      for (int q = 0; q < a.nsum; ++q) {
        const double v = final_sum<VEC>(a.partial + q * ps, a.G, S, fin);
        if (t < S) m.result[(size_t)t * 16 + q] = a.scale * v;
      }
      return;
    }
  }
}

// ------------------------------------------------------------ launchers
#define ENS_LAUNCH_VEC(vec, kern, grid, stream, ...)                        \
  do {                                                                       \
    if ((vec) == 2) hipLaunchKernelGGL(kern<2>, grid, dim3(kNT), 0, stream, __VA_ARGS__); \
    else hipLaunchKernelGGL(kern<1>, grid, dim3(kNT), 0, stream, __VA_ARGS__); \
  } while (0)

void launch_assemble(const AsmArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.nelem + kNT - 1) / kNT);
  hipLaunchKernelGGL(assemble_kernel, dim3(blocks), dim3(kNT), 0, s, a);
}

template <int MODE>
void launch_stencil(const StencilArgs& a, hipStream_t s) {
  if (a.g.vec == 2) hipLaunchKernelGGL((stencil_kernel<2, MODE>), dim3(a.g.groups), dim3(kNT), 0, s, a);
  else hipLaunchKernelGGL((stencil_kernel<1, MODE>), dim3(a.g.groups), dim3(kNT), 0, s, a);
}
template void launch_stencil<M_SPMV>(const StencilArgs&, hipStream_t);
template void launch_stencil<M_PCG_J>(const StencilArgs&, hipStream_t);
template void launch_stencil<M_PCG_Z>(const StencilArgs&, hipStream_t);
template void launch_stencil<M_CHEB>(const StencilArgs&, hipStream_t);

void launch_update(const UpdateArgs& a, bool cheb, int groups, hipStream_t s) {
  if (a.g.vec == 2) {
    if (cheb) hipLaunchKernelGGL((update_kernel<2, true>), dim3(groups), dim3(kNT), 0, s, a);
    else hipLaunchKernelGGL((update_kernel<2, false>), dim3(groups), dim3(kNT), 0, s, a);
  } else {
    if (cheb) hipLaunchKernelGGL((update_kernel<1, true>), dim3(groups), dim3(kNT), 0, s, a);
    else hipLaunchKernelGGL((update_kernel<1, false>), dim3(groups), dim3(kNT), 0, s, a);
  }
}

void launch_init(const InitArgs& a, int groups, hipStream_t s) {
  ENS_LAUNCH_VEC(a.g.vec, init_kernel, dim3(groups), s, a);
}

void launch_cheb_start(const double* V, const double* r, double* d, double* z, const Members& m,
                       const Geometry& g, int groups, hipStream_t s) {
  ENS_LAUNCH_VEC(g.vec, cheb_start_kernel, dim3(groups), s, V, r, d, z, m, g);
}

void launch_final(double* x, const double* p0, const double* p1, const Members& m,
                  const Geometry& g, int groups, hipStream_t s) {
  ENS_LAUNCH_VEC(g.vec, final_kernel, dim3(groups), s, x, p0, p1, m, g);
}

void launch_finish(const FinishArgs& a, hipStream_t s) {
  ENS_LAUNCH_VEC(a.g.vec, finish_kernel, dim3(1), s, a);
}

void launch_dot(const double* x, const double* y, int y_bcast, double* partial, const Geometry& g,
                int groups, hipStream_t s) {
  ENS_LAUNCH_VEC(g.vec, dot_kernel, dim3(groups), s, x, y, y_bcast, partial, g);
}

}  // namespace ens
