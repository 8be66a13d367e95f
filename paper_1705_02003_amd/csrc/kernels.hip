// HIP kernels of the ensemble PCG hot path for CDNA4 (gfx950).
//
// Data layout: member index innermost (paper, Section 2.3, commuted Kronecker
// ordering): vectors X[r * S + s], matrix values V[(k * N_r + r) * S + s].
// A grid point's S members are contiguous, so every load and store moves
// whole 8*S-byte runs, and the stencil structure (the shared sparsity
// pattern) is implicit: there is no index array at all, it is "read" once
// per tile for all S members (Section 2.3, reuse of sample-independent data).
//
// Thread mapping: VEC = 2 members per thread (one 16-byte load) when S is
// even, else VEC = 1.  A power-of-two group of tpp >= S / VEC threads covers
// one grid point (slots past S are idle lanes); a wave64 covers 64 / tpp
// consecutive points of one grid line.  The element-wise kernels stride over
// points: thread t of workgroup b handles points b P + t / tpp + k G P
// (P = kNT / tpp points per workgroup, G workgroups) and slots
// (t % tpp) VEC .. + VEC - 1.
//
// Reductions: every per-member inner product is reduced in a fixed tree
// (per-thread sequential sums, xor-shuffles across lanes that hold the same
// members, a fixed-order sum across the four waves, then a fixed-order sum
// over the workgroup partials in a one-workgroup finishing kernel).  The tree does
// not depend on the member index, so results are deterministic and
// permuting members permutes results bit for bit.  No floating-point
// atomics are used.
#include <algorithm>
#include <cmath>

#include "device.h"

namespace ens {

// ------------------------------------------------------------ assembly
// One workgroup per tile of kAsmTX x kAsmTY grid points, for the members
// m0 .. m0 + mc - 1 of one launch.  What does not depend on the member is
// computed once per tile: the mode tables sin(k pi I h) at the tile's node
// columns I and rows J (paper, Section 2.3: sample-independent quantities
// are computed once for the whole ensemble); what depends only on the
// member once per member and tile: the entries of K(eps, theta) and the mode
// weights amp y_{k+1} / k^2.  Then every (point, member) forms a at its node
// and the four neighbours as 1 + sum_k weight_k sin(k pi x1) sin(k pi x2)
// from the tables, the face means and the nine values.  No division is left
// in the per-element work.  Contraction into FMA is off so every product
// and sum is the plainly rounded one.
__global__ __launch_bounds__(kNT) void assemble_kernel(AsmArgs a) {
#pragma clang fp contract(off)
  __shared__ double sI[kMaxModes][kAsmTX + 2];
  __shared__ double sJ[kMaxModes][kAsmTY + 2];
  __shared__ double kc[3][kMaxS];
  __shared__ double wk[kMaxS][kMaxModes];
  __shared__ double ys[kAsmY];
  const int n = a.n, d = a.d, t = threadIdx.x, nm = a.d - 2;
  for (int x = t; x < a.mc * d; x += kNT) ys[x] = a.y[x];
  const int i0 = (blockIdx.x % a.ntx) * kAsmTX, j0 = (blockIdx.x / a.ntx) * kAsmTY;
  const double np1 = (double)(n + 1);
  // sin(k pi x) at nodes I = i0 + q (q = 0 .. kAsmTX + 1) and J = j0 + q
  for (int x = t; x < nm * (kAsmTX + 2); x += kNT) {
    const int k = x / (kAsmTX + 2), q = x % (kAsmTX + 2);
    const double kp = (double)(k + 1) * M_PI;
    sI[k][q] = sin(kp * ((double)(i0 + q) / np1));
  }
  for (int x = t; x < nm * (kAsmTY + 2); x += kNT) {
    const int k = x / (kAsmTY + 2), q = x % (kAsmTY + 2);
    const double kp = (double)(k + 1) * M_PI;
    sJ[k][q] = sin(kp * ((double)(j0 + q) / np1));
  }
  __syncthreads();
  for (int x = t; x < a.mc * nm; x += kNT) {
    const int m = x / nm, k = x % nm + 1;
    wk[m][k - 1] = (a.amp * ys[m * d + k + 1]) / (double)(k * k);
  }
  if (t < a.mc) {
    const double* y = ys + t * d;
    const double eps = (a.eps_model == 0) ? pow(10.0, -(1.0 + y[0])) : pow(10.0, -(1.5 + 1.5 * y[0]));
    const double theta = (M_PI / 4.0) * (1.0 + y[1]);
    const double c = cos(theta), sn = sin(theta);
    kc[0][t] = c * c + eps * (sn * sn);
    kc[1][t] = sn * sn + eps * (c * c);
    kc[2][t] = (1.0 - eps) * (sn * c);
  }
  __syncthreads();
  const int cl = t % a.mcp;
  if (cl >= a.mc) return;
  const double k11 = kc[0][cl], k22 = kc[1][cl], k12 = kc[2][cl];
  const double inv_h2 = np1 * np1;
  for (int pt = t / a.mcp; pt < kAsmTX * kAsmTY; pt += kNT / a.mcp) {
    const int i = i0 + pt % kAsmTX, j = j0 + pt / kAsmTX;
    if (i >= n || j >= n) continue;
    // table columns of the nodes i, i + 1, i + 2 (1-based node I = i + 1)
    const int qi = i - i0 + 1, qj = j - j0 + 1;
    double aC = 1.0, aE = 1.0, aW = 1.0, aN = 1.0, aS = 1.0;
    for (int k = 0; k < nm; ++k) {
      const double sIm = sI[k][qi - 1], sIc = sI[k][qi], sIp = sI[k][qi + 1];
      const double sJm = sJ[k][qj - 1], sJc = sJ[k][qj], sJp = sJ[k][qj + 1];
      const double w = wk[cl][k];
      aC = aC + w * (sJc * sIc);
      aE = aE + w * (sJc * sIp);
      aW = aW + w * (sJc * sIm);
      aN = aN + w * (sJp * sIc);
      aS = aS + w * (sJm * sIc);
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
    const size_t e = ((size_t)j * n + i) * a.S + a.m0 + cl;
#pragma unroll
    for (int k = 0; k < 9; ++k) a.V[(size_t)k * a.vstride + e] = h2[k] * inv_h2;
    a.b[e] = 1.0;
  }
}

// ------------------------------------------------------------ stencil
// Fused tile kernel.  A tile is tx grid points of one line chunk times ty
// lines.  The tile is swept line by line; the values the stencil reads
// (M_PCG_J: the new direction p = r / diag + beta p_old; M_PCG_Z: p = z +
// beta p_old; M_SPMV: p; M_CHEB: z) are formed once per point, including a
// one-point halo, into a four-line LDS ring, so each line needs one barrier.
// Then, per point and member, the nine-point product is taken from the ring
// and the mode's fused updates follow:
//   M_PCG_*: store p and q = A p, accumulate p^T q, apply the deferred
//            x += alpha_prev p_old (the finishing kernel then turns p^T q
//            into alpha, or freezes a member whose p^T A p is not a positive
//            finite number -- the paper's guard).
//   M_CHEB:  one Chebyshev step d = c1 d_prev + c2 D^-1 (r - A z), z += d,
//            with d_prev taken from the z iterates rather than stored; the
//            last step accumulates r^T z.
template <int VEC, int MODE, bool SYM>
__global__ __launch_bounds__(kNT) void stencil_kernel(StencilArgs a) {
  __shared__ __attribute__((aligned(16))) double ring[4][kRing];
  __shared__ __attribute__((aligned(16))) double sym[SYM ? 6 * kRing : 2];
  __shared__ double red[kWaves * 64 * 2];
  const Geometry& g = a.g;
  if constexpr (MODE != M_SPMV) {
    if (a.m.ctl[CTL_DONE]) return;
  }
  const int t = threadIdx.x;
  const int tpp = g.stpp;
  TileView tv;
  tv.swp = g.swp;
  tv.V = a.V;
  tv.r = a.r;
  tv.src = a.src;
  tv.pold = a.pold;
  tv.pnew = a.pnew;
  tv.q = a.q;
  tv.x = a.x;
  tv.zout = a.zout;
  tv.zprev = a.zprev;
  tv.q_in = a.q_in;
  tv.r_out = a.r_out;
  tv.n = g.n;
  tv.S = g.S;
  tv.tpp = tpp;
  tv.tx = g.tx;
  tv.ty = g.ty;
  tv.nchunk = g.nchunk;
  tv.nelem = g.nelem;
  tv.vstride = g.vstride;
  tv.cheb_step = a.cheb_step;
  tv.cheb_last = a.cheb_last;
  // Every workgroup sweeps the same spatial tiles for each member tile, so
  // each member's partial sums follow the same tree.
  for (int js = 0; js < g.nstile; ++js) {
    tv.s0 = js * g.sw;
    tv.sw = min(g.sw, g.S - tv.s0);
    const int sv = tv.s0 + (t % tpp) * VEC;   // member slot (< Sp)
    double beta[VEC], aprev[VEC], c1[VEC], c2[VEC], acc[VEC], acc2[VEC];
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      beta[c] = 0.0;
      aprev[c] = 0.0;
      c1[c] = 0.0;
      c2[c] = 0.0;
      acc[c] = 0.0;
      acc2[c] = 0.0;
      if constexpr (MODE == M_PCG_J || MODE == M_PCG_Z) {
        beta[c] = a.m.beta[sv + c];
        aprev[c] = a.m.alpha_prev[sv + c];
      }
      if constexpr (MODE == M_CHEB1) {
        // alpha of active members
        beta[c] = a.m.active[sv + c] ? a.m.alpha[sv + c] : 0.0;
      }
      if constexpr (MODE == M_CHEB || MODE == M_CHEB1) {
        aprev[c] = a.m.cheb[(size_t)(sv + c) * kChebCoef];   // theta
        c1[c] = a.m.cheb[(size_t)(sv + c) * kChebCoef + 2 * a.cheb_step - 1];
        c2[c] = a.m.cheb[(size_t)(sv + c) * kChebCoef + 2 * a.cheb_step];
      }
    }
    int tile, tstep, tend;
    tile_range(g, tile, tstep, tend);
    if (MODE == M_CHEB && a.cheb_step >= 3) {
      for (; tile < tend; tile += tstep)
        stencil_tile<VEC, MODE, SYM, true>(tv, tile, ring, sym, beta, aprev, c1, c2, acc, acc2);
    } else {
      for (; tile < tend; tile += tstep)
        stencil_tile<VEC, MODE, SYM>(tv, tile, ring, sym, beta, aprev, c1, c2, acc, acc2);
    }
    if constexpr (MODE == M_PCG_J || MODE == M_PCG_Z) {
      group_reduce<VEC>(acc, tpp, red);
      put_partial<VEC>(a.partial, g.Sp, tpp, acc, tv.s0);
    } else if constexpr (MODE == M_CHEB) {
      if (a.cheb_last) {
        group_reduce<VEC>(acc, tpp, red);
        put_partial<VEC>(a.partial, g.Sp, tpp, acc, tv.s0);
      }
    } else if constexpr (MODE == M_CHEB1) {
      // r^T r into the second partial array (the convergence test), r^T z
      // into the first when this is the application's last step
      group_reduce<VEC>(acc, tpp, red);
      put_partial<VEC>(a.partial + (size_t)gridDim.x * g.Sp, g.Sp, tpp, acc, tv.s0);
      if (a.cheb_last) {
        group_reduce<VEC>(acc2, tpp, red);
        put_partial<VEC>(a.partial, g.Sp, tpp, acc2, tv.s0);
      }
    }
  }
}

// ------------------------------------------------------------ update
// r -= alpha q for active members; then (Jacobi) z = D^-1 r and partial
// r^T z, r^T r, or (Chebyshev, the 3-D model and multigrid) the start of the
// preconditioner application z_0 = D^-1 r / theta and partial r^T r.  The
// finishing kernel then applies the convergence test ||r_k|| <= rtol ||b||
// per member, records the member's iteration count, forms beta (Jacobi) and
// raises the done flag when no member is active.
template <int VEC, bool CHEB>
__global__ __launch_bounds__(kNT) void update_kernel(UpdateArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  if (a.m.ctl[CTL_DONE]) return;
  const Geometry& g = a.g;
  const int S = g.S, tpp = g.tpp;
  const int t = threadIdx.x;
  const int sv = (t % tpp) * VEC;
  const bool lane_ok = sv < S;
  double alpha[VEC], act[VEC], ith[VEC], rz[VEC], rr[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) {
    act[c] = a.m.active[sv + c] ? 1.0 : 0.0;
    alpha[c] = a.m.alpha[sv + c];
    ith[c] = CHEB ? a.m.cheb[(size_t)(sv + c) * kChebCoef] : 0.0;
    rz[c] = 0.0;
    rr[c] = 0.0;
  }
  // point-strided loop, four strides per pass so 12 loads are in flight
  constexpr int U = 4;
  const size_t P = (size_t)(kNT / tpp);
  const size_t stride = (size_t)gridDim.x * P;
  const double* diag = a.V + (size_t)g.cslot * g.vstride;
  for (size_t p0 = (size_t)blockIdx.x * P + t / tpp; lane_ok && p0 < g.nr; p0 += U * stride) {
    double rv[U][VEC], qv[U][VEC], dv[U][VEC];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t p = p0 + u * stride;
      if (p < g.nr) {
        const size_t e = p * S + sv;
        ld<VEC>(rv[u], a.r + e);
        ld<VEC>(qv[u], a.q + e);
        ld<VEC>(dv[u], diag + e);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t p = p0 + u * stride;
      if (p >= g.nr) break;
      const size_t e = p * S + sv;
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
        st<VEC>(a.z + e, zz);
      }
    }
  }
  const size_t pstride = (size_t)gridDim.x * g.Sp;
  group_reduce<VEC>(rr, tpp, red);
  put_partial<VEC>(a.partial + pstride, g.Sp, tpp, rr);
  if constexpr (!CHEB) {
    group_reduce<VEC>(rz, tpp, red);
    put_partial<VEC>(a.partial, g.Sp, tpp, rz);
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
  const int sv = (t % tpp) * VEC;
  const bool lane_ok = sv < S;
  double rz[VEC], bb[VEC], gm[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) rz[c] = bb[c] = gm[c] = 0.0;
  const size_t P = (size_t)(kNT / tpp);
  const size_t stride = (size_t)gridDim.x * P;
  for (size_t p = (size_t)blockIdx.x * P + t / tpp; lane_ok && p < g.nr; p += stride) {
    const size_t e = p * S + sv;
    double bv[VEC], dv[VEC], zero[VEC];
    if (a.b_broadcast) {
#pragma unroll
      for (int c = 0; c < VEC; ++c) bv[c] = a.b[p];
    } else {
      ld<VEC>(bv, a.b + e);
    }
    ld<VEC>(dv, a.V + (size_t)g.cslot * g.vstride + e);
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
      for (int k = 0; k < g.nslot; ++k) {
        double vk[VEC];
        ld<VEC>(vk, a.V + (size_t)k * g.vstride + e);
#pragma unroll
        for (int c = 0; c < VEC; ++c) rs[c] = rs[c] + fabs(vk[c]);
      }
#pragma unroll
      for (int c = 0; c < VEC; ++c) gm[c] = fmax(gm[c], rs[c] / dv[c]);
    }
  }
  const size_t ps = (size_t)gridDim.x * g.Sp;
  group_reduce<VEC>(bb, tpp, red);
  put_partial<VEC>(a.partial + ps, g.Sp, tpp, bb);
  if (!a.cheb) {
    group_reduce<VEC>(rz, tpp, red);
    put_partial<VEC>(a.partial, g.Sp, tpp, rz);
  } else {
    group_max<VEC>(gm, tpp, red);
    put_partial<VEC>(a.partial + 2 * ps, g.Sp, tpp, gm);
  }
}

// Chebyshev: z_0 = D^-1 r / theta for every member (start of an application;
// the first step's increment d_0 is z_0 itself)
template <int VEC>
__global__ __launch_bounds__(kNT) void cheb_start_kernel(const double* V, const double* r,
                                                         double* z, Members m, Geometry g) {
  const int t = threadIdx.x, sv = (t % g.tpp) * VEC;
  if (sv >= g.S) return;
  double ith[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) ith[c] = m.cheb[(size_t)(sv + c) * kChebCoef];
  const size_t P = (size_t)(kNT / g.tpp);
  const size_t stride = (size_t)gridDim.x * P;
  for (size_t p = (size_t)blockIdx.x * P + t / g.tpp; p < g.nr; p += stride) {
    const size_t e = p * g.S + sv;
    double rv[VEC], dv[VEC], zz[VEC];
    ld<VEC>(rv, r + e);
    ld<VEC>(dv, V + (size_t)g.cslot * g.vstride + e);
#pragma unroll
    for (int c = 0; c < VEC; ++c) zz[c] = (rv[c] / dv[c]) / ith[c];
    st<VEC>(z + e, zz);
  }
}

// the deferred x += alpha p of the last iteration
template <int VEC>
__global__ __launch_bounds__(kNT) void final_kernel(double* x, const double* p0, const double* p1,
                                                    Members m, Geometry g) {
  const int t = threadIdx.x, sv = (t % g.tpp) * VEC;
  if (sv >= g.S) return;
  const double* p = (m.ctl[CTL_K] & 1) ? p1 : p0;
  double ap[VEC];
  bool any = false;
#pragma unroll
  for (int c = 0; c < VEC; ++c) {
    ap[c] = m.alpha_prev[sv + c];
    any |= (ap[c] != 0.0);
  }
  if (!any) return;
  const size_t P = (size_t)(kNT / g.tpp);
  const size_t stride = (size_t)gridDim.x * P;
  for (size_t q = (size_t)blockIdx.x * P + t / g.tpp; q < g.nr; q += stride) {
    const size_t e = q * g.S + sv;
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
  const int sv = (t % tpp) * VEC;
  const bool lane_ok = sv < S;
  double acc[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) acc[c] = 0.0;
  const size_t P = (size_t)(kNT / tpp);
  const size_t stride = (size_t)gridDim.x * P;
  for (size_t p = (size_t)blockIdx.x * P + t / tpp; lane_ok && p < g.nr; p += stride) {
    const size_t e = p * S + sv;
    double xv[VEC], yv[VEC];
    ld<VEC>(xv, x + e);
    if (y_bcast) {
#pragma unroll
      for (int c = 0; c < VEC; ++c) yv[c] = y[p];
    } else {
      ld<VEC>(yv, y + e);
    }
#pragma unroll
    for (int c = 0; c < VEC; ++c) acc[c] = fma(xv[c], yv[c], acc[c]);
  }
  group_reduce<VEC>(acc, tpp, red);
  put_partial<VEC>(partial, g.Sp, tpp, acc);
}


// ------------------------------------------------------------ finish
// One workgroup, launched right after a producer kernel: reduces the
// producer's per-workgroup partials in a fixed order and applies the
// per-member scalar logic of the step.
template <int VEC>
__global__ __launch_bounds__(kFinNT) void finish_kernel(FinishArgs a) {
  __shared__ double fin[2 * kFinNT * 2];
  __shared__ int live;
  (void)finish_body<VEC>(a, fin, live);
}

// ------------------------------------------------------------ launchers
#define ENS_LAUNCH_VEC(vec, kern, grid, stream, ...)                        \
  do {                                                                       \
    if ((vec) == 2) hipLaunchKernelGGL(kern<2>, grid, dim3(kNT), 0, stream, __VA_ARGS__); \
    else hipLaunchKernelGGL(kern<1>, grid, dim3(kNT), 0, stream, __VA_ARGS__); \
  } while (0)

void launch_assemble(const AsmArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)a.ntx * (unsigned)((a.n + kAsmTY - 1) / kAsmTY);
  hipLaunchKernelGGL(assemble_kernel, dim3(blocks), dim3(kNT), 0, s, a);
}

template <int MODE>
void launch_stencil(const StencilArgs& a, hipStream_t s) {
  if constexpr (MODE != M_CHEB1) {   // the 3-D model has no fused first step
    if (a.g.dim == 3) {
      launch_fe3d<MODE>(a, s);
      return;
    }
  }
  const dim3 grid(a.g.groups), block(kNT);
  if (a.g.vec == 2) {
    if (a.g.full) hipLaunchKernelGGL((stencil_kernel<2, MODE, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((stencil_kernel<2, MODE, true>), grid, block, 0, s, a);
  } else {
    if (a.g.full) hipLaunchKernelGGL((stencil_kernel<1, MODE, false>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((stencil_kernel<1, MODE, true>), grid, block, 0, s, a);
  }
}
template void launch_stencil<M_SPMV>(const StencilArgs&, hipStream_t);
template void launch_stencil<M_PCG_J>(const StencilArgs&, hipStream_t);
template void launch_stencil<M_PCG_Z>(const StencilArgs&, hipStream_t);
template void launch_stencil<M_CHEB>(const StencilArgs&, hipStream_t);
template void launch_stencil<M_CHEB1>(const StencilArgs&, hipStream_t);

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

void launch_cheb_start(const double* V, const double* r, double* z, const Members& m,
                       const Geometry& g, int groups, hipStream_t s) {
  ENS_LAUNCH_VEC(g.vec, cheb_start_kernel, dim3(groups), s, V, r, z, m, g);
}

void launch_final(double* x, const double* p0, const double* p1, const Members& m,
                  const Geometry& g, int groups, hipStream_t s) {
  ENS_LAUNCH_VEC(g.vec, final_kernel, dim3(groups), s, x, p0, p1, m, g);
}

void launch_finish(const FinishArgs& a, hipStream_t s) {
  if (a.g.vec == 2) hipLaunchKernelGGL(finish_kernel<2>, dim3(1), dim3(kFinNT), 0, s, a);
  else hipLaunchKernelGGL(finish_kernel<1>, dim3(1), dim3(kFinNT), 0, s, a);
}

void launch_dot(const double* x, const double* y, int y_bcast, double* partial, const Geometry& g,
                int groups, hipStream_t s) {
  ENS_LAUNCH_VEC(g.vec, dot_kernel, dim3(groups), s, x, y, y_bcast, partial, g);
}

}  // namespace ens
