// dQ/dy kernel: -lambda^T (dA/dy_j) u per member, from the coefficient
// derivatives of the nine-point scheme.
//
// With D+ the difference across a face and D0 the undivided central
// difference at a node (lambda = u = 0 on boundary nodes),
//   h^2 lambda^T A u = sum_{x-faces} k11 a_f (D+ lambda)(D+ u)
//                    + sum_{y-faces} k22 a_f (D+ lambda)(D+ u)
//                    + sum_{nodes} (k12 a / 4) [(D0_1 lambda)(D0_2 u) + (D0_2 lambda)(D0_1 u)],
// so dQ/dy_j = -lambda^T (dA/dy_j) u replaces (k11, k22, k12, a) by their
// derivatives: d eps/d y1 = -c ln10 eps (c = 1 or 1.5 by model),
// d(k11,k22,k12)/d eps = (s^2, c^2, -s c); d theta/d y2 = pi/4,
// d(k11,k22,k12)/d theta = (1-eps)(-sin 2theta, sin 2theta, cos 2theta);
// d a/d y_{k+2} = amp sin(k pi x1) sin(k pi x2) / k^2.
// Each interior node owns its east and north faces, plus its west (south)
// face when it is the first node of its line (column).
#include <cmath>

#include "common.h"

namespace ens {

typedef double d2 __attribute__((ext_vector_type(2)));

namespace {

template <int VEC>
__device__ __forceinline__ void ldv(double (&v)[VEC], const double* p) {
  if constexpr (VEC == 2) {
    const d2 t = *reinterpret_cast<const d2*>(p);
    v[0] = t.x;
    v[1] = t.y;
  } else {
    v[0] = *p;
  }
}

template <int VEC>
__device__ __forceinline__ void reduce_group(double (&v)[VEC], int tpp, double* lds) {
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

}  // namespace

constexpr int kMaxD = 16;

// Tiles of kAsmTX x kAsmTY grid points, grid-strided over the workgroups.
// Per tile the mode tables sin(k pi I h) at the tile's node columns and rows
// are computed once and shared by every point and member of the tile (the
// sample-independent part of the form); per (point, member) the five a
// values and their mode derivatives follow from the tables.
template <int VEC>
__global__ __launch_bounds__(kNT) void dqdy_kernel(DqdyArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  __shared__ double sI[kMaxModes][kAsmTX + 2];
  __shared__ double sJ[kMaxModes][kAsmTY + 2];
  const Geometry& g = a.g;
  const int S = g.S, n = g.n, tpp = g.tpp, t = threadIdx.x, d = a.d, nm = a.d - 2;
  const int sv = (t % tpp) * VEC;
  const bool lane_ok = sv < S;
  const int svl = lane_ok ? sv : S - VEC;   // idle slots compute on real members, add nothing

  // per-member coefficients and their derivatives
  double k11[VEC], k22[VEC], k12[VEC], dk[2][3][VEC], ym[VEC][kMaxD];
#pragma unroll
  for (int c = 0; c < VEC; ++c) {
    const double* y = a.y + (size_t)(svl + c) * d;
#pragma unroll
    for (int q = 0; q < kMaxD; ++q) ym[c][q] = (q < d) ? y[q] : 0.0;
    const double eps = (a.eps_model == 0) ? pow(10.0, -(1.0 + y[0])) : pow(10.0, -(1.5 + 1.5 * y[0]));
    const double th = (M_PI / 4.0) * (1.0 + y[1]);
    const double co = cos(th), si = sin(th);
    k11[c] = co * co + eps * (si * si);
    k22[c] = si * si + eps * (co * co);
    k12[c] = (1.0 - eps) * (si * co);
    const double deps = -((a.eps_model == 0) ? 1.0 : 1.5) * log(10.0) * eps;
    dk[0][0][c] = si * si * deps;
    dk[0][1][c] = co * co * deps;
    dk[0][2][c] = -si * co * deps;
    const double dth = M_PI / 4.0, s2 = sin(2.0 * th), c2 = cos(2.0 * th);
    dk[1][0][c] = -(1.0 - eps) * s2 * dth;
    dk[1][1][c] = (1.0 - eps) * s2 * dth;
    dk[1][2][c] = (1.0 - eps) * c2 * dth;
  }
  double acc[kMaxD][VEC];
#pragma unroll
  for (int q = 0; q < kMaxD; ++q)
#pragma unroll
    for (int c = 0; c < VEC; ++c) acc[q][c] = 0.0;

  const double np1 = (double)(n + 1);
  const size_t rS = (size_t)S;
  for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
    const int i0 = (tile % a.ntx) * kAsmTX, j0 = (tile / a.ntx) * kAsmTY;
    __syncthreads();   // the previous tile's readers are done with the tables
    for (int x = t; x < nm * (kAsmTX + 2); x += kNT) {
      const int k = x / (kAsmTX + 2), q = x % (kAsmTX + 2);
      sI[k][q] = sin((double)(k + 1) * M_PI * ((double)(i0 + q) / np1));
    }
    for (int x = t; x < nm * (kAsmTY + 2); x += kNT) {
      const int k = x / (kAsmTY + 2), q = x % (kAsmTY + 2);
      sJ[k][q] = sin((double)(k + 1) * M_PI * ((double)(j0 + q) / np1));
    }
    __syncthreads();
    if (!lane_ok) continue;
    for (int pt = t / tpp; pt < kAsmTX * kAsmTY; pt += kNT / tpp) {
      const int i = i0 + pt % kAsmTX, j = j0 + pt / kAsmTX;
      if (i >= n || j >= n) continue;
      const size_t e = ((size_t)j * n + i) * rS + sv;
      double uC[VEC], uE[VEC], uW[VEC], uN[VEC], uS[VEC];
      double lC[VEC], lE[VEC], lW[VEC], lN[VEC], lS[VEC];
      ldv<VEC>(uC, a.u + e);
      ldv<VEC>(lC, a.lam + e);
#pragma unroll
      for (int c = 0; c < VEC; ++c) uE[c] = uW[c] = uN[c] = uS[c] = lE[c] = lW[c] = lN[c] = lS[c] = 0.0;
      if (i + 1 < n) { ldv<VEC>(uE, a.u + e + rS); ldv<VEC>(lE, a.lam + e + rS); }
      if (i > 0) { ldv<VEC>(uW, a.u + e - rS); ldv<VEC>(lW, a.lam + e - rS); }
      if (j + 1 < n) { ldv<VEC>(uN, a.u + e + rS * n); ldv<VEC>(lN, a.lam + e + rS * n); }
      if (j > 0) { ldv<VEC>(uS, a.u + e - rS * n); ldv<VEC>(lS, a.lam + e - rS * n); }
      double fE[VEC], fN[VEC], fW[VEC], fS[VEC], fm[VEC];
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        fE[c] = (lE[c] - lC[c]) * (uE[c] - uC[c]);
        fN[c] = (lN[c] - lC[c]) * (uN[c] - uC[c]);
        fW[c] = (i == 0) ? lC[c] * uC[c] : 0.0;   // face from the boundary node
        fS[c] = (j == 0) ? lC[c] * uC[c] : 0.0;
        fm[c] = (lE[c] - lW[c]) * (uN[c] - uS[c]) + (lN[c] - lS[c]) * (uE[c] - uW[c]);
      }
      // a and its mode derivatives at C, E, W, N, S; table columns of the
      // nodes i, i + 1, i + 2 (1-based node I = i + 1)
      const int qi = i - i0 + 1, qj = j - j0 + 1;
      double aC[VEC], aE[VEC], aW[VEC], aN[VEC], aS[VEC];
#pragma unroll
      for (int c = 0; c < VEC; ++c) aC[c] = aE[c] = aW[c] = aN[c] = aS[c] = 1.0;
#pragma unroll
      for (int k = 1; k <= kMaxD - 2; ++k) {
        if (k <= nm) {
          const double sIm = sI[k - 1][qi - 1], sIc = sI[k - 1][qi], sIp = sI[k - 1][qi + 1];
          const double sJm = sJ[k - 1][qj - 1], sJc = sJ[k - 1][qj], sJp = sJ[k - 1][qj + 1];
          const double w = a.amp / (double)(k * k);
          const double mC = w * sJc * sIc, mE = w * sJc * sIp, mW = w * sJc * sIm;
          const double mN = w * sJp * sIc, mS = w * sJm * sIc;
#pragma unroll
          for (int c = 0; c < VEC; ++c) {
            const double yk = ym[c][k + 1];
            aC[c] += yk * mC;
            aE[c] += yk * mE;
            aW[c] += yk * mW;
            aN[c] += yk * mN;
            aS[c] += yk * mS;
            // mode derivative contributions
            const double gx = ((mC + mE) / 2.0) * fE[c] + ((mW + mC) / 2.0) * fW[c];
            const double gy = ((mC + mN) / 2.0) * fN[c] + ((mS + mC) / 2.0) * fS[c];
            acc[k + 1][c] += k11[c] * gx + k22[c] * gy + k12[c] * mC * fm[c] / 4.0;
          }
        }
      }
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        const double gx = ((aC[c] + aE[c]) / 2.0) * fE[c] + ((aW[c] + aC[c]) / 2.0) * fW[c];
        const double gy = ((aC[c] + aN[c]) / 2.0) * fN[c] + ((aS[c] + aC[c]) / 2.0) * fS[c];
        const double gm = aC[c] * fm[c] / 4.0;
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[q][c] += dk[q][0][c] * gx + dk[q][1][c] * gy + dk[q][2][c] * gm;
      }
    }
  }
  const size_t ps = (size_t)gridDim.x * g.Sp;
#pragma unroll
  for (int q = 0; q < kMaxD; ++q) {
    if (q < d) {
      double v[VEC];
#pragma unroll
      for (int c = 0; c < VEC; ++c) v[c] = acc[q][c];
      reduce_group<VEC>(v, tpp, red);
      if (t < tpp) {
#pragma unroll
        for (int c = 0; c < VEC; ++c) a.partial[q * ps + (size_t)blockIdx.x * g.Sp + t * VEC + c] = v[c];
      }
    }
  }
}

void launch_dqdy(const DqdyArgs& a, int groups, hipStream_t s) {
  if (a.g.vec == 2) hipLaunchKernelGGL(dqdy_kernel<2>, dim3(groups), dim3(kNT), 0, s, a);
  else hipLaunchKernelGGL(dqdy_kernel<1>, dim3(groups), dim3(kNT), 0, s, a);
}

}  // namespace ens
