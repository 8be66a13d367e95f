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


// Tiles of kAsmTX x kAsmTY grid points, grid-strided over the workgroups.
// Per tile the mode tables sin(k pi I h) at the tile's node columns and rows
// are computed once and shared by every point and member of the tile (the
// sample-independent part of the form).  Per (point, member) the form is
// regrouped by the node a mode value sits at: the x-face terms, y-face
// terms and cross terms of the row give five coefficients cC, cE, cW, cN, cS
// (independent of the mode), and the mode-k derivative adds
//   cC sC + cE sE + cW sW + cN sN + cS sS,   sX = sin(k pi x1) sin(k pi x2) at X,
// its factor amp / k^2 applied once to the workgroup's sum.  The same
// products give a = 1 + sum_k (amp y_{k+1} / k^2) sX at the five nodes for
// the anisotropy derivatives.  NM = d - 2 is a template parameter: the
// mode loops unroll to exactly NM and the accumulators hold exactly d
// values per member, which keeps the register count at the occupancy the
// loads need (a runtime mode count held all 16 accumulators and 14 modes).
template <int VEC, int NM>
__global__ __launch_bounds__(kNT) void dqdy_kernel(DqdyArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  __shared__ double sI[kMaxModes][kAsmTX + 2];
  __shared__ double sJ[kMaxModes][kAsmTY + 2];
  __shared__ double wy[kMaxS][kMaxModes];   // amp y_{k+1} / k^2 per member slot
  __shared__ double wk[kMaxModes];          // amp / k^2
  __shared__ double coef[9][kMaxS];         // per member slot: K entries and their derivatives
  const Geometry& g = a.g;
  constexpr int D = NM + 2;
  const int S = g.S, n = g.n, tpp = g.tpp, t = threadIdx.x, d = D, nm = NM;
  const int sv = (t % tpp) * VEC;
  const bool lane_ok = sv < S;
  const int svl = lane_ok ? sv : S - VEC;   // idle slots compute on real members, add nothing
  if (t < nm) wk[t] = a.amp / (double)((t + 1) * (t + 1));
  for (int x = t; x < S * nm; x += kNT) {
    const int m = x / (NM > 0 ? NM : 1), k = x % (NM > 0 ? NM : 1);
    wy[m][k] = (a.amp * a.y[(size_t)m * d + k + 2]) / (double)((k + 1) * (k + 1));
  }

  // per-member coefficients and their derivatives, once per member and
  // workgroup: K's entries, and d/dy1 (through eps), d/dy2 (through theta)
  // of them
  if (t < S) {
    const double* y = a.y + (size_t)t * d;
    const double eps = (a.eps_model == 0) ? pow(10.0, -(1.0 + y[0])) : pow(10.0, -(1.5 + 1.5 * y[0]));
    const double th = (M_PI / 4.0) * (1.0 + y[1]);
    const double co = cos(th), si = sin(th);
    coef[0][t] = co * co + eps * (si * si);
    coef[1][t] = si * si + eps * (co * co);
    coef[2][t] = (1.0 - eps) * (si * co);
    const double deps = -((a.eps_model == 0) ? 1.0 : 1.5) * log(10.0) * eps;
    coef[3][t] = si * si * deps;
    coef[4][t] = co * co * deps;
    coef[5][t] = -si * co * deps;
    const double dth = M_PI / 4.0, s2 = sin(2.0 * th), c2 = cos(2.0 * th);
    coef[6][t] = -(1.0 - eps) * s2 * dth;
    coef[7][t] = (1.0 - eps) * s2 * dth;
    coef[8][t] = (1.0 - eps) * c2 * dth;
  }
  __syncthreads();
  double k11[VEC], k22[VEC], k12[VEC], dk[2][3][VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) {
    const int m = svl + c;
    k11[c] = coef[0][m];
    k22[c] = coef[1][m];
    k12[c] = coef[2][m];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 3; ++r) dk[q][r][c] = coef[3 + 3 * q + r][m];
  }
  // the member's mode weights amp y_{k+1} / k^2, fixed for the thread
  double wyr[NM > 0 ? NM : 1][VEC];
#pragma unroll
  for (int k = 0; k < NM; ++k)
#pragma unroll
    for (int c = 0; c < VEC; ++c) wyr[k][c] = wy[svl + c][k];
  double acc[D][VEC];
#pragma unroll
  for (int q = 0; q < D; ++q)
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
      // All ten loads are issued unconditionally, a neighbour outside the
      // grid reading the point itself, and its values are zeroed after:
      // loads inside lane-dependent branches would each be waited for at
      // the branch's end, one memory round trip per neighbour.
      const bool okE = i + 1 < n, okW = i > 0, okN = j + 1 < n, okS = j > 0;
      const size_t eE = okE ? e + rS : e, eW = okW ? e - rS : e;
      const size_t eN = okN ? e + rS * n : e, eS = okS ? e - rS * n : e;
      double uC[VEC], uE[VEC], uW[VEC], uN[VEC], uS[VEC];
      double lC[VEC], lE[VEC], lW[VEC], lN[VEC], lS[VEC];
      ldv<VEC>(uC, a.u + e);
      ldv<VEC>(lC, a.lam + e);
      ldv<VEC>(uE, a.u + eE);
      ldv<VEC>(lE, a.lam + eE);
      ldv<VEC>(uW, a.u + eW);
      ldv<VEC>(lW, a.lam + eW);
      ldv<VEC>(uN, a.u + eN);
      ldv<VEC>(lN, a.lam + eN);
      ldv<VEC>(uS, a.u + eS);
      ldv<VEC>(lS, a.lam + eS);
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        uE[c] = okE ? uE[c] : 0.0;
        lE[c] = okE ? lE[c] : 0.0;
        uW[c] = okW ? uW[c] : 0.0;
        lW[c] = okW ? lW[c] : 0.0;
        uN[c] = okN ? uN[c] : 0.0;
        lN[c] = okN ? lN[c] : 0.0;
        uS[c] = okS ? uS[c] : 0.0;
        lS[c] = okS ? lS[c] : 0.0;
      }
      double fE[VEC], fN[VEC], fW[VEC], fS[VEC], fm[VEC];
      double cC[VEC], cE[VEC], cW[VEC], cN[VEC], cS[VEC];
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        fE[c] = (lE[c] - lC[c]) * (uE[c] - uC[c]);
        fN[c] = (lN[c] - lC[c]) * (uN[c] - uC[c]);
        fW[c] = (i == 0) ? lC[c] * uC[c] : 0.0;   // face from the boundary node
        fS[c] = (j == 0) ? lC[c] * uC[c] : 0.0;
        fm[c] = (lE[c] - lW[c]) * (uN[c] - uS[c]) + (lN[c] - lS[c]) * (uE[c] - uW[c]);
        cE[c] = 0.5 * (k11[c] * fE[c]);
        cW[c] = 0.5 * (k11[c] * fW[c]);
        cN[c] = 0.5 * (k22[c] * fN[c]);
        cS[c] = 0.5 * (k22[c] * fS[c]);
        cC[c] = (cE[c] + cW[c]) + (cN[c] + cS[c]) + 0.25 * (k12[c] * fm[c]);
      }
      // table columns of the nodes i, i + 1, i + 2 (1-based node I = i + 1)
      const int qi = i - i0 + 1, qj = j - j0 + 1;
      double aC[VEC], aE[VEC], aW[VEC], aN[VEC], aS[VEC];
#pragma unroll
      for (int c = 0; c < VEC; ++c) aC[c] = aE[c] = aW[c] = aN[c] = aS[c] = 1.0;
#pragma unroll
      for (int k = 0; k < NM; ++k) {
        const double sIm = sI[k][qi - 1], sIc = sI[k][qi], sIp = sI[k][qi + 1];
        const double sJm = sJ[k][qj - 1], sJc = sJ[k][qj], sJp = sJ[k][qj + 1];
        const double pC = sJc * sIc, pE = sJc * sIp, pW = sJc * sIm;
        const double pN = sJp * sIc, pS = sJm * sIc;
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          const double w = wyr[k][c];
          aC[c] = fma(w, pC, aC[c]);
          aE[c] = fma(w, pE, aE[c]);
          aW[c] = fma(w, pW, aW[c]);
          aN[c] = fma(w, pN, aN[c]);
          aS[c] = fma(w, pS, aS[c]);
          double v = cC[c] * pC;
          v = fma(cE[c], pE, v);
          v = fma(cW[c], pW, v);
          v = fma(cN[c], pN, v);
          v = fma(cS[c], pS, v);
          acc[k + 2][c] += v;
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
  // the modes' factor amp / k^2
#pragma unroll
  for (int k = 0; k < NM; ++k)
#pragma unroll
    for (int c = 0; c < VEC; ++c) acc[k + 2][c] *= wk[k];
  const size_t ps = (size_t)gridDim.x * g.Sp;
#pragma unroll
  for (int q = 0; q < D; ++q) {
    {
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

template <int NM>
static void launch_dqdy_nm(const DqdyArgs& a, int groups, hipStream_t s) {
  if (a.g.vec == 2) hipLaunchKernelGGL((dqdy_kernel<2, NM>), dim3(groups), dim3(kNT), 0, s, a);
  else hipLaunchKernelGGL((dqdy_kernel<1, NM>), dim3(groups), dim3(kNT), 0, s, a);
}

// d - 2 sine modes, 0 .. kMaxModes (the caller has checked the range)
void launch_dqdy(const DqdyArgs& a, int groups, hipStream_t s) {
  switch (a.d - 2) {
    case 0: launch_dqdy_nm<0>(a, groups, s); break;
    case 1: launch_dqdy_nm<1>(a, groups, s); break;
    case 2: launch_dqdy_nm<2>(a, groups, s); break;
    case 3: launch_dqdy_nm<3>(a, groups, s); break;
    case 4: launch_dqdy_nm<4>(a, groups, s); break;
    case 5: launch_dqdy_nm<5>(a, groups, s); break;
    case 6: launch_dqdy_nm<6>(a, groups, s); break;
    case 7: launch_dqdy_nm<7>(a, groups, s); break;
    case 8: launch_dqdy_nm<8>(a, groups, s); break;
    case 9: launch_dqdy_nm<9>(a, groups, s); break;
    case 10: launch_dqdy_nm<10>(a, groups, s); break;
    case 11: launch_dqdy_nm<11>(a, groups, s); break;
    case 12: launch_dqdy_nm<12>(a, groups, s); break;
    case 13: launch_dqdy_nm<13>(a, groups, s); break;
    default: launch_dqdy_nm<14>(a, groups, s); break;
  }
}

}  // namespace ens
