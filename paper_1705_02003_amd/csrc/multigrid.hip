// Geometric multigrid V-cycle for the 3-D model, a CG preconditioner of the
// kind the paper's numerical tests use (Section 4: CG with a multigrid
// hierarchy, a degree-2 Chebyshev smoother on every level and a direct solve
// on the coarsest).  On the structured trilinear mesh of n + 1 = 2^k cells
// per direction the levels halve the cells down to 2 (one interior node,
// solved exactly); prolongation P is trilinear interpolation, restriction
// its transpose, and the coarse operators are the Galerkin products P^T A P,
// formed per member on the device.  The smoothing steps and residuals run in
// the 3-D product kernel (fe3d.hip); this file holds the Galerkin product,
// the smoothers' spectral bounds and coefficients, the grid transfers and
// the coarse levels' V-cycle in one launch.
//
// Layout as everywhere: member innermost, X[r * S + s], V[k * L + r * S + s]
// with the 27 slots k = 9 (dk + 1) + 3 (dj + 1) + (di + 1).  One thread per
// (node, member slot): Sp = 2^ceil(log2 S) slots per node, kNT / Sp nodes
// per workgroup and pass; slots s >= S do nothing.  Every kernel that runs
// inside a solve returns at once when the solve's done flag is up.
#include <algorithm>
#include <cstring>

#include "device.h"
#include "multigrid.h"

namespace ens {

namespace {

// interpolation weight of fine node i from coarse node I (1-based, one
// direction): 1 at i = 2I, 1/2 at i = 2I -+ 1, else 0
__device__ __forceinline__ double w1(int i, int I) {
  const int t = i - 2 * I;
  return t == 0 ? 1.0 : ((t == 1 || t == -1) ? 0.5 : 0.0);
}

__device__ __forceinline__ double wt(int t) { return t == 0 ? 1.0 : 0.5; }

struct Lane {
  size_t p, pstride;   // first node, node stride of the grid-strided loop
  int s;               // member slot
  bool ok;             // s < S
};

__device__ __forceinline__ Lane lane_of(int Sp, int S) {
  Lane l;
  const int t = threadIdx.x, per = kNT / Sp;
  l.s = t % Sp;
  l.ok = l.s < S;
  l.p = (size_t)blockIdx.x * per + t / Sp;
  l.pstride = (size_t)gridDim.x * per;
  return l;
}

__device__ __forceinline__ bool is_done(const int* done) { return done && gload(done) != 0; }

}  // namespace

// ------------------------------------------------------------ Galerkin product
// Ac(I, I + delta) = sum over fine nodes i = 2I + f and their neighbours
// j = i + e of w(f) A(i, j) w(f + e - 2 delta), f, e, delta in {-1, 0, 1}^3,
// w the product of the per-direction weights (1 at offset 0, 1/2 at +-1,
// 0 beyond).  Per direction only 13 of the 27 (f, e, delta) triples have
// |f + e - 2 delta| <= 1, so 13^3 = 2197 of the 19683 products are nonzero:
// the loops over e and delta are unrolled, which makes them and their
// weights compile-time constants and drops the zero terms.  The loops over
// f carry unroll requests too: the compiler declines them (the code would
// exceed its size limit) but then schedules the rows three times faster
// than with no request (62 against 189 us at 15^3, S = 32).  Coarse neighbours
// outside the grid get 0, as the fine slots of neighbours outside do (those
// fine values are 0 and add nothing).  One thread per (coarse node,
// member); a fine row's 27 values are loaded together, one fine row at a
// time (the empty asm with a memory clobber keeps the compiler from hoisting
// the next row's loads, which would exhaust the registers).
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wpass-failed"
__global__ __launch_bounds__(kNT) void mg_rap_kernel(MgRapArgs a) {
  const int mc = a.mc, mf = 2 * mc + 1, S = a.S;
  const Lane l = lane_of(a.Sp, S);
  if (!l.ok) return;
  for (size_t pc = l.p; pc < a.nrc; pc += l.pstride) {
    const int I = (int)(pc % mc) + 1, J = (int)((pc / mc) % mc) + 1, K = (int)(pc / ((size_t)mc * mc)) + 1;
    double acc[27];
#pragma unroll
    for (int k = 0; k < 27; ++k) acc[k] = 0.0;
#pragma unroll
    for (int fz = -1; fz <= 1; ++fz)
#pragma unroll
      for (int fy = -1; fy <= 1; ++fy)
#pragma unroll
        for (int fx = -1; fx <= 1; ++fx) {
          // fine node 2I + f is always interior: 1 <= 2I + f <= 2 mc + 1
          const size_t rf = ((size_t)(2 * K + fz - 1) * mf + (2 * J + fy - 1)) * mf + (2 * I + fx - 1);
          double v[27];
#pragma unroll
          for (int k = 0; k < 27; ++k) v[k] = gload(&a.Vf[(size_t)k * a.vstride_f + rf * S + l.s]);
#pragma unroll
          for (int ez = -1; ez <= 1; ++ez)
#pragma unroll
            for (int ey = -1; ey <= 1; ++ey)
#pragma unroll
              for (int ex = -1; ex <= 1; ++ex) {
                const int k = 9 * (ez + 1) + 3 * (ey + 1) + (ex + 1);
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
                  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) {
                      const int tx = fx + ex - 2 * dx, ty = fy + ey - 2 * dy, tz = fz + ez - 2 * dz;
                      if (tx < -1 || tx > 1 || ty < -1 || ty > 1 || tz < -1 || tz > 1) continue;
                      const double w = (wt(fx) * wt(fy) * wt(fz)) * (wt(tx) * wt(ty) * wt(tz));
                      const int c = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
                      acc[c] = fma(w, v[k], acc[c]);
                    }
              }
          asm volatile("" ::: "memory");
        }
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int k = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
          const bool in = I + dx >= 1 && I + dx <= mc && J + dy >= 1 && J + dy <= mc && K + dz >= 1 &&
                          K + dz <= mc;
          gstore(&a.Vc[(size_t)k * a.vstride_c + pc * S + l.s], in ? acc[k] : 0.0);
        }
  }
}

#pragma clang diagnostic pop

// ------------------------------------------------------------ smoother bounds
// Per member the Gershgorin bound max_i sum_j |a_ij| / a_ii of D^-1 A on a
// level, as per-workgroup maxima.
__global__ __launch_bounds__(kNT) void mg_gersh_kernel(MgGershArgs a) {
  __shared__ double red[kWaves * 64];
  const Lane l = lane_of(a.Sp, a.S);
  double acc[1] = {0.0};
  for (size_t p = l.p; l.ok && p < a.nr; p += l.pstride) {
    const size_t e = p * a.S + l.s;
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < 27; ++k) rs += fabs(gload(&a.V[(size_t)k * a.vstride + e]));
    acc[0] = fmax(acc[0], rs / gload(&a.V[(size_t)13 * a.vstride + e]));
  }
  group_max<1>(acc, a.Sp, red);
  put_partial<1>(a.partial, a.Sp, a.Sp, acc);
}

// lambda_max per member and the coefficients of the degree-2 smoother on
// [lambda_max / ratio, lambda_max] (theta, delta the interval's centre and
// half-width, sigma = theta / delta, rho0 = 1 / sigma, rho1 = 1 / (2 sigma -
// rho0); the one step uses rho1 rho0 and 2 rho1 / delta); idle slots get
// theta = 1 and zero steps.
__global__ __launch_bounds__(kFinNT) void mg_coef_kernel(MgCoefArgs a) {
  __shared__ double fin[kFinNT];
  const int t = threadIdx.x;
  const double lmax = final_max(a.partial, a.G, a.Sp, fin);
  if (t >= a.Sp) return;
  double* cf = a.cheb + (size_t)t * kChebCoef;
  if (t >= a.S) {
    gstore(&a.lmax[t], 0.0);
    gstore(&cf[0], 1.0);
    for (int k = 1; k < kChebCoef; ++k) gstore(&cf[k], 0.0);
    return;
  }
  const double lmin = lmax / a.ratio;
  const double theta = (lmax + lmin) / 2.0;
  const double delta = (lmax - lmin) / 2.0;
  const double sigma1 = theta / delta;
  const double rho0 = 1.0 / sigma1;
  const double rho1 = 1.0 / (2.0 * sigma1 - rho0);
  gstore(&a.lmax[t], lmax);
  gstore(&cf[0], theta);
  gstore(&cf[1], rho1 * rho0);
  gstore(&cf[2], 2.0 * rho1 / delta);
  for (int k = 3; k < kChebCoef; ++k) gstore(&cf[k], 0.0);
}

// ------------------------------------------------------------ grid transfer
// Restriction b_c(I) = sum_f w(f) res(2I + f), one thread per (coarse node,
// member).  MG_RESTRICT_START also starts the coarse pre-smoother,
// z = D_c^-1 b_c / theta; MG_RESTRICT_SOLVE solves the one-node coarsest
// level, x = b_c / a.
__global__ __launch_bounds__(kNT) void mg_restrict_kernel(MgTransferArgs a) {
  if (is_done(a.done)) return;
  const int mc = a.mc, mf = 2 * mc + 1, S = a.S;
  const size_t nrc = (size_t)mc * mc * mc;
  const Lane l = lane_of(a.Sp, S);
  if (!l.ok) return;
  const double th = (a.op == MG_RESTRICT_START) ? gload(&a.cheb[(size_t)l.s * kChebCoef]) : 1.0;
  for (size_t pc = l.p; pc < nrc; pc += l.pstride) {
    const int I = (int)(pc % mc) + 1, J = (int)((pc / mc) % mc) + 1, K = (int)(pc / ((size_t)mc * mc)) + 1;
    double acc = 0.0;
    for (int fz = -1; fz <= 1; ++fz)
      for (int fy = -1; fy <= 1; ++fy)
#pragma unroll
        for (int fx = -1; fx <= 1; ++fx) {
          const size_t rf = ((size_t)(2 * K + fz - 1) * mf + (2 * J + fy - 1)) * mf + (2 * I + fx - 1);
          acc = fma(wt(fx) * wt(fy) * wt(fz), gload(&a.fine_in[rf * S + l.s]), acc);
        }
    const size_t e = pc * S + l.s;
    gstore(&a.coarse_out[e], acc);
    if (a.op == MG_RESTRICT_START) {
      const double z = (acc / gload(&a.Vc[(size_t)13 * a.vstride_c + e])) / th;
      gstore(&a.z[e], z);
    } else if (a.op == MG_RESTRICT_SOLVE) {
      gstore(&a.x[e], acc / gload(&a.Vc[(size_t)13 * a.vstride_c + e]));
    }
  }
}

// Prolongation and correction x_f(i) += sum_I w(i - 2I) x_c(I) over the up
// to eight coarse nodes I in [floor(i / 2), ceil(i / 2)]^3 (1-based), one
// thread per (fine node, member).
__global__ __launch_bounds__(kNT) void mg_prolong_kernel(MgTransferArgs a) {
  if (is_done(a.done)) return;
  const int mc = a.mc, mf = 2 * mc + 1, S = a.S;
  const size_t nrf = (size_t)mf * mf * mf;
  const Lane l = lane_of(a.Sp, S);
  if (!l.ok) return;
  for (size_t pf = l.p; pf < nrf; pf += l.pstride) {
    const int i = (int)(pf % mf) + 1, j = (int)((pf / mf) % mf) + 1, k = (int)(pf / ((size_t)mf * mf)) + 1;
    double acc = 0.0;
    for (int cz = k / 2; cz <= (k + 1) / 2; ++cz)
      for (int cy = j / 2; cy <= (j + 1) / 2; ++cy)
        for (int cx = i / 2; cx <= (i + 1) / 2; ++cx) {
          if (cx < 1 || cx > mc || cy < 1 || cy > mc || cz < 1 || cz > mc) continue;
          const size_t pc = ((size_t)(cz - 1) * mc + (cy - 1)) * mc + (cx - 1);
          acc = fma(w1(i, cx) * w1(j, cy) * w1(k, cz), gload(&a.coarse_in[pc * S + l.s]), acc);
        }
    const size_t e = pf * S + l.s;
    gstore(&a.fine_x[e], gload(&a.fine_x[e]) + acc);
  }
}

// ------------------------------------------------------------ coarse tail
// One workgroup per member s runs the V-cycle of the tail levels (at most 7^3
// nodes, then 3^3, then 1) with each level's 27 operator slots and its
// vectors b, x, res, d, za in LDS ([slot][row] and [row], row = (k m + j) m +
// i); phases are separated by barriers.  Every operation is the per-level
// kernels' own, in their order: the 27-term product in slot order starting
// with a product (neighbours outside the grid count zero), the Chebyshev
// step dd = c1 d + c2 (r - q) / diag, z = src + dd, the residual with its
// optional start z = (res / diag) / theta, the restriction over fz, fy, fx,
// the prolongation over cz, cy, cx, and x + (za + dd) for the post-smoother's
// correction; so the results are the same bits.
constexpr int kMgTailPool = 32 * (343 + 27 + 1);   // 27 slots + 5 vectors per node
constexpr int kTailNT = 512;     // threads of the tail workgroup: one 7^3 node each
constexpr int kTailStage = 21;   // staged elements a thread has in flight (one batch at 7^3)

namespace {

struct TailLv {
  double *A, *b, *x, *res, *d, *za;
  int m, nr;
  double th, c1, c2;
};

__device__ __forceinline__ double tail_apply(const TailLv& L, const double* p, int r) {
  const int m = L.m, i = r % m, j = (r / m) % m, k = r / (m * m);
  double q = 0.0;
#pragma unroll
  for (int dk = -1; dk <= 1; ++dk)
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
      for (int di = -1; di <= 1; ++di) {
        const int slot = 9 * (dk + 1) + 3 * (dj + 1) + (di + 1);
        const bool in = (unsigned)(i + di) < (unsigned)m && (unsigned)(j + dj) < (unsigned)m &&
                        (unsigned)(k + dk) < (unsigned)m;
        const double pv = in ? p[r + (dk * m + dj) * m + di] : 0.0;
        const double v = L.A[slot * L.nr + r];
        q = (slot == 0) ? v * pv : fma(v, pv, q);
      }
  return q;
}

// one Chebyshev step from src (d in place): out = src + dd, or x += src + dd
__device__ __forceinline__ void tail_cheb(const TailLv& L, const double* rv, const double* src, double* out,
                                          bool accumulate) {
  for (int r = threadIdx.x; r < L.nr; r += kTailNT) {
    const double q = tail_apply(L, src, r);
    const double dd = fma(L.c1, L.d[r], L.c2 * ((rv[r] - q) / L.A[13 * L.nr + r]));
    L.d[r] = dd;
    const double zn = src[r] + dd;
    if (accumulate) L.x[r] = L.x[r] + zn;
    else out[r] = zn;
  }
}

// res = b - A x, with `start` also d = za = (res / diag) / theta
__device__ __forceinline__ void tail_resid(const TailLv& L, bool start) {
  for (int r = threadIdx.x; r < L.nr; r += kTailNT) {
    const double rr = L.b[r] - tail_apply(L, L.x, r);
    L.res[r] = rr;
    if (start) {
      const double z = (rr / L.A[13 * L.nr + r]) / L.th;
      L.d[r] = z;
      L.za[r] = z;
    }
  }
}

}  // namespace

// One workgroup of kTailNT threads per member.  Workgroups go round-robin
// over the eight XCDs, and a cache line of b or x holds 16 consecutive
// members: with 8 or more members, workgroup b takes member
// (b mod 8) ceil(S / 8) + b / 8, so each XCD reads and writes a run of
// consecutive members and fetches their shared lines once.
__global__ __launch_bounds__(kTailNT) void mg_tail_kernel(MgTailArgs a) {
  __shared__ double pool[kMgTailPool];
  const int b = blockIdx.x, t = threadIdx.x, S = a.S, nlev = a.nlev;
  const int s = (S >= 8) ? (b & 7) * ((S + 7) >> 3) + (b >> 3) : b;
  if (s >= S || is_done(a.done)) return;
  // the loops over levels are unrolled, so L[] stays in registers
  TailLv L[kMgTailLevels];
  double* p = pool;
#pragma unroll
  for (int j = 0; j < kMgTailLevels; ++j) {
    TailLv& v = L[j];
    const int m = j < nlev ? a.lv[j].m : 1;
    v.m = m;
    v.nr = m * m * m;
    v.A = p;
    v.b = p + 27 * v.nr;
    v.x = v.b + v.nr;
    v.res = v.x + v.nr;
    v.d = v.res + v.nr;
    v.za = v.d + v.nr;
    p += 32 * v.nr;
    v.th = v.c1 = v.c2 = 0.0;
    if (j < nlev) {
      const double* cf = a.lv[j].cheb + (size_t)s * kChebCoef;
      v.th = gload(&cf[0]);
      v.c1 = gload(&cf[1]);
      v.c2 = gload(&cf[2]);
    }
  }
  // Stage the operators (member-major copies: one contiguous run per
  // level) and the first level's right-hand side: element idx of
  // [A_0 | A_1 | A_2 | b_0] (empty segments for absent levels).  A thread
  // issues the loads of kTailStage elements (at clamped indices, no branch)
  // before it stores any, so staging costs a few memory round trips.
  {
    int end[kMgTailLevels + 1];
    int tot = 0;
#pragma unroll
    for (int j = 0; j < kMgTailLevels; ++j) {
      tot += j < nlev ? 27 * L[j].nr : 0;
      end[j] = tot;
    }
    tot += L[0].nr;
    end[kMgTailLevels] = tot;
    const int off0 = (int)(L[0].A - pool), off1 = (int)(L[1].A - pool),
              off2 = (int)(L[2].A - pool), offb = (int)(L[0].b - pool);
    static_assert(kMgTailLevels == 3, "the staging map names three levels");
    // level j's run for member s starts at Vt_j + s 27 nr_j; b_0 is strided
    const double* V0 = a.lv[0].Vt + (size_t)s * 27 * L[0].nr;
    const double* V1 = nlev > 1 ? a.lv[1].Vt + (size_t)s * 27 * L[1].nr : V0;
    const double* V2 = nlev > 2 ? a.lv[2].Vt + (size_t)s * 27 * L[2].nr : V0;
    for (int base = t; base < tot; base += kTailStage * kTailNT) {
      double val[kTailStage];
      int dst[kTailStage];
#pragma unroll
      for (int u = 0; u < kTailStage; ++u) {
        const int idx = min(base + u * kTailNT, tot - 1);
        const int j = (idx >= end[0]) + (idx >= end[1]) + (idx >= end[2]);   // 3: b
        const int lo = j == 0 ? 0 : (j == 1 ? end[0] : (j == 2 ? end[1] : end[2]));
        const int loc = idx - lo;
        const double* src = j == 0 ? V0 + loc
                                   : (j == 1 ? V1 + loc
                                             : (j == 2 ? V2 + loc : a.b + (size_t)loc * S + s));
        val[u] = gload(src);
        dst[u] = (j == 0 ? off0 : (j == 1 ? off1 : (j == 2 ? off2 : offb))) + loc;
      }
#pragma unroll
      for (int u = 0; u < kTailStage; ++u)
        if (base + u * kTailNT < tot) pool[dst[u]] = val[u];
    }
  }
  __syncthreads();
  {
    const TailLv& v = L[0];
    for (int r = t; r < v.nr; r += kTailNT) {
      const double z = (v.b[r] / v.A[13 * v.nr + r]) / v.th;
      v.d[r] = z;
      v.za[r] = z;
    }
  }
  __syncthreads();
  // down: pre-smoothing, residual, restriction (starting the next level's
  // smoother, or solving the one-node last level)
#pragma unroll
  for (int j = 0; j + 1 < kMgTailLevels; ++j) {
    if (j + 1 >= nlev) break;
    const TailLv& v = L[j];
    tail_cheb(v, v.b, v.za, v.x, false);
    __syncthreads();
    tail_resid(v, false);
    __syncthreads();
    const TailLv& c = L[j + 1];
    const int mc = c.m, mf = v.m;
    for (int pc = t; pc < c.nr; pc += kTailNT) {
      const int I = pc % mc + 1, J = (pc / mc) % mc + 1, K = pc / (mc * mc) + 1;
      double acc = 0.0;
      for (int fz = -1; fz <= 1; ++fz)
        for (int fy = -1; fy <= 1; ++fy)
#pragma unroll
          for (int fx = -1; fx <= 1; ++fx) {
            const int rf = ((2 * K + fz - 1) * mf + (2 * J + fy - 1)) * mf + (2 * I + fx - 1);
            acc = fma(wt(fx) * wt(fy) * wt(fz), v.res[rf], acc);
          }
      c.b[pc] = acc;
      if (j + 2 == nlev) {
        c.x[pc] = acc / c.A[13 * c.nr + pc];
      } else {
        const double z = (acc / c.A[13 * c.nr + pc]) / c.th;
        c.d[pc] = z;
        c.za[pc] = z;
      }
    }
    __syncthreads();
  }
  // up: prolongation, residual with the post-smoother's start, post-smoothing
#pragma unroll
  for (int j = kMgTailLevels - 2; j >= 0; --j) {
    if (j + 1 >= nlev) continue;
    const TailLv& v = L[j];
    const TailLv& c = L[j + 1];
    const int mc = c.m, mf = v.m;
    for (int pf = t; pf < v.nr; pf += kTailNT) {
      const int i = pf % mf + 1, jj = (pf / mf) % mf + 1, k = pf / (mf * mf) + 1;
      double acc = 0.0;
      for (int cz = k / 2; cz <= (k + 1) / 2; ++cz)
        for (int cy = jj / 2; cy <= (jj + 1) / 2; ++cy)
          for (int cx = i / 2; cx <= (i + 1) / 2; ++cx) {
            if (cx < 1 || cx > mc || cy < 1 || cy > mc || cz < 1 || cz > mc) continue;
            const int pc = ((cz - 1) * mc + (cy - 1)) * mc + (cx - 1);
            acc = fma(w1(i, cx) * w1(jj, cy) * w1(k, cz), c.x[pc], acc);
          }
      v.x[pf] = v.x[pf] + acc;
    }
    __syncthreads();
    tail_resid(v, true);
    __syncthreads();
    tail_cheb(v, v.res, v.za, nullptr, true);
    __syncthreads();
  }
  for (int r = t; r < L[0].nr; r += kTailNT) gstore(&a.x[(size_t)r * S + s], L[0].x[r]);
}

// The member-major copy of a level's operator for the fused tail:
// Vt[s][slot][r] = V[slot * vstride + r * S + s].
__global__ __launch_bounds__(kNT) void mg_pack_kernel(const double* V, size_t vstride, double* Vt,
                                                      int nr, int S) {
  const size_t per = (size_t)27 * nr, n = per * S;
  for (size_t e = (size_t)blockIdx.x * kNT + threadIdx.x; e < n; e += (size_t)gridDim.x * kNT) {
    const size_t s = e / per, rem = e - s * per;
    const size_t slot = rem / nr, r = rem - slot * nr;
    Vt[e] = V[slot * vstride + r * S + s];
  }
}

// ------------------------------------------------------------ hierarchy
int mg_levels(int n, int* ms) {
  if (n < 1 || ((n + 1) & n) != 0) return 0;
  int L = 0, m = n;
  while (true) {
    if (L == kMgMaxLevels) return 0;
    ms[L++] = m;
    if (m == 1) break;
    m = (m - 1) / 2;
  }
  return L;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
static size_t mg_header_bytes() {
  return align256(sizeof(double) * (size_t)kMgMaxLevels * kMaxS * (kChebCoef + 1));
}
// the coarse level's 27 slots and four vectors
static size_t mg_level_doubles(int m, int S) {
  const size_t nr = (size_t)m * m * m;
  return slot_stride(nr * S) * (27 + 4);
}

// the member-major operator copy that the fused coarse tail stages
static size_t mg_tail_copy_bytes(int m, int S) {
  return m <= kMgTailNodes ? align256(sizeof(double) * 27 * (size_t)m * m * m * S) : 0;
}

size_t mg_bytes(int n, int S) {
  int ms[kMgMaxLevels];
  const int L = mg_levels(n, ms);
  if (L == 0) return 0;
  size_t b = mg_header_bytes();
  for (int l = 1; l < L; ++l)
    b += sizeof(double) * mg_level_doubles(ms[l], S) + mg_tail_copy_bytes(ms[l], S);
  return b;
}

void mg_carve(void* base, int n, int S, const int* ctl, MgHierarchy& H) {
  int ms[kMgMaxLevels];
  H.L = mg_levels(n, ms);
  double* hd = static_cast<double*>(base);
  char* p = static_cast<char*>(base) + mg_header_bytes();
  for (int l = 0; l < H.L; ++l) {
    MgLevel& v = H.lv[l];
    std::memset(&v, 0, sizeof(v));
    v.m = ms[l];
    v.g = make_geometry3(ms[l], S);
    if (l == 0) continue;
    v.g.full = 1;   // the Galerkin products are used as computed
    v.mem.cheb = hd + (size_t)l * kMaxS * kChebCoef;
    v.mem.lmax = hd + (size_t)kMgMaxLevels * kMaxS * kChebCoef + (size_t)l * kMaxS;
    v.mem.ctl = const_cast<int*>(ctl);
    double* q = reinterpret_cast<double*>(p);
    const size_t vs = v.g.vstride;
    v.V = q;
    double* vec = q + 27 * vs;
    v.b = vec;
    v.x = vec + vs;
    v.res = vec + 2 * vs;
    v.za = vec + 3 * vs;
    p += sizeof(double) * mg_level_doubles(ms[l], S);
    if (ms[l] <= kMgTailNodes) {
      v.Vt = reinterpret_cast<double*>(p);
      p += mg_tail_copy_bytes(ms[l], S);
    }
  }
}

// ------------------------------------------------------------ launchers
int mg_groups(size_t nr, int Sp) {
  const size_t per = (size_t)(kNT / Sp);
  return (int)std::min<size_t>(std::max<size_t>((nr + per - 1) / per, 1), 1024);
}

void launch_mg_rap(const MgRapArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mg_rap_kernel, dim3(mg_groups(a.nrc, a.Sp)), dim3(kNT), 0, s, a);
}

void launch_mg_tail(const MgTailArgs& a, hipStream_t s) {
  const int blocks = (a.S >= 8) ? 8 * ((a.S + 7) / 8) : a.S;
  hipLaunchKernelGGL(mg_tail_kernel, dim3(blocks), dim3(kTailNT), 0, s, a);
}

void launch_mg_pack(const double* V, size_t vstride, double* Vt, int m, int S, hipStream_t s) {
  const size_t n = (size_t)27 * m * m * m * S;
  const int groups = (int)std::min<size_t>((n + kNT - 1) / kNT, 1024);
  hipLaunchKernelGGL(mg_pack_kernel, dim3(groups), dim3(kNT), 0, s, V, vstride, Vt, m * m * m, S);
}

void launch_mg_gersh(const MgGershArgs& a, int groups, hipStream_t s) {
  hipLaunchKernelGGL(mg_gersh_kernel, dim3(groups), dim3(kNT), 0, s, a);
}

void launch_mg_coef(const MgCoefArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(mg_coef_kernel, dim3(1), dim3(kFinNT), 0, s, a);
}

void launch_mg_transfer(const MgTransferArgs& a, hipStream_t s) {
  const size_t mc = (size_t)a.mc, mf = 2 * mc + 1;
  if (a.op == MG_PROLONG)
    hipLaunchKernelGGL(mg_prolong_kernel, dim3(mg_groups(mf * mf * mf, a.Sp)), dim3(kNT), 0, s, a);
  else
    hipLaunchKernelGGL(mg_restrict_kernel, dim3(mg_groups(mc * mc * mc, a.Sp)), dim3(kNT), 0, s, a);
}


}  // namespace ens
