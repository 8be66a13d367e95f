// The 3-D model of the paper's numerical tests (Section 2.1, eqs.
// (elliptic-SPDE) and (diff-coeff); Section 4): -div(diag(a, a_y, a_z) grad u)
// = 1 on the unit cube, u = 0 on the boundary, trilinear finite elements on a
// uniform mesh of (m+1)^3 cubes, a log-normal diffusivity
//   a(x, y) = a_min + a_hat exp(sum_k sqrt(lambda_k) b_k(x) y_k)
// built from the eigenpairs of the covariance sigma_0 exp(-|x - x'|_1 / delta).
//
// Host: the covariance eigenpairs.  The kernel is a product of three 1-D
// kernels exp(-|s - t| / delta), whose eigenpairs on [0, 1] are the classical
// closed forms: cos(w (s - 1/2)) with c cos(w/2) = w sin(w/2) and
// sin(w (s - 1/2)) with w cos(w/2) + c sin(w/2) = 0, c = 1/delta, eigenvalue
// 2c / (w^2 + c^2); the frequencies are found by bisection.
//
// Device: ensemble assembly of the 27-point matrix (member innermost, as in
// the 2-D model), and one solver step of every mode:
//   M_PCG_*: a direction kernel (p = D^-1 r + beta p_old or z + beta p_old,
//            and the deferred x += alpha_prev p_old), then the product
//            q = A p with the partial sums of p^T q;
//   M_SPMV:  q = A p;
//   M_CHEB:  one Chebyshev step d = c1 d_prev + c2 D^-1 (r - A z),
//            z_out = z + d (d_prev formed from the iterates), on the last step
//            with the partial sums of r^T z_out;
//   M_RESID: the residual q = r - A x of a multigrid level, optionally with
//            its smoother's start z_out = D^-1 q / theta;
//   M_CHEBX: a multigrid post-smoother's Chebyshev step added to the
//            level's x in place, optionally with the partial sums of
//            dotv^T x.
// The neighbours' values of the product come through the caches (a point's
// 27 neighbours lie on three planes of the grid, all near in memory); of the
// 27 matrix values of a row, the 14 of slots 13..26 are read and the other
// 13 are the neighbours' rows' upper values (symmetry), also through the
// caches.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device.h"
#include "fe3d.h"

namespace ens {

namespace {

constexpr double kDelta = 0.25;
constexpr double kAmin = 0.1, kAhat = 1.0, kAy = 1.0, kAz = 1.0;
constexpr int kModes1d = 8;   // 1-D modes from which the 3-D products are drawn

struct Mode1 {
  int kind;
  double w, lam, norm;
};

// the root in [lo, hi] of a function that changes sign there, to the last bit
template <class F>
double bisect(F f, double lo, double hi) {
  const bool neg_lo = f(lo) < 0.0;
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if ((f(mid) < 0.0) == neg_lo) lo = mid;
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

std::vector<Mode1> kl_1d(int count) {
  const double c = 1.0 / kDelta, a = 0.5, pi = M_PI;
  std::vector<Mode1> out;
  for (int j = 0; j < count; ++j) {
    double w = bisect([&](double v) { return c * std::cos(v * a) - v * std::sin(v * a); },
                      j * pi / a + 1e-12, (j * pi + pi / 2) / a - 1e-12);
    out.push_back({0, w, 2 * c / (w * w + c * c), 1.0 / std::sqrt(a + std::sin(2 * w * a) / (2 * w))});
    w = bisect([&](double v) { return v * std::cos(v * a) + c * std::sin(v * a); },
               (j * pi + pi / 2) / a + 1e-12, (j + 1) * pi / a - 1e-12);
    out.push_back({1, w, 2 * c / (w * w + c * c), 1.0 / std::sqrt(a - std::sin(2 * w * a) / (2 * w))});
  }
  std::stable_sort(out.begin(), out.end(), [](const Mode1& x, const Mode1& y) { return x.lam > y.lam; });
  out.resize(count);
  return out;
}

__device__ __forceinline__ double phi1(int kind, double w, double norm, double s) {
  const double u = w * (s - 0.5);
  return norm * (kind == 0 ? cos(u) : sin(u));
}

// The factor a_hat of eq. (diff-coeff): 1 in Test 1; in Test 2 (Section 4,
// Test 2 equation) 1, 100 or 10 as r(y) = |y|_2 lies below d/4, between d/4
// and d/2, or at or above d/2 (d = sqrt(3)), decided on r^2 = sum_n y_n^2
// (each product and sum rounded, in index order) against the exact
// d^2/16 = 3/16 and d^2/4 = 3/4.
__device__ __forceinline__ double fe3d_ahat(const double* y, int d, int test) {
#pragma clang fp contract(off)
  if (test == 0) return kAhat;
  double r2 = 0.0;
  for (int n = 0; n < d; ++n) r2 = r2 + y[n] * y[n];
  return r2 < 0.1875 ? 1.0 : (r2 < 0.75 ? 100.0 : 10.0);
}

}  // namespace

int fe3d_setup(const ens_problem* p, Fe3dAsmArgs& a) {
  if (p->d < 1 || p->d > kMaxTerms) return ENS_EINVAL;
  const std::vector<Mode1> m1 = kl_1d(kModes1d);
  struct T {
    double lam;
    int idx[3];
  };
  std::vector<T> t;
  const double sigma0 = std::sqrt(300.0);
  for (int x = 0; x < kModes1d; ++x)
    for (int y = 0; y < kModes1d; ++y)
      for (int z = 0; z < kModes1d; ++z) {
        int s3[3] = {x, y, z};
        std::sort(s3, s3 + 3);   // the same product for every permutation
        t.push_back({sigma0 * (m1[s3[0]].lam * m1[s3[1]].lam * m1[s3[2]].lam), {x, y, z}});
      }
  // enumeration order is (x, y, z) lexicographic: a stable sort keeps it for ties
  std::stable_sort(t.begin(), t.end(), [](const T& u, const T& v) { return u.lam > v.lam; });
  for (int k = 0; k < p->d; ++k) {
    Fe3dTerm& f = a.term[k];
    for (int q = 0; q < 3; ++q) {
      const Mode1& md = m1[t[k].idx[q]];
      f.w[q] = md.w;
      f.norm[q] = md.norm;
      f.kind[q] = md.kind;
    }
    f.sq = std::sqrt(t[k].lam);
  }
  return ENS_OK;
}

// ------------------------------------------------------------ assembly
// One thread per (row, member) of the launch's members m0 .. m0 + mc - 1
// (mcp threads per row).  The cube matrices follow from the 1-D
// linear-element stiffness K1 = [[1, -1], [-1, 1]] / h and mass
// M1 = [[2, 1], [1, 2]] h / 6: a cube with coefficient a_c adds
// a_c Kx My Mz + a_y Mx Ky Mz + a_z Mx My Kz between two of its nodes; the
// value of slot (di, dj, dk) sums the cubes holding both nodes.
__global__ __launch_bounds__(kNT) void fe3d_assemble_kernel(Fe3dAsmArgs a) {
#pragma clang fp contract(off)
  __shared__ double ys[kAsmY];
  const int t = threadIdx.x;
  for (int x = t; x < a.mc * a.d; x += kNT) ys[x] = a.y[x];
  __syncthreads();
  const int cl = t % a.mcp;
  const size_t row = (size_t)blockIdx.x * (kNT / a.mcp) + t / a.mcp;
  if (cl >= a.mc || row >= a.nr) return;
  const int m = a.m;
  const size_t e = row * a.S + a.m0 + cl;
  const int i = (int)(row % m), j = (int)((row / m) % m), k = (int)(row / ((size_t)m * m));
  const double* y = ys + cl * a.d;
  const double ahat = fe3d_ahat(y, a.d, a.test);
  const double h = 1.0 / (double)(m + 1);

  // a at the centres of the eight cubes around mesh node (i+1, j+1, k+1):
  // cube (i + cx, j + cy, k + cz), cx, cy, cz in {0, 1}
  double ac[2][2][2];
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const double xc = ((double)(i + cx) + 0.5) * h;
        const double yc = ((double)(j + cy) + 0.5) * h;
        const double zc = ((double)(k + cz) + 0.5) * h;
        double g = 0.0;
        for (int n = 0; n < a.d; ++n) {
          const Fe3dTerm& f = a.term[n];
          const double bx = phi1(f.kind[0], f.w[0], f.norm[0], xc);
          const double by = phi1(f.kind[1], f.w[1], f.norm[1], yc);
          const double bz = phi1(f.kind[2], f.w[2], f.norm[2], zc);
          g = g + (f.sq * y[n]) * ((bz * by) * bx);
        }
        ac[cz][cy][cx] = kAmin + ahat * exp(g);
      }
  const double kd = 1.0 / h, ko = -1.0 / h;               // K1 diagonal / off-diagonal
  const double md = (2.0 * h) / 6.0, mo = (1.0 * h) / 6.0;  // M1
  auto K1 = [&](int l, int l2) { return l == l2 ? kd : ko; };
  auto M1 = [&](int l, int l2) { return l == l2 ? md : mo; };
  for (int dk = -1; dk <= 1; ++dk)
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int slot = 9 * (dk + 1) + 3 * (dj + 1) + (di + 1);
        double v = 0.0;
        const bool inside = i + di >= 0 && i + di < m && j + dj >= 0 && j + dj < m &&
                            k + dk >= 0 && k + dk < m;
        if (inside) {
          for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
              for (int cx = 0; cx < 2; ++cx) {
                // local coordinates of the node and its neighbour in the cube
                const int lx = 1 - cx, ly = 1 - cy, lz = 1 - cz;
                const int nx = lx + di, ny = ly + dj, nz = lz + dk;
                if (nx < 0 || nx > 1 || ny < 0 || ny > 1 || nz < 0 || nz > 1) continue;
                const double t = ac[cz][cy][cx] * K1(lx, nx) * M1(ly, ny) * M1(lz, nz) +
                                 kAy * M1(lx, nx) * K1(ly, ny) * M1(lz, nz) +
                                 kAz * M1(lx, nx) * M1(ly, ny) * K1(lz, nz);
                v = v + t;
              }
        }
        a.V[(size_t)slot * a.vstride + e] = v;
      }
  a.b[e] = h * h * h;
}

// ------------------------------------------------------------ indicator
// Paper, Section 3.2, eq. (pb-indicator): H(y) = sup over the domain of
// lambda_max / lambda_min of the diffusion tensor.  3-D: the tensor is
// diag(a, a_y, a_z) with a constant on each cube, so H is the largest
// max(a, a_y, a_z) / min(a, a_y, a_z) over the cubes.  2-D: a(x) K(y) has
// eigenvalues a(x) and a(x) eps, so H = 1 / eps(y_0) everywhere.  One thread
// per (cube, member), grid-strided; per-workgroup maxima per member.
__global__ __launch_bounds__(kNT) void indicator_kernel(IndArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  const int Sp = a.Sp, t = threadIdx.x, s = t & (Sp - 1);
  const bool lane_ok = s < a.S;
  const double* y = a.y + (size_t)(lane_ok ? s : a.S - 1) * a.d;
  const double ahat = (a.dim == 3) ? fe3d_ahat(y, a.d, a.eps_model) : 0.0;
  double hv[1] = {0.0};
  const size_t cpb = (size_t)(kNT / Sp);   // cubes per workgroup and pass
  const size_t stride = (size_t)gridDim.x * cpb;
  for (size_t c = (size_t)blockIdx.x * cpb + t / Sp; lane_ok && c < a.ncell; c += stride) {
    double r;
    if (a.dim == 3) {
      const int mc = a.m + 1;
      const int cx = (int)(c % mc), cy = (int)((c / mc) % mc), cz = (int)(c / ((size_t)mc * mc));
      const double h = 1.0 / (double)(a.m + 1);
      const double xc = ((double)cx + 0.5) * h, yc = ((double)cy + 0.5) * h, zc = ((double)cz + 0.5) * h;
      double g = 0.0;
      for (int n = 0; n < a.d; ++n) {
        const Fe3dTerm& f = a.term[n];
        const double bx = phi1(f.kind[0], f.w[0], f.norm[0], xc);
        const double by = phi1(f.kind[1], f.w[1], f.norm[1], yc);
        const double bz = phi1(f.kind[2], f.w[2], f.norm[2], zc);
        g = g + (f.sq * y[n]) * ((bz * by) * bx);
      }
      const double ac = kAmin + ahat * exp(g);
      r = fmax(fmax(ac, kAy), kAz) / fmin(fmin(ac, kAy), kAz);
    } else {
      const double eps = (a.eps_model == 0) ? pow(10.0, -(1.0 + y[0])) : pow(10.0, -(1.5 + 1.5 * y[0]));
      r = 1.0 / eps;
    }
    hv[0] = fmax(hv[0], r);
  }
  group_max<1>(hv, Sp, red);
  put_partial<1>(a.partial, Sp, Sp, hv);
}

// ------------------------------------------------------------ adjoint form
// lambda^T (dA/dy_j) u for every member and j < d.  Only a depends on y:
// on cube c, da_c/dy_j = a_hat exp(g_c) sqrt(lambda_j) b_j(x_c), and a
// multiplies the cube matrix Kx My Mz, so the form is the sum over cubes of
// that derivative times lambda_c^T (Kx My Mz) u_c over the cube's eight
// nodes (boundary nodes hold 0).  One thread per (cube, member),
// grid-strided; per-workgroup sums per member for each j.
__global__ __launch_bounds__(kNT) void fe3d_dqdy_kernel(Fe3dDqdyArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  const int S = a.S, Sp = a.Sp, t = threadIdx.x, m = a.m, mc = m + 1;
  const int s0 = t & (Sp - 1);
  const bool lane_ok = s0 < S;
  const int s = lane_ok ? s0 : S - 1;   // idle slots compute on a real member, add nothing
  const double* y = a.y + (size_t)s * a.d;
  const double ahat = fe3d_ahat(y, a.d, a.test);
  const double h = 1.0 / (double)mc;
  const double kd = 1.0 / h, ko = -1.0 / h, md = (2.0 * h) / 6.0, mo = (1.0 * h) / 6.0;
  double acc[kMaxTerms];
#pragma unroll
  for (int q = 0; q < kMaxTerms; ++q) acc[q] = 0.0;
  const size_t cpb = (size_t)(kNT / Sp);   // cubes per workgroup and pass
  const size_t stride = (size_t)gridDim.x * cpb;
  for (size_t c = (size_t)blockIdx.x * cpb + t / Sp; lane_ok && c < a.ncell; c += stride) {
    const int cx = (int)(c % mc), cy = (int)((c / mc) % mc), cz = (int)(c / ((size_t)mc * mc));
    // nodal values of lambda and u at the cube's corners (mesh node
    // (cx + lx, cy + ly, cz + lz); interior when 1 <= index <= m)
    double lv[8], uv[8];
#pragma unroll
    for (int l = 0; l < 8; ++l) {
      const int I = cx + (l & 1), J = cy + ((l >> 1) & 1), K = cz + (l >> 2);
      const bool in = I >= 1 && I <= m && J >= 1 && J <= m && K >= 1 && K <= m;
      const size_t row = in ? ((size_t)(K - 1) * m + (J - 1)) * m + (I - 1) : 0;
      const double lx = a.lam[row * S + s], ux = a.u[row * S + s];
      lv[l] = in ? lx : 0.0;
      uv[l] = in ? ux : 0.0;
    }
    double B = 0.0;
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const double kx = ((p & 1) == (q & 1)) ? kd : ko;
        const double my = (((p >> 1) & 1) == ((q >> 1) & 1)) ? md : mo;
        const double mz = ((p >> 2) == (q >> 2)) ? md : mo;
        B = B + lv[p] * (kx * my * mz) * uv[q];
      }
    const double xc = ((double)cx + 0.5) * h, yc = ((double)cy + 0.5) * h, zc = ((double)cz + 0.5) * h;
    double bj[kMaxTerms];
    double g = 0.0;
#pragma unroll
    for (int n = 0; n < kMaxTerms; ++n) {
      bj[n] = 0.0;
      if (n < a.d) {
        const Fe3dTerm& f = a.term[n];
        const double bx = phi1(f.kind[0], f.w[0], f.norm[0], xc);
        const double by = phi1(f.kind[1], f.w[1], f.norm[1], yc);
        const double bz = phi1(f.kind[2], f.w[2], f.norm[2], zc);
        bj[n] = (bz * by) * bx;
        g = g + (f.sq * y[n]) * bj[n];
      }
    }
    const double eg = ahat * exp(g);
#pragma unroll
    for (int n = 0; n < kMaxTerms; ++n)
      if (n < a.d) acc[n] += eg * a.term[n].sq * bj[n] * B;
  }
  const size_t ps = (size_t)gridDim.x * Sp;
#pragma unroll
  for (int q = 0; q < kMaxTerms; ++q) {
    if (q < a.d) {
      double v[1] = {acc[q]};
      group_reduce<1>(v, Sp, red);
      put_partial<1>(a.partial + q * ps, Sp, Sp, v);
    }
  }
}

void launch_fe3d_dqdy(const Fe3dDqdyArgs& a, int groups, hipStream_t s) {
  hipLaunchKernelGGL(fe3d_dqdy_kernel, dim3(groups), dim3(kNT), 0, s, a);
}

void launch_indicator(const IndArgs& a, int groups, hipStream_t s) {
  hipLaunchKernelGGL(indicator_kernel, dim3(groups), dim3(kNT), 0, s, a);
}

// ------------------------------------------------------------ solver step
// p = D^-1 r + beta p_old (M_PCG_J) or z + beta p_old (M_PCG_Z) and the
// deferred x += alpha_prev p_old, element by element.
template <int VEC, int MODE>
__global__ __launch_bounds__(kNT) void fe3d_dir_kernel(StencilArgs a) {
  if (gload(&a.m.ctl[CTL_DONE])) return;
  const Geometry& g = a.g;
  const int t = threadIdx.x, sv = (t % g.tpp) * VEC;
  if (sv >= g.S) return;
  double beta[VEC], aprev[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) {
    beta[c] = gload(&a.m.beta[sv + c]);
    aprev[c] = gload(&a.m.alpha_prev[sv + c]);
  }
  const double* diag = a.V + (size_t)g.cslot * g.vstride;
  const size_t P = (size_t)(kNT / g.tpp);
  const size_t stride = (size_t)gridDim.x * P;
  for (size_t p = (size_t)blockIdx.x * P + t / g.tpp; p < g.nr; p += stride) {
    const size_t e = p * g.S + sv;
    double v0[VEC], dv[VEC], po[VEC], xv[VEC], pv[VEC];
    if constexpr (MODE == M_PCG_J) {
      ld<VEC>(v0, a.r + e);
      ld<VEC>(dv, diag + e);
    } else {
      ld<VEC>(v0, a.src + e);
    }
    ld<VEC>(po, a.pold + e);
    ld<VEC>(xv, a.x + e);
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
      if constexpr (MODE == M_PCG_J) pv[c] = fma(beta[c], po[c], v0[c] / dv[c]);
      else pv[c] = fma(beta[c], po[c], v0[c]);
      if (aprev[c] != 0.0) xv[c] = fma(aprev[c], po[c], xv[c]);
    }
    st<VEC>(a.pnew + e, pv);
    st<VEC>(a.x + e, xv);
  }
}

// The 27-point product, grid-strided over runs of NP x-neighbouring points
// (pairs, or single points on grids too small to fill the chip with pairs)
// with VEC members per thread; the mode's fused work follows
// (see the top of this file).  A pair shares the p values of a 4-wide window
// on each of its nine (dj, dk) rows, loaded once: 36 loads of p per pair
// instead of 54.  Neighbour offsets are the pair's offset plus a uniform row
// offset, with no per-neighbour multiplication.  On MI355X (31^3 points,
// S = 32) these make the launch 32 % shorter than one point per thread with
// an index product per neighbour, which at twice the workgroups was still
// 14 % slower and would double the finishing kernels' partials.  The dk loop is
// not unrolled: unrolled, the compiler hoists every load of the pair and
// spills registers.  The register budget allows three waves per SIMD: one
// launch of 512 workgroups fills two, and the third leaves room for another
// ensemble's kernel on another stream (at two, two ensembles solved
// concurrently ran slower than one at a time).
// SYM: the matrix is symmetric, so the thirteen lower values of row P are
// read as the upper values of the neighbours' rows, A(P, P + o) =
// A(P + o, P) = slot 26 - s of row P + o; those rows are being read by their
// own threads at about the same time, so the values come through the caches
// and the matrix streams from memory about once at 14 words per row.  The
// products are formed in the same order, so on a bitwise-symmetric matrix
// both reads give the same bits.
template <int VEC, int MODE, bool SYM, int NP>
__global__ __launch_bounds__(kNT) __attribute__((amdgpu_waves_per_eu(3)))
void fe3d_stencil_kernel(StencilArgs a) {
  __shared__ double red[kWaves * 64 * 2];
  constexpr bool PCG = (MODE == M_PCG_J || MODE == M_PCG_Z);
  const Geometry& g = a.g;
  if constexpr (MODE != M_SPMV) {
    if (gload(&a.m.ctl[CTL_DONE])) return;
  }
  const int S = g.S, tpp = g.tpp, t = threadIdx.x, m = g.n;
  const int sv = (t % tpp) * VEC;
  // idle slots (sv >= S) load the last members' values and store and sum nothing
  const bool lane_ok = sv < S;
  const int svl = lane_ok ? sv : S - VEC;
  const int ppb = kNT / tpp;   // pairs per workgroup and pass
  const int mi = (m + NP - 1) / NP;
  const size_t npair = (size_t)mi * m * m;
  const size_t vs = g.vstride;
  double acc[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) acc[c] = 0.0;
  const double* src = PCG ? a.pnew : a.src;
  // Chunks of ppb consecutive pairs.  Consecutive workgroup ids are
  // dispatched round-robin over the eight XCDs, each with its own L2: the
  // chunks are split into eight contiguous ranges, one per XCD, so that a
  // point's neighbours (one row and one plane away), whose values this
  // thread reads, are mostly handled -- and cached -- on the same XCD.
  const size_t nchunk = (npair + ppb - 1) / ppb;
  size_t c0 = blockIdx.x, cstep = gridDim.x, cend = nchunk;
  if (gridDim.x >= 8 && (gridDim.x & 7) == 0) {
    const size_t x = blockIdx.x & 7;
    c0 = (x * nchunk >> 3) + (blockIdx.x >> 3);
    cstep = gridDim.x >> 3;
    cend = (x + 1) * nchunk >> 3;
  }
  for (size_t ch = c0; ch < cend; ch += cstep) {
    const size_t gi = ch * ppb + t / tpp;
    if (gi >= npair) continue;
    const int ig = (int)(gi % mi), j = (int)((gi / mi) % m), k = (int)(gi / ((size_t)mi * m));
    const int i0 = ig * NP;
    // offset of the pair's first point; x = i0 - 1 + c is inside for colok[c]
    const size_t eb = (((size_t)k * m + j) * m + i0) * S + svl;
    bool colok[NP + 2];
#pragma unroll
    for (int c = 0; c < NP + 2; ++c) colok[c] = (unsigned)(i0 - 1 + c) < (unsigned)m;
    const bool jlo = j > 0, jhi = j + 1 < m, klo = k > 0, khi = k + 1 < m;
    double q[NP][VEC], own[NP][VEC];
#pragma unroll 1
    for (int dk = -1; dk <= 1; ++dk) {
      const bool kok = dk < 0 ? klo : (dk > 0 ? khi : true);
#pragma unroll
      for (int dj = -1; dj <= 1; ++dj) {
        const bool rok = kok && (dj < 0 ? jlo : (dj > 0 ? jhi : true));
        const size_t rs = (size_t)(((long long)dk * m + dj) * m * S);   // the row's offset (wraps)
        // p at x = i0 - 1 .. i0 + NP on this row; outside the grid the load
        // reads the pair's first point and the value counts zero
        double pw[NP + 2][VEC];
#pragma unroll
        for (int c = 0; c < NP + 2; ++c) {
          const bool ok = rok && colok[c];
          ld<VEC>(pw[c], src + (ok ? eb + rs + (size_t)((c - 1) * S) : eb));
#pragma unroll
          for (int cc = 0; cc < VEC; ++cc) pw[c][cc] = ok ? pw[c][cc] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NP; ++u) {
          // the second point of a pair past the grid's end (odd m) computes
          // on the first point's row and stores nothing
          const bool uv = colok[u + 1];
          const size_t eu = uv ? eb + (size_t)(u * S) : eb;
#pragma unroll
          for (int di = -1; di <= 1; ++di) {
            const int slot = 9 * (dk + 1) + 3 * (dj + 1) + (di + 1);
            const bool ok = uv && rok && colok[u + di + 1];
            double vk[VEC];
            if (SYM && slot < 13) {
              ld<VEC>(vk, a.V + (size_t)(26 - slot) * vs +
                              (ok ? eb + rs + (size_t)((u + di) * S) : eu));
            } else if (SYM) {
              ld<VEC>(vk, a.V + (size_t)slot * vs + eu);
            } else {
              ld_stream<VEC>(vk, a.V + (size_t)slot * vs + eu);
            }
#pragma unroll
            for (int c = 0; c < VEC; ++c) {
              const double pv = pw[u + di + 1][c];
              if (SYM) vk[c] = ok ? vk[c] : 0.0;
              q[u][c] = (slot == 0) ? vk[c] * pv : fma(vk[c], pv, q[u][c]);
              if (slot == 13) own[u][c] = pv;
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      if (!colok[u + 1] || !lane_ok) continue;
      const size_t e = eb + (size_t)(u * S);
      if constexpr (MODE == M_SPMV) {
        st<VEC>(a.q + e, q[u]);
      } else if constexpr (PCG) {
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[c] = fma(own[u][c], q[u][c], acc[c]);
        st<VEC>(a.q + e, q[u]);
      } else if constexpr (MODE == M_RESID) {
        double rr[VEC];
        ld<VEC>(rr, a.r + e);
#pragma unroll
        for (int c = 0; c < VEC; ++c) rr[c] = rr[c] - q[u][c];
        st<VEC>(a.q + e, rr);
        if (a.cheb_init) {
          double dg[VEC], zn[VEC];
          ld<VEC>(dg, a.V + (size_t)g.cslot * vs + e);
#pragma unroll
          for (int c = 0; c < VEC; ++c)
            zn[c] = (rr[c] / dg[c]) / gload(&a.m.cheb[(size_t)(sv + c) * kChebCoef]);
          st<VEC>(a.zout + e, zn);
        }
      } else {  // M_CHEB, M_CHEBX
        // the step's coefficients and the diagonal are loaded again here
        // (cached) rather than held in registers across the sweep, which
        // keeps the kernel at three waves per SIMD without spilling.  No
        // increment vector is kept: d_0 = z_0 is the source itself (M_CHEBX
        // is always a first step), d_1 = z_1 - z_0 with z_0 = D^-1 r / theta
        // formed again, and from the third step on d_{k-1} = z_{k-1} - z_{k-2}
        // with z_{k-2} read at the own point (zprev, which zout overwrites).
        const int step = (MODE == M_CHEBX) ? 1 : a.cheb_step;
        double rr[VEC], zp[VEC], zn[VEC], dg[VEC], c1[VEC], c2[VEC], xv[VEC], dv[VEC];
        ld<VEC>(rr, a.r + e);
        ld<VEC>(dg, a.V + (size_t)g.cslot * vs + e);
#pragma unroll
        for (int c = 0; c < VEC; ++c) zp[c] = 0.0;
        if (step >= 3) ld<VEC>(zp, a.zprev + e);
        if constexpr (MODE == M_CHEBX) {
          ld<VEC>(xv, a.x + e);
          if (a.dotv) ld<VEC>(dv, a.dotv + e);
        }
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          c1[c] = gload(&a.m.cheb[(size_t)(sv + c) * kChebCoef + 2 * step - 1]);
          c2[c] = gload(&a.m.cheb[(size_t)(sv + c) * kChebCoef + 2 * step]);
        }
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          double dp = own[u][c];   // d_{k-1}
          if (step == 2) dp = own[u][c] - (rr[c] / dg[c]) / gload(&a.m.cheb[(size_t)(sv + c) * kChebCoef]);
          else if (step >= 3) dp = own[u][c] - zp[c];
          // explicit fma: the same rounding in every instantiation (and in
          // the multigrid tail kernel, which repeats this step)
          const double dd = fma(c1[c], dp, c2[c] * ((rr[c] - q[u][c]) / dg[c]));
          zn[c] = own[u][c] + dd;
          if constexpr (MODE == M_CHEBX) {
            xv[c] = xv[c] + zn[c];
            if (a.dotv) acc[c] = fma(dv[c], xv[c], acc[c]);
          } else if (a.cheb_last) {
            acc[c] = fma(rr[c], zn[c], acc[c]);
          }
        }
        if constexpr (MODE == M_CHEBX) st<VEC>(a.x + e, xv);
        else st<VEC>(a.zout + e, zn);
      }
    }
  }
  if constexpr (PCG) {
    group_reduce<VEC>(acc, tpp, red);
    put_partial<VEC>(a.partial, g.Sp, tpp, acc);
  } else if constexpr (MODE == M_CHEB) {
    if (a.cheb_last) {
      group_reduce<VEC>(acc, tpp, red);
      put_partial<VEC>(a.partial, g.Sp, tpp, acc);
    }
  } else if constexpr (MODE == M_CHEBX) {
    if (a.dotv) {
      group_reduce<VEC>(acc, tpp, red);
      put_partial<VEC>(a.partial, g.Sp, tpp, acc);
    }
  }
}

// ------------------------------------------------------------ launchers
void launch_fe3d_assemble(const Fe3dAsmArgs& a, hipStream_t s) {
  const size_t rpb = (size_t)(kNT / a.mcp);   // rows per workgroup
  const unsigned blocks = (unsigned)((a.nr + rpb - 1) / rpb);
  hipLaunchKernelGGL(fe3d_assemble_kernel, dim3(blocks), dim3(kNT), 0, s, a);
}

template <int VEC, int MODE>
static void fe3d_step(const StencilArgs& a, hipStream_t s) {
  if constexpr (MODE == M_PCG_J || MODE == M_PCG_Z)
    hipLaunchKernelGGL((fe3d_dir_kernel<VEC, MODE>), dim3(init_groups(a.g)), dim3(kNT), 0, s, a);
  // g.np points per thread (pairs on grids that fill the chip with them)
  const dim3 grid(a.g.groups), block(kNT);
  if (a.g.np == 1) {
    if (a.g.full) hipLaunchKernelGGL((fe3d_stencil_kernel<VEC, MODE, false, 1>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((fe3d_stencil_kernel<VEC, MODE, true, 1>), grid, block, 0, s, a);
  } else {
    if (a.g.full) hipLaunchKernelGGL((fe3d_stencil_kernel<VEC, MODE, false, kFe3dPair>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((fe3d_stencil_kernel<VEC, MODE, true, kFe3dPair>), grid, block, 0, s, a);
  }
}

template <int MODE>
void launch_fe3d(const StencilArgs& a, hipStream_t s) {
  if (a.g.vec == 2) fe3d_step<2, MODE>(a, s);
  else fe3d_step<1, MODE>(a, s);
}
template void launch_fe3d<M_SPMV>(const StencilArgs&, hipStream_t);
template void launch_fe3d<M_PCG_J>(const StencilArgs&, hipStream_t);
template void launch_fe3d<M_PCG_Z>(const StencilArgs&, hipStream_t);
template void launch_fe3d<M_CHEB>(const StencilArgs&, hipStream_t);
template void launch_fe3d<M_RESID>(const StencilArgs&, hipStream_t);
template void launch_fe3d<M_CHEBX>(const StencilArgs&, hipStream_t);

}  // namespace ens
