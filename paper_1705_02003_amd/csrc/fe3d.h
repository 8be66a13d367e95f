// The 3-D model's kernel arguments and launchers (fe3d.hip): assembly,
// the parameter-based indicator and the adjoint form.
#pragma once

#include "common.h"

namespace ens {

// 3-D model: one term of the log-diffusivity expansion, a product of three
// 1-D covariance eigenfunctions (kind 0: norm cos(w (s - 1/2)), kind 1:
// norm sin(w (s - 1/2))) scaled by sqrt(lambda)
constexpr int kMaxTerms = 16;
constexpr int kFe3dPair = 2;   // x-neighbouring points per thread of the product kernel
struct Fe3dTerm {
  double w[3], norm[3];
  int kind[3];
  double sq;
};

struct Fe3dAsmArgs {
  double y[kAsmY];  // [mc][d]: members m0 .. m0 + mc - 1 (by value, as in AsmArgs)
  double* V;        // [27][vstride], slot k holds [N_r][S]
  double* b;        // [N_r][S]
  int m, S, d;
  int m0, mc, mcp;  // first member, members, threads per row (power of two >= mc)
  int test;         // coefficient a_hat: 0 Test 1 (1), 1 Test 2 (banded by |y|)
  size_t nr, vstride;
  Fe3dTerm term[kMaxTerms];
};

// 3-D model: lambda^T (dA/dy_j) u per member (the adjoint gradient's form)
struct Fe3dDqdyArgs {
  const double* y;    // [S][d]
  const double* u;    // [N_r][S]
  const double* lam;  // [N_r][S]
  double* partial;    // [d][groups][Sp]
  int m, S, Sp, d;    // Sp: member slots (power of two >= S); one thread per slot and cube
  int test;           // as in Fe3dAsmArgs
  size_t ncell;       // (m+1)^3 cubes
  Fe3dTerm term[kMaxTerms];
};

// Parameter-based grouping indicator (both models): per member the largest
// ratio lambda_max / lambda_min of the diffusion tensor over the domain.
struct IndArgs {
  const double* y;   // [S][d]
  double* partial;   // [groups][Sp] per-workgroup maxima
  int dim, m, S, Sp, d, eps_model;   // 3-D: eps_model selects a_hat as Fe3dAsmArgs::test
  size_t ncell;      // 3-D: cubes (m+1)^3; 2-D: 1 (the ratio does not depend on x)
  Fe3dTerm term[kMaxTerms];
};

int fe3d_setup(const ens_problem* p, Fe3dAsmArgs& a);
void launch_fe3d_assemble(const Fe3dAsmArgs& a, hipStream_t s);
void launch_indicator(const IndArgs& a, int groups, hipStream_t s);
void launch_fe3d_dqdy(const Fe3dDqdyArgs& a, int groups, hipStream_t s);

}  // namespace ens
