// STREAM triad: the achievable-HBM-bandwidth reference of the roofline.
#include <algorithm>

#include "device.h"

namespace ens {

// ------------------------------------------------------------ STREAM triad
// c = a + s b over n doubles: the HBM calibration of the roofline (two reads,
// one write per element).  Pairs of doubles per lane, four strides in flight.
__global__ __launch_bounds__(kNT) void triad_kernel(const double* a, const double* b, double* c,
                                                    double s, size_t n2) {
  const size_t stride = (size_t)gridDim.x * kNT;
  constexpr int U = 4;
  for (size_t i = (size_t)blockIdx.x * kNT + threadIdx.x; i < n2; i += U * stride) {
    double av[U][2], bv[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t k = i + u * stride;
      if (k < n2) {
        ld<2>(av[u], a + 2 * k);
        ld<2>(bv[u], b + 2 * k);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t k = i + u * stride;
      if (k < n2) {
        double cv[2] = {fma(s, bv[u][0], av[u][0]), fma(s, bv[u][1], av[u][1])};
        st<2>(c + 2 * k, cv);
      }
    }
  }
}

__global__ void triad_tail_kernel(const double* a, const double* b, double* c, double s, size_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[n - 1] = fma(s, b[n - 1], a[n - 1]);
}

void launch_triad(const double* a, const double* b, double* c, double s, size_t n, hipStream_t st) {
  const size_t n2 = n / 2;
  if (n2 > 0) {
    const size_t want = (n2 + 4 * (size_t)kNT - 1) / (4 * (size_t)kNT);
    const unsigned blocks = (unsigned)std::min<size_t>(std::max<size_t>(want, 1), 8192);
    hipLaunchKernelGGL(triad_kernel, dim3(blocks), dim3(kNT), 0, st, a, b, c, s, n2);
  }
  if (n & 1) hipLaunchKernelGGL(triad_tail_kernel, dim3(1), dim3(64), 0, st, a, b, c, s, n);
}

}  // namespace ens
