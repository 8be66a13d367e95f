// STREAM triad: the achievable-HBM-bandwidth reference of the roofline.
#include <algorithm>

#include "device.h"

namespace ens {

// ------------------------------------------------------------ STREAM triad
// c = a + s b over n doubles: the HBM calibration of the roofline (two reads,
// one write per element).  Pairs of doubles per lane, eight strides in flight,
// non-temporal loads and stores (the arrays are streamed once); the fastest
// of the variants tried on MI355X (2, 4, 8 strides; plain or non-temporal).
__global__ __launch_bounds__(kNT) void triad_kernel(const double* a, const double* b, double* c,
                                                    double s, size_t n2) {
  const size_t stride = (size_t)gridDim.x * kNT;
  constexpr int U = 8;
  typedef __attribute__((address_space(1))) const d2 gcd2;
  typedef __attribute__((address_space(1))) d2 gd2;
  for (size_t i = (size_t)blockIdx.x * kNT + threadIdx.x; i < n2; i += U * stride) {
    d2 av[U], bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t k = i + u * stride;
      if (k < n2) {
        av[u] = __builtin_nontemporal_load((gcd2*)a + k);
        bv[u] = __builtin_nontemporal_load((gcd2*)b + k);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t k = i + u * stride;
      if (k < n2) {
        d2 cv;
        cv.x = fma(s, bv[u].x, av[u].x);
        cv.y = fma(s, bv[u].y, av[u].y);
        __builtin_nontemporal_store(cv, (gd2*)c + k);
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
    const size_t want = (n2 + 8 * (size_t)kNT - 1) / (8 * (size_t)kNT);
    const unsigned blocks = (unsigned)std::min<size_t>(std::max<size_t>(want, 1), 16384);
    hipLaunchKernelGGL(triad_kernel, dim3(blocks), dim3(kNT), 0, st, a, b, c, s, n2);
  }
  if (n & 1) hipLaunchKernelGGL(triad_tail_kernel, dim3(1), dim3(64), 0, st, a, b, c, s, n);
}

}  // namespace ens
