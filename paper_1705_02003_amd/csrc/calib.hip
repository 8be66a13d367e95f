// STREAM triad: the achievable-HBM-bandwidth reference of the roofline.
#include <algorithm>

#include "device.h"

namespace ens {

// ------------------------------------------------------------ STREAM triad
// c = a + s b over n doubles: the HBM calibration of the roofline (two reads,
// one write per element).  One pair of doubles per lane and a grid that
// covers the arrays once (the loop only guards grids at their cap), with
// non-temporal loads and stores (the arrays are streamed once).  On MI355X
// this was the fastest of the variants tried (1 GiB arrays: 2, 4 or 8 pairs
// per lane on grids of 4096 to 262144 workgroups, plain or non-temporal
// accesses): HBM needs many requests in flight, which the widest grid gives.
__global__ __launch_bounds__(kNT) void triad_kernel(const double* a, const double* b, double* c,
                                                    double s, size_t n2) {
  const size_t stride = (size_t)gridDim.x * kNT;
  typedef __attribute__((address_space(1))) const d2 gcd2;
  typedef __attribute__((address_space(1))) d2 gd2;
  for (size_t i = (size_t)blockIdx.x * kNT + threadIdx.x; i < n2; i += stride) {
    const d2 av = __builtin_nontemporal_load((gcd2*)a + i);
    const d2 bv = __builtin_nontemporal_load((gcd2*)b + i);
    d2 cv;
    cv.x = fma(s, bv.x, av.x);
    cv.y = fma(s, bv.y, av.y);
    __builtin_nontemporal_store(cv, (gd2*)c + i);
  }
}

static unsigned stream_blocks(size_t n2) {
  return (unsigned)std::min<size_t>(std::max<size_t>((n2 + kNT - 1) / kNT, 1), (size_t)1 << 20);
}

__global__ void triad_tail_kernel(const double* a, const double* b, double* c, double s, size_t n) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[n - 1] = fma(s, b[n - 1], a[n - 1]);
}

void launch_triad(const double* a, const double* b, double* c, double s, size_t n, hipStream_t st) {
  const size_t n2 = n / 2;
  if (n2 > 0) hipLaunchKernelGGL(triad_kernel, dim3(stream_blocks(n2)), dim3(kNT), 0, st, a, b, c, s, n2);
  if (n & 1) hipLaunchKernelGGL(triad_tail_kernel, dim3(1), dim3(64), 0, st, a, b, c, s, n);
}

// ------------------------------------------------------------ read/write mix
// The same streaming with another mix of reads and writes: out_w = sum of
// the nread input arrays (input k at src + k * stride, output w at dst +
// w * stride), pairs of doubles per lane, non-temporal loads and stores.
// With 8 reads and 3 writes it moves the byte mix of the fused solver step.
// Grid and accesses as the triad's (two pairs per lane measured best here).
template <int NR, int NW>
__global__ __launch_bounds__(kNT) void stream_mix_kernel(const double* src, double* dst, size_t stride,
                                                         size_t n2) {
  typedef __attribute__((address_space(1))) const d2 gcd2;
  typedef __attribute__((address_space(1))) d2 gd2;
  const size_t gstride = (size_t)gridDim.x * kNT;
  constexpr int U = 2;
  for (size_t i = (size_t)blockIdx.x * kNT + threadIdx.x; i < n2; i += U * gstride) {
    d2 acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[u].x = 0.0;
      acc[u].y = 0.0;
    }
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t e = i + u * gstride;
        if (e < n2) {
          const d2 v = __builtin_nontemporal_load((gcd2*)(src + k * stride) + e);
          acc[u].x += v.x;
          acc[u].y += v.y;
        }
      }
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t e = i + u * gstride;
        if (e < n2) __builtin_nontemporal_store(acc[u], (gd2*)(dst + w * stride) + e);
      }
  }
}

int launch_stream_mix(const double* src, double* dst, size_t stride, size_t n, int nread, int nwrite,
                      hipStream_t st) {
  const size_t n2 = n / 2;
  const unsigned blocks = stream_blocks(n2);
#define ENS_MIX(R, W)                                                                           \
  if (nread == R && nwrite == W) {                                                              \
    hipLaunchKernelGGL((stream_mix_kernel<R, W>), dim3(blocks), dim3(kNT), 0, st, src, dst,     \
                       stride, n2);                                                             \
    return ENS_OK;                                                                              \
  }
  ENS_MIX(8, 3)
  ENS_MIX(2, 1)
  ENS_MIX(3, 1)
  ENS_MIX(1, 1)
#undef ENS_MIX
  return ENS_ENOTSUP;
}

}  // namespace ens
