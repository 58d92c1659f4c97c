// Device code of the noise estimates.  Included by the host-side translation unit only.
#pragma once
#include "gbx_kernels.h"

namespace gbx {

// One window of the local noise estimate: where its C x W block of data and weights starts.
struct NoiseWin {
  int64_t data_off;
  int32_t W, C;
};

constexpr int kNoiseMaxW = 4096;  // the largest padded window: one LDS array of doubles

// Local noise level of every (window, channel) (Sec. III, noise within a frequency segment):
// the median over the window's bins of the one-sided periodogram 2 |d_k|^2 / T, and the
// scalar-product weights 4 / (T S) written over the channel's bins.  One workgroup of 1024
// threads per (window = blockIdx.x, channel = blockIdx.y): the W periodogram values, padded
// with +inf to a power of two, are sorted in LDS by a bitonic network; the median is the
// middle value (odd W) or the mean of the two middle values (even W).
__global__ void __launch_bounds__(1024) k_noise_median(const NoiseWin* __restrict__ wins, const double* __restrict__ d,
                                                       double T, double* __restrict__ w, double* __restrict__ S) {
  __shared__ double s[kNoiseMaxW];
  const NoiseWin nw = wins[blockIdx.x];
  const int c = blockIdx.y;
  if (c >= nw.C) return;  // uniform over the workgroup
  const int W = nw.W;
  int P = 1;
  while (P < W) P <<= 1;
  const int64_t base = nw.data_off + (int64_t)c * W;
  for (int k = threadIdx.x; k < P; k += blockDim.x) {
    double v = __builtin_inf();
    if (k < W) {
      const double re = d[2 * (base + k)], im = d[2 * (base + k) + 1];
      v = 2.0 * (re * re + im * im) / T;
    }
    s[k] = v;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
        const int lo = 2 * stride * (t / stride) + t % stride;
        const int hi = lo + stride;
        const bool ascending = (lo & size) == 0;
        const double a = s[lo], b = s[hi];
        if ((a > b) == ascending) {
          s[lo] = b;
          s[hi] = a;
        }
      }
      __syncthreads();
    }
  }
  const double med = (W & 1) ? s[W / 2] : 0.5 * (s[W / 2 - 1] + s[W / 2]);
  if (threadIdx.x == 0 && S) S[3 * (int64_t)blockIdx.x + c] = med;
  const double wk = 4.0 / (T * med);
  for (int k = threadIdx.x; k < W; k += blockDim.x) w[base + k] = wk;
}

}  // namespace gbx
