// Device code of the global noise estimate (Sec. III F: Welch's method on the residual, the
// 30/15-bin median clip, Savitzky-Golay of order 1, spline).  Included by the host-side
// translation unit only.  All arithmetic in FP64.
#pragma once
#include "gbx_kernels.h"

namespace gbx {

// A window of the band and the segment of absolute bins [lo, hi) it owns.
struct SegWin {
  int64_t k0, data_off, lo, hi;
  int32_t W, C;
};

__global__ void __launch_bounds__(256) k_fill_zero(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// tw[m] = e^{-2 pi i m / n}
__global__ void __launch_bounds__(256) k_twiddle64(double* tw, int n) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)n, &s, &c);
  tw[2 * m] = c;
  tw[2 * m + 1] = s;
}

// Hermitian spectrum Y[0..M) of channel c: bin k of every window's segment, and its conjugate
// at M - k (segments lie inside [1, M/2), checked on the host).  One workgroup per window.
__global__ void __launch_bounds__(256) k_assemble(const SegWin* __restrict__ wins, const double* __restrict__ d, int c,
                                                  int64_t M, double* __restrict__ Y) {
  const SegWin s = wins[blockIdx.x];
  if (c >= s.C) return;
  const double* blk = d + 2 * (s.data_off + (int64_t)c * s.W);
  for (int64_t k = s.lo + threadIdx.x; k < s.hi; k += blockDim.x) {
    const double re = blk[2 * (k - s.k0)], im = blk[2 * (k - s.k0) + 1];
    Y[2 * k] = re;
    Y[2 * k + 1] = im;
    Y[2 * (M - k)] = re;
    Y[2 * (M - k) + 1] = -im;
  }
}

// Inverse DFT of length M = M1 M2 in two passes (four-step), x_n = sum_k Y_k e^{2 pi i k n / M}
// with k = k1 + M1 k2 and n = n2 + M2 n1:
//   pass A, one workgroup per k1: Z[k1][n2] = w^{k1 n2} sum_k2 Y[k1 + M1 k2] e^{2 pi i k2 n2 / M2},
//   pass B, one workgroup per n2: x[n2 + M2 n1] = sum_k1 Z[k1][n2] e^{2 pi i k1 n1 / M1},
// w = e^{2 pi i / M}; each sum is an in-LDS Stockham DFT of NF points, 8 per lane.
template <int NF>
__global__ void __launch_bounds__(NF / 8) k_ifft_a(const double* __restrict__ Y, double* __restrict__ Z,
                                                   const double* __restrict__ tw, int64_t M1) {
  constexpr int LPC = NF / 8;
  __shared__ cplx<double> buf[NF];
  const int64_t k1 = blockIdx.x;
  const int lane = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k2 = lane + LPC * e;
    const int64_t g = k1 + M1 * k2;
    buf[k2] = mk<double>(Y[2 * g], Y[2 * g + 1]);
  }
  slot_sync<LPC>();
  fft_lds<double, NF, LPC, 1, +1>(buf, lane, (const cplx<double>*)tw);
  const int64_t M = M1 * NF;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int n2 = lane + LPC * e;
    const int64_t r = (k1 * n2) % M;  // exact reduction of the twiddle's argument
    double s, c;
    sincospi(2.0 * (double)r / (double)M, &s, &c);
    const cplx<double> v = buf[n2] * mk<double>(c, s);
    Z[2 * (k1 * NF + n2)] = v.x;
    Z[2 * (k1 * NF + n2) + 1] = v.y;
  }
}

template <int NF>
__global__ void __launch_bounds__(NF / 8) k_ifft_b(const double* __restrict__ Z, double* __restrict__ x,
                                                   const double* __restrict__ tw, int64_t M2, double scale) {
  constexpr int LPC = NF / 8;
  __shared__ cplx<double> buf[NF];
  const int64_t n2 = blockIdx.x;
  const int lane = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int k1 = lane + LPC * e;
    const int64_t g = (int64_t)k1 * M2 + n2;
    buf[k1] = mk<double>(Z[2 * g], Z[2 * g + 1]);
  }
  slot_sync<LPC>();
  fft_lds<double, NF, LPC, 1, +1>(buf, lane, (const cplx<double>*)tw);
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int n1 = lane + LPC * e;
    x[n2 + M2 * n1] = buf[n1].x * scale;  // the Hermitian input leaves a real series
  }
}

// Welch segment s (samples s L/2 .. s L/2 + L - 1, L = 2 NF): the Hann-weighted real samples
// packed as NF complex values z_n = w_{2n} x_{a+2n} + i w_{2n+1} x_{a+2n+1}, one forward DFT of
// NF points, then the untangling of the real series' DFT: with E_k = (Z_k + conj Z_{NF-k}) / 2
// and O_k = (Z_k - conj Z_{NF-k}) / (2i), X_k = E_k + e^{-2 pi i k / L} O_k, k = 0..NF.
// Writes |X_k|^2 to Pseg[s][k].
template <int NF>
__global__ void __launch_bounds__(NF / 8) k_welch_seg(const double* __restrict__ x, const double* __restrict__ hann,
                                                      const double* __restrict__ tw, double* __restrict__ Pseg) {
  constexpr int LPC = NF / 8;
  __shared__ cplx<double> buf[NF];
  const int64_t s = blockIdx.x;
  const int lane = threadIdx.x;
  const double* xs = x + s * NF;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int n = lane + LPC * e;
    buf[n] = mk<double>(hann[2 * n] * xs[2 * n], hann[2 * n + 1] * xs[2 * n + 1]);
  }
  slot_sync<LPC>();
  fft_lds<double, NF, LPC, 1, -1>(buf, lane, (const cplx<double>*)tw);
  double* out = Pseg + s * (NF + 1);
  for (int k = lane; k <= NF; k += LPC) {
    const cplx<double> zk = buf[k & (NF - 1)];
    const cplx<double> zc = conjg(buf[(NF - k) & (NF - 1)]);
    const cplx<double> E = scal(zk + zc, 0.5);
    const cplx<double> O = scal(mul_mi(zk - zc), 0.5);
    double sn, cs;
    sincospi(-(double)k / (double)NF, &sn, &cs);  // e^{-2 pi i k / L}
    const cplx<double> X = E + O * mk<double>(cs, sn);
    out[k] = X.x * X.x + X.y * X.y;
  }
}

// P[k] = scale * mean over the K segments of Pseg[s][k] (segments summed in order), DC and the
// Nyquist bin at half the one-sided factor.
__global__ void __launch_bounds__(256) k_welch_mean(const double* __restrict__ Pseg, int K, int nb, double scale,
                                                    double* __restrict__ P) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  double acc = 0.0;
  for (int s = 0; s < K; ++s) acc += Pseg[(int64_t)s * nb + k];
  double v = acc / (double)K * scale;
  if (k == 0 || k == nb - 1) v *= 0.5;
  P[k] = v;
}

constexpr int kClipMaxBand = 8193;  // Welch bins of the longest segment (L = 16384)

// The median clip over the band of channel blockIdx.x: windows [s, s + width) for s = 0, stride,
// ... (cut at the band's end), in order, each on the values the previous ones left; values above
// twice the window's median become twice the median.  One wave: the band in LDS, each window's
// values ranked by lane (ties by position), the median from the ranked copy (the middle value, or
// the mean of the two middle ones for an even count).
__global__ void __launch_bounds__(64) k_median_clip(const double* __restrict__ P, double* __restrict__ out,
                                                    int64_t pitch, const int* __restrict__ lo,
                                                    const int* __restrict__ nbins, int width, int stride) {
  __shared__ double v[kClipMaxBand];
  __shared__ double srt[64];
  const int c = blockIdx.x;
  const int n = nbins[c];
  if (n <= 0) return;  // uniform over the workgroup
  const int lane = threadIdx.x;
  const double* src = P + c * pitch + lo[c];
  for (int j = lane; j < n; j += 64) v[j] = src[j];
  __syncthreads();
  for (int s = 0; s < n; s += stride) {
    const int m = min(width, n - s);
    const double xv = lane < m ? v[s + lane] : 0.0;
    int r = 0;
    for (int j = 0; j < m; ++j) {
      const double y = v[s + j];
      r += (y < xv) || (y == xv && j < lane);
    }
    if (lane < m) srt[r] = xv;
    __syncthreads();
    const double med = (m & 1) ? srt[m / 2] : 0.5 * (srt[m / 2 - 1] + srt[m / 2]);
    const double cap = 2.0 * med;
    if (lane < m && xv > cap) v[s + lane] = cap;
    __syncthreads();
  }
  double* dst = out + c * pitch + lo[c];
  for (int j = lane; j < n; j += 64) dst[j] = v[j];
}

// Order-1 Savitzky-Golay of y[0..n) at point i, window length wl: the window mean in the interior
// (window y[i - (wl-1)/2 .. i + wl/2]); the first and last wl/2 points from the least-squares line
// through the first and last wl points, at their own positions.
__device__ __forceinline__ double savgol1_at(const double* __restrict__ y, int n, int wl, int i) {
  const int h = wl / 2;
  if (i >= h && i < n - h) {
    double acc = 0.0;
    for (int j = i - (wl - 1) / 2; j <= i + wl / 2; ++j) acc += y[j];
    return acc / (double)wl;
  }
  const int a = i < h ? 0 : n - wl;
  const double pm = 0.5 * (double)(wl - 1);
  double ym = 0.0;
  for (int p = 0; p < wl; ++p) ym += y[a + p];
  ym /= (double)wl;
  double sxy = 0.0, sxx = 0.0;
  for (int p = 0; p < wl; ++p) {
    sxy += ((double)p - pm) * (y[a + p] - ym);
    sxx += ((double)p - pm) * ((double)p - pm);
  }
  return ym + sxy / sxx * ((double)(i - a) - pm);
}

// Smoothed band of every channel: wl_short below f_switch, wl_long above (f_j = j / (L dt)).
__global__ void __launch_bounds__(256) k_savgol(const double* __restrict__ Pc, double* __restrict__ Sm, int64_t pitch,
                                                const int* __restrict__ lo, const int* __restrict__ nbins, int L,
                                                double dt, double f_switch, int wl_short, int wl_long) {
  const int c = blockIdx.y;
  const int n = nbins[c];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* y = Pc + c * pitch + lo[c];
  const double f = (double)(lo[c] + i) / ((double)L * dt);
  Sm[c * pitch + lo[c] + i] = savgol1_at(y, n, f < f_switch ? wl_short : wl_long, i);
}

// Second derivatives of the natural cubic spline through the band of channel blockIdx.x (unit
// spacing): m_{j-1} + 4 m_j + m_{j+1} = 6 (y_{j+1} - 2 y_j + y_{j-1}), m_0 = m_{n-1} = 0, by
// forward elimination and back substitution in one thread (diag and rhs in the scratch arrays).
__global__ void k_spline_m(const double* __restrict__ Sm, double* __restrict__ mm, double* __restrict__ diag,
                           int64_t pitch, const int* __restrict__ lo, const int* __restrict__ nbins) {
  const int c = blockIdx.x;
  const int n = nbins[c];
  if (threadIdx.x != 0 || n <= 0) return;
  const double* y = Sm + c * pitch + lo[c];
  double* m = mm + c * pitch;
  double* dg = diag + c * pitch;
  m[0] = 0.0;
  m[n - 1] = 0.0;
  if (n < 3) {
    for (int j = 0; j < n; ++j) m[j] = 0.0;
    return;
  }
  const int k = n - 2;
  // rhs kept in m[1..n-2]
  for (int i = 0; i < k; ++i) {
    m[i + 1] = 6.0 * (y[i + 2] - 2.0 * y[i + 1] + y[i]);
    dg[i] = 4.0;
  }
  for (int i = 1; i < k; ++i) {
    const double r = 1.0 / dg[i - 1];
    dg[i] -= r;
    m[i + 1] -= r * m[i];
  }
  m[k] = m[k] / dg[k - 1];
  for (int i = k - 2; i >= 0; --i) m[i + 1] = (m[i + 1] - m[i + 2]) / dg[i];
}

// S and the weights 4 / (T S) at every bin of every window: the spline of the channel's band at
// position k L / M - lo (held at its end values outside the band).
__global__ void __launch_bounds__(256) k_spline_eval(const SegWin* __restrict__ wins, const double* __restrict__ Sm,
                                                     const double* __restrict__ mm, int64_t pitch,
                                                     const int* __restrict__ lo, const int* __restrict__ nbins,
                                                     int64_t M_over_L, double T, double* __restrict__ w,
                                                     double* __restrict__ S) {
  const SegWin sw = wins[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)sw.C * sw.W) return;
  const int c = (int)(e / sw.W);
  const int64_t k = sw.k0 + (e - (int64_t)c * sw.W);
  const int n = nbins[c];
  double val;
  if (n <= 0) {
    val = __builtin_nan("");
  } else if (n == 1) {
    val = Sm[c * pitch + lo[c]];
  } else {
    const double* y = Sm + c * pitch + lo[c];
    const double* m = mm + c * pitch;
    double t = (double)k / (double)M_over_L - (double)lo[c];
    t = fmin(fmax(t, 0.0), (double)(n - 1));
    const int i = min((int)floor(t), n - 2);
    const double u = t - (double)i, v = 1.0 - u;
    val = v * y[i] + u * y[i + 1] + ((v * v * v - v) * m[i] + (u * u * u - u) * m[i + 1]) / 6.0;
  }
  const int64_t g = sw.data_off + e;
  w[g] = 4.0 / (T * val);
  if (S) S[g] = val;
}

}  // namespace gbx
