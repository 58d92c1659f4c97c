// Device code of the search and posterior stages' helpers: the Fisher information matrix by
// finite differences of templates, weighted 2-D kernel density estimates (Sec. III G), and
// data minus (or plus) lists of templates (Algorithm 2 residuals).  Included by the host-side
// translation unit only (the kernels are not templates).
#pragma once
#include "gbx_kernels.h"

namespace gbx {

// One window of a source whose Fisher matrix is wanted: where its bins and weights are.
struct FisherWin {
  int64_t k0, data_off;
  int32_t W, pad;
};

constexpr int kFdPoints = 17;  // theta, and theta + e_i, theta + 2 e_i for the 8 parameters

// Table I coordinates u (sin beta, log10 A, cos iota in place of beta, A, iota) and back.
__device__ __forceinline__ void to_table1_d(const double* th, double* u) {
#pragma unroll
  for (int i = 0; i < 8; ++i) u[i] = th[i];
  u[2] = sin(th[2]);
  u[4] = log10(th[4]);
  u[5] = cos(th[5]);
}
__device__ __forceinline__ void from_table1_d(const double* u, double* th) {
#pragma unroll
  for (int i = 0; i < 8; ++i) th[i] = u[i];
  th[2] = asin(fmin(1.0, fmax(-1.0, u[2])));
  th[4] = exp10(u[4]);
  th[5] = acos(fmin(1.0, fmax(-1.0, u[5])));
}

// The 17 parameter points of every source of a group (the sources idx[0..m)): point 0 is the
// source itself, point 1 + 2p (2 + 2p) moves Table I coordinate p by one (two) steps.  All 17
// go through the same coordinate round trip, so their differences see the steps only.
__global__ void __launch_bounds__(256) k_fisher_points(const double* __restrict__ theta, const double* __restrict__ steps,
                                                       const int32_t* __restrict__ idx, int m, double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= m * kFdPoints) return;
  const int s = g / kFdPoints, j = g % kFdPoints;
  const int src = idx[s];
  double u[8], th[8];
  to_table1_d(theta + 8 * (int64_t)src, u);
  if (j > 0) {
    const int p = (j - 1) / 2, k = (j - 1) % 2 + 1;
    u[p] += (double)k * steps[8 * (int64_t)src + p];
  }
  from_table1_d(u, th);
#pragma unroll
  for (int i = 0; i < 8; ++i) out[8 * (int64_t)g + i] = th[i];
}

// F_pq = sum_c sum_k w_k Re(D_p D_q^*) over the bins k of the source's window, with the
// second-order forward difference D_p = (-3 h(u) + 4 h(u + e_p) - h(u + 2 e_p)) / (2 e_p) of
// the templates (each template read at its own first bin).  One workgroup per source.
__global__ void __launch_bounds__(256) k_fisher_reduce(const double* __restrict__ h, const int64_t* __restrict__ fb,
                                                       const int32_t* __restrict__ idx, int m,
                                                       const FisherWin* __restrict__ fw, const double* __restrict__ w,
                                                       const double* __restrict__ steps, int N, int C,
                                                       double* __restrict__ F) {
  __shared__ double s_part[4][36];
  const int s = blockIdx.x;
  const int src = idx[s];
  const FisherWin win = fw[src];
  const int tid = threadIdx.x;
  const int64_t t0 = (int64_t)s * kFdPoints;
  const int64_t base = fb[t0];
  double inv2e[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const double e = steps[8 * (int64_t)src + p];
    inv2e[p] = e != 0.0 ? 0.5 / e : 0.0;
  }
  double acc[36];
#pragma unroll
  for (int i = 0; i < 36; ++i) acc[i] = 0.0;
  auto tmpl = [&](int j, int c, int64_t k) -> cplx<double> {
    const int64_t off = k - fb[t0 + j];
    if (off < 0 || off >= N) return mk<double>(0.0, 0.0);
    const double* e = h + 2 * (((t0 + j) * C + c) * N + off);
    return mk<double>(e[0], e[1]);
  };
  for (int ii = tid; ii < C * (N + 2); ii += blockDim.x) {
    const int c = ii / (N + 2);
    const int64_t k = base - 1 + ii % (N + 2);
    if (k < win.k0 || k >= win.k0 + win.W) continue;
    const double wk = w[win.data_off + (int64_t)c * win.W + (k - win.k0)];
    const cplx<double> h0 = tmpl(0, c, k);
    cplx<double> D[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const cplx<double> h1 = tmpl(1 + 2 * p, c, k), h2 = tmpl(2 + 2 * p, c, k);
      D[p] = scal(scal(h0, -3.0) + scal(h1, 4.0) - h2, inv2e[p]);
    }
    int q = 0;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = a; b < 8; ++b) acc[q++] += wk * (D[a].x * D[b].x + D[a].y * D[b].y);
  }
  // reduce over the workgroup: wave shuffles, then one LDS step
#pragma unroll
  for (int i = 0; i < 36; ++i) {
    double v = acc[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((tid & 63) == 0) s_part[tid >> 6][i] = v;
  }
  __syncthreads();
  if (tid < 36) {
    const double v = s_part[0][tid] + s_part[1][tid] + s_part[2][tid] + s_part[3][tid];
    int a = 0, r = tid;
    while (r >= 8 - a) {
      r -= 8 - a;
      ++a;
    }
    const int b = a + r;
    F[64 * (int64_t)src + 8 * a + b] = v;
    F[64 * (int64_t)src + 8 * b + a] = v;
  }
}

// Weighted 2-D Gaussian kernel density estimates of P parameter pairs, evaluated at q points,
// for independent sets (one per source; blockIdx.y):
//   out[i] = sum_p log( sum_j w_pj N(x_ip; y_pj, L_p L_p^T) ),
// with the bandwidth's Cholesky factor L_p = [[l00, 0], [l10, l11]].  One thread per query;
// the kernel points are staged through LDS in tiles and summed by a running log-sum-exp.
__global__ void __launch_bounds__(256) k_kde_logpdf(const double* __restrict__ pts, const double* __restrict__ wts, int P,
                                                    int64_t m, const double* __restrict__ chol,
                                                    const double* __restrict__ x, int64_t q, double* __restrict__ out) {
  __shared__ double s_y[256][3];
  const int tid = threadIdx.x;
  const int64_t set = blockIdx.y;
  pts += set * P * m * 2;
  wts += set * P * m;
  chol += set * P * 3;
  x += set * q * P * 2;
  out += set * q;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + tid;
  const bool act = g < q;
  double total = 0.0;
  for (int p = 0; p < P; ++p) {
    const double l00 = chol[3 * p], l10 = chol[3 * p + 1], l11 = chol[3 * p + 2];
    const double a = 1.0 / l00, b = -l10 / (l00 * l11), c = 1.0 / l11;  // L^{-1}
    double z0 = 0.0, z1 = 0.0;
    if (act) {
      const double x0 = x[2 * (g * P + p)], x1 = x[2 * (g * P + p) + 1];
      z0 = a * x0;
      z1 = b * x0 + c * x1;
    }
    double M = -__builtin_inf(), S = 0.0;
    for (int64_t t = 0; t < m; t += 256) {
      const int64_t j = t + tid;
      if (j < m) {
        const double y0 = pts[2 * (p * m + j)], y1 = pts[2 * (p * m + j) + 1];
        const double wj = wts[p * m + j];
        s_y[tid][0] = a * y0;
        s_y[tid][1] = b * y0 + c * y1;
        s_y[tid][2] = wj > 0.0 ? log(wj) : -__builtin_inf();
      }
      __syncthreads();
      const int nt = (int)((m - t) < 256 ? (m - t) : 256);
      if (act) {
        for (int jj = 0; jj < nt; ++jj) {
          const double lw = s_y[jj][2];
          if (!(lw > -__builtin_inf())) continue;
          const double d0 = z0 - s_y[jj][0], d1 = z1 - s_y[jj][1];
          const double e = lw - 0.5 * (d0 * d0 + d1 * d1);
          if (e > M) {
            S = S * exp(M - e) + 1.0;
            M = e;
          } else {
            S += exp(e - M);
          }
        }
      }
      __syncthreads();
    }
    total += M + log(S) - log(2.0 * kPi * l00 * l11);
  }
  if (act) out[g] = total;
}

// Rows idx[0..m) of an [n][8] parameter array, gathered into out [m][8].
__global__ void __launch_bounds__(256) k_gather_rows(const double* __restrict__ theta, const int32_t* __restrict__ idx,
                                                     int m, double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= 8 * m) return;
  out[g] = theta[8 * (int64_t)idx[g / 8] + g % 8];
}

// One window of gb_add_templates: its bins, and where its sources' templates are.
struct AddWin {
  int64_t k0, data_off;
  const double* h;       // complex templates [n][C][N] of the window's (N, C) group
  const int64_t* fb;     // their first bins
  const int32_t* src;    // indices (within the group's template list) of the window's sources
  int32_t W, N, C, n_src;
};

// d_out = d_in + sign * sum of the window's templates, bin by bin, the sources in their listed
// order (deterministic).  One workgroup per window.
__global__ void __launch_bounds__(256) k_add_templates(const AddWin* __restrict__ wins, double sign,
                                                       const double* d_in, double* d_out) {
  const AddWin aw = wins[blockIdx.x];
  for (int64_t e = threadIdx.x; e < (int64_t)aw.C * aw.W; e += blockDim.x) {
    const int c = (int)(e / aw.W);
    const int64_t k = aw.k0 + e % aw.W;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < aw.n_src; ++s) {
      const int j = aw.src[s];
      const int64_t off = k - aw.fb[j];
      if (off < 0 || off >= aw.N) continue;
      const double* hv = aw.h + 2 * (((int64_t)j * aw.C + c) * aw.N + off);
      re += hv[0];
      im += hv[1];
    }
    const int64_t g = 2 * (aw.data_off + e);
    d_out[g] = d_in[g] + sign * re;
    d_out[g + 1] = d_in[g + 1] + sign * im;
  }
}

}  // namespace gbx
