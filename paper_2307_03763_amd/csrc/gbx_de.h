// Device code of the differential-evolution search step (DE/rand/1/bin of Storn and Price, the
// optimiser of the paper's search in Sec. III): trial vectors for every member of every
// window's population, and the greedy selection by the SNR of the trials.  Included by the
// host-side translation unit only (the kernels are not templates).
#pragma once
#include "gbx_kernels.h"

namespace gbx {

// The seven searched coordinates (Table I coordinates without the amplitude, which the SNR
// does not depend on): f0, fdot, sin(beta), lambda, cos(iota), psi, phi0.
constexpr int kDeDim = 7;

// lambda, psi and phi0 wrap around their ranges; the others reflect at the box walls
__device__ __forceinline__ bool de_periodic(int k) { return k == 3 || k == 5 || k == 6; }

// floor(u n) for u in [0, 1), kept inside [0, n - 1]
__device__ __forceinline__ int de_pick(double u, int n) {
  const int v = (int)floor(u * (double)n);
  return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// One trial per (window, member) thread.  Donors a, b, c: uniform over the population without
// the member and each other, from three uniforms (each draw counts the free slots and skips the
// taken indices in increasing order).  Mutant a + F (b - c) (DE/rand/1), or, with base given,
// x_base[w] + F (a - b) (DE/best/1: the window's best member plus a difference of two donors),
// folded back into the box (periodic coordinates wrap, the others reflect at the walls and are
// clipped); binomial crossover with rate cr, the coordinate floor(u_j 7) always from the mutant.
// The arithmetic is not contracted into fused multiply-adds, so that it rounds as the plain
// reference does.
__global__ void __launch_bounds__(256) k_de_trial(int n_win, int pop, const double* __restrict__ lo,
                                                  const double* __restrict__ hi, const double* __restrict__ x,
                                                  const double* __restrict__ u_idx, const double* __restrict__ u_cross,
                                                  const double* __restrict__ u_j, const double* __restrict__ F,
                                                  const int32_t* __restrict__ base, double cr, double amp,
                                                  double* __restrict__ trial_x, double* __restrict__ trial_theta) {
#pragma clang fp contract(off)
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)n_win * pop) return;
  const int w = (int)(g / pop), i = (int)(g % pop);
  int a = de_pick(u_idx[3 * g], pop - 1);
  if (a >= i) ++a;
  int b = de_pick(u_idx[3 * g + 1], pop - 2);
  {
    const int s0 = min(i, a), s1 = max(i, a);
    if (b >= s0) ++b;
    if (b >= s1) ++b;
  }
  int c = de_pick(u_idx[3 * g + 2], pop - 3);
  {
    int s0 = i, s1 = a, s2 = b, t;
    if (s0 > s1) { t = s0; s0 = s1; s1 = t; }
    if (s1 > s2) { t = s1; s1 = s2; s2 = t; }
    if (s0 > s1) { t = s0; s0 = s1; s1 = t; }
    if (c >= s0) ++c;
    if (c >= s1) ++c;
    if (c >= s2) ++c;
  }
  const int jr = de_pick(u_j[g], kDeDim);
  const double f = F[w];
  // DE/best/1: base member plus the difference of the first two donors
  const int m0 = base ? min(max(base[w], 0), pop - 1) : a, m1 = base ? a : b, m2 = base ? b : c;
  const double* xa = x + ((int64_t)w * pop + m0) * kDeDim;
  const double* xb = x + ((int64_t)w * pop + m1) * kDeDim;
  const double* xc = x + ((int64_t)w * pop + m2) * kDeDim;
  const double* xi = x + g * kDeDim;
  double v[kDeDim];
#pragma unroll
  for (int k = 0; k < kDeDim; ++k) {
    if (u_cross[kDeDim * g + k] < cr || k == jr) {
      const double diff = xb[k] - xc[k];
      const double step = f * diff;
      double m = xa[k] + step;
      const double l = lo[kDeDim * w + k], h = hi[kDeDim * w + k];
      if (de_periodic(k)) {
        const double wd = h - l;
        double r = fmod(m - l, wd);  // exact
        if (r != 0.0 && ((r < 0.0) != (wd < 0.0))) r += wd;
        m = l + r;
      } else {
        if (m < l) m = 2.0 * l - m;
        if (m > h) m = 2.0 * h - m;
        m = fmin(fmax(m, l), h);
      }
      v[k] = m;
    } else {
      v[k] = xi[k];
    }
    trial_x[kDeDim * g + k] = v[k];
  }
  // back to the physical parameters, the amplitude fixed at `amp`
  double* th = trial_theta + 8 * g;
  th[0] = v[0];
  th[1] = v[1];
  th[2] = asin(fmin(1.0, fmax(-1.0, v[2])));
  th[3] = v[3];
  th[4] = amp;
  th[5] = acos(fmin(1.0, fmax(-1.0, v[4])));
  th[6] = v[5];
  th[7] = v[6];
}

// Greedy selection, one workgroup per window: rho = <d|h> / sqrt(<h|h>) of every trial (not a
// finite number: -inf); a trial replaces its member when its rho is larger.  best[w] = the
// largest rho of the window's population afterwards, best_idx[w] (if given) the smallest index
// holding it.  x and trial_x may be the same array (a first scoring of the initial population
// with s = -inf).
__global__ void __launch_bounds__(256) k_de_select(int pop, const double* __restrict__ comps, double* x, double* s,
                                                   const double* trial_x, double* __restrict__ best,
                                                   int32_t* __restrict__ best_idx) {
  __shared__ double s_red[4];
  __shared__ int s_idx[4];
  const int w = blockIdx.x;
  const int tid = threadIdx.x;
  double mx = -__builtin_inf();
  int mi = 0x7fffffff;
  for (int i = tid; i < pop; i += blockDim.x) {
    const int64_t g = (int64_t)w * pop + i;
    const double r = comps[2 * g] / sqrt(comps[2 * g + 1]);
    const double rt = isfinite(r) ? r : -__builtin_inf();
    double si = s[g];
    if (rt > si) {
      si = rt;
      s[g] = rt;
#pragma unroll
      for (int k = 0; k < kDeDim; ++k) x[kDeDim * g + k] = trial_x[kDeDim * g + k];
    }
    if (si > mx || (si == mx && i < mi)) {
      mx = si;
      mi = i;
    }
  }
  // (value, index) maximum: larger value first, then the smaller index
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(mx, o, 64);
    const int oi = __shfl_xor(mi, o, 64);
    if (ov > mx || (ov == mx && oi < mi)) {
      mx = ov;
      mi = oi;
    }
  }
  if ((tid & 63) == 0) {
    s_red[tid >> 6] = mx;
    s_idx[tid >> 6] = mi;
  }
  __syncthreads();
  if (tid == 0) {
    double v = s_red[0];
    int k = s_idx[0];
    for (int q = 1; q < 4; ++q)
      if (s_red[q] > v || (s_red[q] == v && s_idx[q] < k)) {
        v = s_red[q];
        k = s_idx[q];
      }
    best[w] = v;
    if (best_idx) best_idx[w] = k < pop ? k : 0;
  }
}

}  // namespace gbx
