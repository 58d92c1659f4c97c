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
// taken indices in increasing order).  Mutant a + F (b - c), folded back into the box (periodic
// coordinates wrap, the others reflect at the walls and are clipped); binomial crossover with
// rate cr, the coordinate floor(u_j 7) always from the mutant.  The arithmetic is not contracted
// into fused multiply-adds, so that it rounds as the plain reference does.
__global__ void __launch_bounds__(256) k_de_trial(int n_win, int pop, const double* __restrict__ lo,
                                                  const double* __restrict__ hi, const double* __restrict__ x,
                                                  const double* __restrict__ u_idx, const double* __restrict__ u_cross,
                                                  const double* __restrict__ u_j, const double* __restrict__ F,
                                                  double cr, double amp, double* __restrict__ trial_x,
                                                  double* __restrict__ trial_theta) {
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
  const double* xa = x + ((int64_t)w * pop + a) * kDeDim;
  const double* xb = x + ((int64_t)w * pop + b) * kDeDim;
  const double* xc = x + ((int64_t)w * pop + c) * kDeDim;
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
// largest rho of the window's population afterwards.  x and trial_x may be the same array
// (a first scoring of the initial population with s = -inf).
__global__ void __launch_bounds__(256) k_de_select(int pop, const double* __restrict__ comps, double* x, double* s,
                                                   const double* trial_x, double* __restrict__ best) {
  __shared__ double s_red[4];
  const int w = blockIdx.x;
  const int tid = threadIdx.x;
  double mx = -__builtin_inf();
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
    mx = fmax(mx, si);
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((tid & 63) == 0) s_red[tid >> 6] = mx;
  __syncthreads();
  if (tid == 0) best[w] = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
}

}  // namespace gbx
