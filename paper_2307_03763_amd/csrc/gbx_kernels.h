// Kernels of the Galactic-binary likelihood path (gfx950).
#pragma once

#include <type_traits>

#include "gbx_device.h"

namespace gbx {

// kernel modes; the last three are the likelihood, the templates and the gradient of numerical
// orbits (one light time per arm), kernels of their own so that the tuned equal-arm kernels keep
// their registers
enum {
  MODE_WAVEFORM = 0, MODE_LOGLIK = 1, MODE_GRAD = 2,
  MODE_LOGLIK_UNEQ = 3, MODE_WAVEFORM_UNEQ = 4, MODE_GRAD_UNEQ = 5
};

// Window descriptor as the kernels see it (device memory of a plan).
struct DevWin {
  int64_t k0;
  int64_t data_off;
  int64_t cand_off;
  int64_t n_cand;
  double dd;   // <d|d> over the whole window, filled by k_prepare
  int32_t W, N, C, prec;
};

// Work item: candidates c0 .. c0 + n - 1 (window-relative) of window `win`.
struct Tile {
  int32_t win;
  int32_t n;
  int64_t c0;
};

struct BatchArgs {
  const DevWin* wins;
  const Tile* tiles;
  int n_tiles;
  unsigned* ctr;          // [2]: dequeue counter, finished-workgroup counter
  const double* d;        // complex128 data
  const double* w;        // weights 4 / (T S)
  const double* theta;    // [rows][8]
  double* logL;           // [rows]
  double* comps;          // [rows][2] or null
  double* grad;           // [rows][8] (MODE_GRAD)
  const double* ob64;     // orbit table, FP64
  const void* obR;        // orbit table in the compute precision
  const void* tw;         // twiddles in the compute precision
  double T;
  double Lc;              // L / c
  int tdi2;               // second-generation TDI
  int64_t B;              // MODE_WAVEFORM: number of templates
  double* h_out;          // MODE_WAVEFORM: complex128 [B][C][N]
  int64_t* first_bin;     // MODE_WAVEFORM: [B]
};

// Sum over the LPC lanes of one template (lanes lane0 .. lane0+LPC-1 of the workgroup).
// LPC <= 64: butterfly shuffles inside the wave.  LPC > 64: shuffles, then one LDS step.
template <int LPC, int WPB, int NV>
__device__ __forceinline__ void slot_reduce(double v[NV], double (*s_red)[16]) {
  constexpr int WL = LPC < 64 ? LPC : 64;
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int o = WL / 2; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
  if (LPC > 64) {
    const int wave = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int i = 0; i < NV; ++i) s_red[wave][i] = v[i];
    __syncthreads();
    const int first = (threadIdx.x / LPC) * (LPC / 64);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < LPC / 64; ++k) acc += s_red[first + k][i];
      v[i] = acc;
    }
    __syncthreads();
  }
}

// Whether the short sinc series covers every link argument of every template in this wave:
// |u| = x |1 -+ k.n| <= 2 pi f L / c with f the largest local frequency f0 + max(0, fdot T).
// The vote makes the choice uniform over the wave, so the sample loop does not diverge.
template <class R>
__device__ __forceinline__ bool wave_sinc_short(const Cand<R>& s, const BatchArgs& a) {
  const double fhi = s.f0 + fmax(0.0, s.fd * a.T);
  return __all(2.0 * kPi * fhi * a.Lc <= sinc_short_max<R>());
}

// Calls body(tdi2, short) with the two compile-time choices of a template's sample loops: the TDI
// generation (uniform over the launch) and the short sinc series (uniform over the wave).
template <class F>
__device__ __forceinline__ void with_loop_flags(bool tdi2, bool shrt, F&& body) {
  if (tdi2) {
    if (shrt) body(std::true_type{}, std::true_type{});
    else body(std::true_type{}, std::false_type{});
  } else {
    if (shrt) body(std::false_type{}, std::true_type{});
    else body(std::false_type{}, std::false_type{});
  }
}

// The slow-series samples of one lane, one at a time (keeps the live state of a single sample
// in registers); TDI2 and SHORT are compile-time choices (with_loop_flags), so that the
// branches on them are taken once per template, outside the loop; UNEQ (numerical orbits) is
// the kernel's own.
template <class R, int N, int LPC, int C, bool TDI2, bool SHORT, bool UNEQ>
__device__ __forceinline__ void series_samples(const Cand<R>& s, const BatchArgs& a, int lane, cplx<R>* buf) {
  constexpr int E = N / LPC;
  const R* obR = (const R*)a.obR;
#pragma unroll 1
  for (int e = 0; e < E; ++e) {
    const int m = lane + LPC * e;
    const double t = a.T * (double)m / (double)N;
    cplx<R> o[C];
    if constexpr (UNEQ)
      slow_sample_uneq<R, C, TDI2>(s, a.ob64, obR, N, m, t, o);
    else
      slow_sample<R, C, TDI2, SHORT>(s, a.ob64, obR, N, m, t, a.Lc, o);
#pragma unroll
    for (int c = 0; c < C; ++c) buf[c * N + m] = o[c];
  }
}

// Slow series of one template into LDS (all its lanes), then the forward DFT.  UNEQ: one light
// time per arm (slow_sample_uneq, general sinc).
template <class R, int N, int LPC, int C, bool UNEQ = false>
__device__ __forceinline__ void template_to_lds(const Cand<R>& s, const BatchArgs& a, int lane, cplx<R>* buf) {
  if constexpr (UNEQ) {
    with_loop_flags(a.tdi2 != 0, false, [&](auto tdi2, auto) {
      series_samples<R, N, LPC, C, decltype(tdi2)::value, false, true>(s, a, lane, buf);
    });
  } else {
    with_loop_flags(a.tdi2 != 0, wave_sinc_short<R>(s, a), [&](auto tdi2, auto shrt) {
      series_samples<R, N, LPC, C, decltype(tdi2)::value, decltype(shrt)::value, false>(s, a, lane, buf);
    });
  }
  slot_sync<LPC>();
  fft_lds<R, N, LPC, C, -1>(buf, lane, (const cplx<R>*)a.tw);
}

// logL and components of one template against one window.
template <class R, int N, int LPC, int C, int WPB, bool UNEQ>
__device__ __forceinline__ void process_loglik(const BatchArgs& a, const DevWin& w, int64_t row, bool active,
                                               int lane, cplx<R>* buf, double (*s_red)[16]) {
  constexpr int E = N / LPC;
  const Cand<R> s = make_cand<R>(a.theta + 8 * row, a.T);
  template_to_lds<R, N, LPC, C, UNEQ>(s, a, lane, buf);
  const double scale = s.amp * a.T / (2.0 * (double)N);
  // <d|h> and <h|h> over the overlap.  The template is zero outside it, so
  // -<d-h|d-h>/2 = -dd/2 + <d|h> - <h|h>/2 with dd the window's data norm.
  double acc[2] = {0.0, 0.0};
  const int64_t off = w.data_off;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = lane + LPC * e;
    const int j = idx < N / 2 ? idx : idx - N;
    const int64_t kk = s.q + j - w.k0;
    if (kk >= 0 && kk < w.W) {
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const cplx<R> hv = buf[c * N + idx];
        const double sc = scale * chan_norm(c);
        const double hre = (double)hv.x * sc, him = (double)hv.y * sc;
        const int64_t g = off + (int64_t)c * w.W + kk;
        const double dre = a.d[2 * g], dim = a.d[2 * g + 1], wk = a.w[g];
        acc[0] += wk * (dre * hre + dim * him);
        acc[1] += wk * (hre * hre + him * him);
      }
    }
  }
  slot_reduce<LPC, WPB, 2>(acc, s_red);
  if (lane == 0 && active) {
    const double nan = __builtin_nan("");
    a.logL[row] = s.ok ? (acc[0] - 0.5 * acc[1]) - 0.5 * w.dd : nan;
    if (a.comps) {
      a.comps[2 * row] = s.ok ? acc[0] : nan;
      a.comps[2 * row + 1] = s.ok ? acc[1] : nan;
    }
  }
  slot_sync<LPC>();
}

// logL and its gradient for one template.  Forward: slow series, DFT, residual.  The
// cotangent c_k = A T/(2N) n_c w_k (d_k - h_k) (n_c the channel normalisation) replaces the
// template in LDS, an inverse DFT turns it into the cotangent of every slow-series sample,
// and each lane contracts it with the derivative of its samples (grad_sample_rev).  The
// amplitude and the three extrinsic angles enter through closed forms; the carrier bin is
// held fixed.
template <class R, int N, int LPC, int C, int WPB, bool UNEQ>
__device__ __forceinline__ void process_grad(const BatchArgs& a, const DevWin& w, int64_t row, bool active,
                                             int lane, cplx<R>* buf, double (*s_red)[16]) {
  constexpr int E = N / LPC;
  const double* th = a.theta + 8 * row;
  const Cand<R> s = make_cand<R>(th, a.T);
  const CandG<R> sg = make_cand_grad<R>(th, s.ok);
  template_to_lds<R, N, LPC, C, UNEQ>(s, a, lane, buf);
  const double sc0 = a.T / (2.0 * (double)N);
  const double scale = s.amp * sc0;
  // v: 0 dlogL/dA = sum w Re((d-h) conj(h_u)), 1 <h_u|h_u>, 2 gf, 3 gtf, 4 gb, 5 gl, 6..9 GU, GV,
  // 10 pt, 11 ptt; h = A h_u.  With r = d - h, -<r|r>/2 = -dd/2 + A v0 + A^2 v1 / 2 (the
  // template is zero outside the overlap).
  double v[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) v[i] = 0.0;
  const int64_t off = w.data_off;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = lane + LPC * e;
    const int j = idx < N / 2 ? idx : idx - N;
    const int64_t kk = s.q + j - w.k0;
    const bool inw = kk >= 0 && kk < w.W;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      cplx<R> cot = mk<R>((R)0, (R)0);
      if (inw) {
        const cplx<R> hv = buf[c * N + idx];
        const double scu = sc0 * chan_norm(c), scn = scale * chan_norm(c);
        const double hur = (double)hv.x * scu, hui = (double)hv.y * scu;
        const double hre = hur * s.amp, him = hui * s.amp;
        const int64_t g = off + (int64_t)c * w.W + kk;
        const double dre = a.d[2 * g], dim = a.d[2 * g + 1], wk = a.w[g];
        const double rre = dre - hre, rim = dim - him;
        v[0] += wk * (rre * hur + rim * hui);
        v[1] += wk * (hur * hur + hui * hui);
        cot = mk<R>((R)(scn * wk * rre), (R)(scn * wk * rim));
      }
      buf[c * N + idx] = cot;
    }
  }
  slot_sync<LPC>();
  fft_lds<R, N, LPC, C, +1>(buf, lane, (const cplx<R>*)a.tw);
  GradAcc& ga = *reinterpret_cast<GradAcc*>(&v[2]);  // v[2..11]: per-sample accumulators
  const R* obR = (const R*)a.obR;
  auto samples = [&](auto tdi2, auto shrt) {
    constexpr bool TDI2 = decltype(tdi2)::value, SHORT = decltype(shrt)::value;
#pragma unroll 1
    for (int e = 0; e < E; ++e) {
      const int m = lane + LPC * e;
      const double t = a.T * (double)m / (double)N;
      cplx<R> sbar[C];
#pragma unroll
      for (int c = 0; c < C; ++c) sbar[c] = buf[c * N + m];
      if constexpr (UNEQ)
        grad_sample_uneq<R, C, TDI2>(s, sg, a.ob64, obR, N, m, t, sbar, ga);
      else
        grad_sample_rev<R, C, TDI2, SHORT>(s, sg, a.ob64, obR, N, m, t, a.Lc, sbar, ga);
    }
  };
  // one branch per template, outside the loop
  with_loop_flags(a.tdi2 != 0, UNEQ ? false : wave_sinc_short<R>(s, a), samples);
  slot_reduce<LPC, WPB, 12>(v, s_red);
  if (lane == 0 && active) {
    const double nan = __builtin_nan("");
    double* g = a.grad + 8 * row;
    if (!s.ok) {
      a.logL[row] = nan;
      for (int i = 0; i < 8; ++i) g[i] = nan;
    } else {
      a.logL[row] = s.amp * (v[0] + 0.5 * s.amp * v[1]) - 0.5 * w.dd;
      double si, ci, s2, c2;
      sincos_rad(th[5], &si, &ci);
      sincos_rad(2.0 * th[6], &s2, &c2);
      const double Ap = 1.0 + ci * ci, Ac = -2.0 * ci;
      const double apx = Ap * c2, apy = Ac * s2, axx = Ap * s2, axy = -Ac * c2;
      const double gur = ga.gu_re, gui = ga.gu_im, gvr = ga.gv_re, gvi = ga.gv_im;
      auto re_lin = [&](double px, double py, double qx, double qy) { return px * gur - py * gui + qx * gvr - qy * gvi; };
      const double dAp = -2.0 * ci * si, dAc = 2.0 * si;
      g[0] = ga.gf - 2.0 * kPi * ga.pt;
      g[1] = ga.gtf - kPi * ga.ptt;
      g[2] = ga.gb;
      g[3] = ga.gl;
      g[4] = v[0];
      g[5] = re_lin(dAp * c2, dAc * s2, dAp * s2, -dAc * c2);
      g[6] = re_lin(-2.0 * Ap * s2, 2.0 * Ac * c2, 2.0 * Ap * c2, 2.0 * Ac * s2);
      g[7] = -(apx * gui + apy * gur + axx * gvi + axy * gvr);
    }
  }
  slot_sync<LPC>();
}

// Persistent batched kernel: workgroups take tiles from the plan's queue until it is empty.
// The last workgroup to finish resets the queue counters for the next launch.
template <class R, int N, int LPC, int C, int WPB, int MODE, int OCC>
__global__ void __launch_bounds__(WPB * 64, OCC) k_batch(BatchArgs a) {
  constexpr int CPB = WPB * 64 / LPC;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_tile;
  __shared__ double s_red[WPB][16];
  const int tid = threadIdx.x;
  const int slot = tid / LPC, lane = tid % LPC;
  cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem) + slot * C * N;
  for (;;) {
    if (tid == 0) s_tile = (int)atomicAdd(a.ctr, 1u);
    __syncthreads();
    const int t = s_tile;
    __syncthreads();
    if (t >= a.n_tiles) break;
    const Tile tl = a.tiles[t];
    const DevWin w = a.wins[tl.win];
    for (int c0 = 0; c0 < tl.n; c0 += CPB) {
      const int ci = c0 + slot;
      const bool active = ci < tl.n;
      const int64_t row = w.cand_off + tl.c0 + (active ? ci : 0);
      if (MODE == MODE_LOGLIK || MODE == MODE_LOGLIK_UNEQ)
        process_loglik<R, N, LPC, C, WPB, MODE == MODE_LOGLIK_UNEQ>(a, w, row, active, lane, buf, s_red);
      if (MODE == MODE_GRAD || MODE == MODE_GRAD_UNEQ)
        process_grad<R, N, LPC, C, WPB, MODE == MODE_GRAD_UNEQ>(a, w, row, active, lane, buf, s_red);
    }
  }
  if (tid == 0) {
    __threadfence();
    const unsigned done = atomicAdd(a.ctr + 1, 1u);
    if (done == gridDim.x - 1) {
      atomicExch(a.ctr, 0u);
      atomicExch(a.ctr + 1, 0u);
    }
  }
}

// Templates on their own bins: one workgroup per CPB templates.  UNEQ: numerical orbits.
template <class R, int N, int LPC, int C, int WPB, bool UNEQ = false>
__global__ void __launch_bounds__(WPB * 64) k_waveform(BatchArgs a) {
  constexpr int CPB = WPB * 64 / LPC;
  constexpr int E = N / LPC;
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int slot = tid / LPC, lane = tid % LPC;
  cplx<R>* buf = reinterpret_cast<cplx<R>*>(smem) + slot * C * N;
  const int64_t row0 = (int64_t)blockIdx.x * CPB + slot;
  const bool active = row0 < a.B;
  const int64_t row = active ? row0 : 0;
  const Cand<R> s = make_cand<R>(a.theta + 8 * row, a.T);
  template_to_lds<R, N, LPC, C, UNEQ>(s, a, lane, buf);
  if (!active) return;
  const double scale = s.amp * a.T / (2.0 * (double)N);
  const double nan = __builtin_nan("");
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = lane + LPC * e;
    const int i = (idx + N / 2) & (N - 1);  // bin q - N/2 + i holds DFT index (i - N/2) mod N
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const cplx<R> hv = buf[c * N + idx];
      const int64_t g = (row * C + c) * N + i;
      a.h_out[2 * g] = s.ok ? (double)hv.x * (scale * chan_norm(c)) : nan;
      a.h_out[2 * g + 1] = s.ok ? (double)hv.y * (scale * chan_norm(c)) : nan;
    }
  }
  if (lane == 0) a.first_bin[row] = s.q - N / 2;
}

}  // namespace gbx
