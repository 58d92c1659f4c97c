// Device-side building blocks of the Galactic-binary likelihood for gfx950.
//
// Model (paper: Strub et al., arXiv:2307.03763, Sec. II channels and Sec. III parameters;
// the response model itself is this project's reading of the cited literature):
//   plane wave H = Re[(A+ e+ - i Ax ex) e^{i Phi(t - k.x/c)}], Phi = 2 pi f0 t + pi fdot t^2 + phi0,
//   single link (light s -> r over L):  z_rs = -i (pi f L/c) sinc(u_rs) (n.H.n)
//                                          e^{i[Phi - 2 pi f (L/2 + k.(x_r + x_s)/2)/c]},
//   first-generation TDI  X = (1 - D^2)[(z13 + D z31) - (z12 + D z21)], D = e^{-2 pi i f L/c};
//   second generation (equal arms): X2 = (1 - D^4) X, the eight further links being the copy of
//   X delayed by four arm lengths with the opposite sign,
//   A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3  (Sec. II),
//   slow series S(t_m) = response with the carrier e^{2 pi i q t/T} removed, q = floor(f0 T),
//   template h(q + j) = T/(2N) DFT_N[S](j mod N), j in [-N/2, N/2).
// Layout of the per-sample work, shared by every kernel variant:
//   common phase p = df t + fdot t^2/2 + phi0/(2pi) - f (L/(2c) + k.R/c)   [cycles, FP64]
//   per arm a (opposite spacecraft o):  P_a = (a+ F+_a + ax Fx_a) e^{i pi f k.dx_o / c}
//   per link: sinc(u), u = pi f L (1 -+ k.n_a)/c
//   X, Y, Z from P_a and the six sincs; K = (1 - D^2)(-i pi f L/c) e^{2 pi i p} applied once.
// The amplitude is factored out (templates are computed for A = 1 and scaled in FP64), so
// FP32 intermediates stay O(1) whatever the amplitude.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbx {

constexpr double kPi = 3.14159265358979323846;
constexpr double kC = 299792458.0;

// orbit table fields, each an array of N samples (structure of arrays)
enum {
  OB_RX = 0, OB_RY = 1,                          // guiding centre / c (s), FP64 only
  OB_N12 = 2, OB_N23 = 5, OB_N31 = 8,            // unit arm vectors (x1-x2)/|.|, (x2-x3)/|.|, (x3-x1)/|.|
  OB_P1 = 11, OB_P2 = 14, OB_P3 = 17,            // spacecraft offsets from the guiding centre / c (s)
  OB_RZ = 20,                                    // guiding centre z / c (s), FP64; 0 for the analytic orbits
  OB_LT12 = 21, OB_LT23 = 22, OB_LT31 = 23,      // arm light times |x_r - x_s| / c (s)
  OB_FIELDS = 24
};

// Normalisation of channel c: A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3
// (Sec. II).  The slow series hold the X, Y, Z combinations without it; it is applied in FP64
// with the amplitude after the DFT.
__device__ __forceinline__ constexpr double chan_norm(int c) {
  return c == 0 ? 0.70710678118654752440 : c == 1 ? 0.40824829046386301637 : 0.57735026918962576451;
}

template <class R>
struct cplx {
  R x, y;
};

template <class R>
__device__ __forceinline__ cplx<R> mk(R x, R y) {
  cplx<R> z;
  z.x = x;
  z.y = y;
  return z;
}
template <class R>
__device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <class R>
__device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <class R>
__device__ __forceinline__ cplx<R> operator*(cplx<R> a, cplx<R> b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <class R>
__device__ __forceinline__ cplx<R> scal(cplx<R> a, R s) { return mk<R>(a.x * s, a.y * s); }
template <class R>
__device__ __forceinline__ cplx<R> conjg(cplx<R> a) { return mk<R>(a.x, -a.y); }
template <class R>
__device__ __forceinline__ cplx<R> mul_i(cplx<R> a) { return mk<R>(-a.y, a.x); }     // i a
template <class R>
__device__ __forceinline__ cplx<R> mul_mi(cplx<R> a) { return mk<R>(a.y, -a.x); }    // -i a

// sin and cos of 2 pi x, x in revolutions (FP64).  Quadrant reduction x = n/4 + r with
// n = rint(4x) and |r| <= 1/8 (both steps exact for |x| < 2^50), the Taylor series of sin and
// cos at theta = 2 pi r, |theta| <= pi/4 (first omitted terms: theta^17/17! < 5e-17 and
// theta^18/18! < 3e-18), then a rotation by n quarter turns (n mod 4 formed in FP64, exact,
// so that no 64-bit integer conversion is needed).
__device__ __forceinline__ void sincos_rev(double x, double* s, double* c) {
  const double n = rint(4.0 * x);
  const double r = fma(n, -0.25, x);
  const double th = r * (2.0 * kPi);
  const double t2 = th * th;
  double ps = -1.0 / 1307674368000.0;      // -1/15!
  ps = fma(ps, t2, 1.0 / 6227020800.0);    // 1/13!
  ps = fma(ps, t2, -1.0 / 39916800.0);     // -1/11!
  ps = fma(ps, t2, 1.0 / 362880.0);        // 1/9!
  ps = fma(ps, t2, -1.0 / 5040.0);         // -1/7!
  ps = fma(ps, t2, 1.0 / 120.0);           // 1/5!
  ps = fma(ps, t2, -1.0 / 6.0);            // -1/3!
  const double sn = fma(ps * t2, th, th);
  double pc = 1.0 / 20922789888000.0;      // 1/16!
  pc = fma(pc, t2, -1.0 / 87178291200.0);  // -1/14!
  pc = fma(pc, t2, 1.0 / 479001600.0);     // 1/12!
  pc = fma(pc, t2, -1.0 / 3628800.0);      // -1/10!
  pc = fma(pc, t2, 1.0 / 40320.0);         // 1/8!
  pc = fma(pc, t2, -1.0 / 720.0);          // -1/6!
  pc = fma(pc, t2, 1.0 / 24.0);            // 1/4!
  pc = fma(pc, t2, -0.5);                  // -1/2!
  const double cs = fma(pc, t2, 1.0);
  // e^{i 2 pi x} = i^n e^{i theta}
  const int q = (int)fma(floor(n * 0.25), -4.0, n);  // n mod 4, in {0, 1, 2, 3}
  const double a = (q & 1) ? cs : sn, b = (q & 1) ? sn : cs;
  *s = (q & 2) ? -a : a;
  *c = (q == 1 || q == 2) ? -b : b;
}
// sin and cos of 2 pi x for |x| <= 0.07 revolution (|theta| <= 0.44), by the Taylor series at
// theta = 2 pi x with no reduction: sin to theta^13 and cos to theta^14 (first omitted terms
// below 4e-18 and 1e-19).  The spacecraft phase factors take it where the short sinc series
// applies: 2 pi f L/c <= 1.5 bounds their argument f k.p/(2c), |p| = L/sqrt3, by 0.069.
// FP32 keeps the hardware unit.
__device__ __forceinline__ void sincos_rev_small(double x, double* s, double* c) {
  const double th = x * (2.0 * kPi);
  const double t2 = th * th;
  double ps = 1.0 / 6227020800.0;          // 1/13!
  ps = fma(ps, t2, -1.0 / 39916800.0);     // -1/11!
  ps = fma(ps, t2, 1.0 / 362880.0);        // 1/9!
  ps = fma(ps, t2, -1.0 / 5040.0);         // -1/7!
  ps = fma(ps, t2, 1.0 / 120.0);           // 1/5!
  ps = fma(ps, t2, -1.0 / 6.0);            // -1/3!
  *s = fma(ps * t2, th, th);
  double pc = 1.0 / 87178291200.0;         // 1/14!
  pc = fma(pc, t2, -1.0 / 479001600.0);    // -1/12!
  pc = fma(pc, t2, 1.0 / 3628800.0);       // 1/10!
  pc = fma(pc, t2, -1.0 / 40320.0);        // -1/8!
  pc = fma(pc, t2, 1.0 / 720.0);           // 1/6!
  pc = fma(pc, t2, -1.0 / 24.0);           // -1/4!
  pc = fma(pc, t2, 0.5);                   // 1/2!
  *c = fma(-pc, t2, 1.0);
}
__device__ __forceinline__ void sincos_rev_small(float x, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(x);
  *c = __builtin_amdgcn_cosf(x);
}

// The link delay D = e^{-2 i x} (x = pi f L/c) for 0 <= x <= 0.75, where the short sinc series
// applies (2 pi f L/c <= 1.5): the Taylor series of sin x to x^17 and cos x to x^16 (first
// omitted terms below 4e-20 and 1e-18 at 0.75), no reduction, then the double angle:
// sin(-2x) = -2 sin x cos x, cos 2x = 1 - 2 sin^2 x.
__device__ __forceinline__ void delay_short(double x, double* sD, double* cD) {
  const double x2 = x * x;
  double ps = 1.0 / 355687428096000.0;     // 1/17!
  ps = fma(ps, x2, -1.0 / 1307674368000.0);  // -1/15!
  ps = fma(ps, x2, 1.0 / 6227020800.0);    // 1/13!
  ps = fma(ps, x2, -1.0 / 39916800.0);     // -1/11!
  ps = fma(ps, x2, 1.0 / 362880.0);        // 1/9!
  ps = fma(ps, x2, -1.0 / 5040.0);         // -1/7!
  ps = fma(ps, x2, 1.0 / 120.0);           // 1/5!
  ps = fma(ps, x2, -1.0 / 6.0);            // -1/3!
  const double sx = fma(ps * x2, x, x);
  double pc = 1.0 / 20922789888000.0;      // 1/16!
  pc = fma(pc, x2, -1.0 / 87178291200.0);  // -1/14!
  pc = fma(pc, x2, 1.0 / 479001600.0);     // 1/12!
  pc = fma(pc, x2, -1.0 / 3628800.0);      // -1/10!
  pc = fma(pc, x2, 1.0 / 40320.0);         // 1/8!
  pc = fma(pc, x2, -1.0 / 720.0);          // -1/6!
  pc = fma(pc, x2, 1.0 / 24.0);            // 1/4!
  pc = fma(pc, x2, -0.5);                  // -1/2!
  const double cx = fma(pc, x2, 1.0);
  *sD = -2.0 * sx * cx;
  *cD = fma(-2.0 * sx, sx, 1.0);
}

// sin and cos of an angle x in radians: x = n 2 pi + r by a two-part 2 pi (Cody-Waite:
// the head is 2 pi rounded to double, the tail the next 53 bits; each product is removed with
// one rounding), then sincos_rev of r / 2 pi.  Absolute error about 5e-16 for |x| up to 1e6.
// Used for the per-candidate angles, in place of the general library routine (whose
// large-argument machinery every lane of a template would run).
__device__ __forceinline__ void sincos_rad(double x, double* s, double* c) {
  const double n = rint(x * (0.5 / kPi));
  double r = fma(-n, 6.283185307179586, x);  // 2 pi, head
  r = fma(-n, 2.4492935982947064e-16, r);    // 2 pi, tail
  sincos_rev(r * (0.5 / kPi), s, c);
}

// FP32: the hardware transcendentals, which take their argument in revolutions (|x| <= 1 on
// every call here).
__device__ __forceinline__ void sincos_rev(float x, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(x);
  *c = __builtin_amdgcn_cosf(x);
}

// sin and cos of 2 pi x for an FP64 argument x in revolutions, in precision R, reduced to the
// nearest quarter turn in FP64.  In FP32 the reduced r (|r| <= 1/8) is rounded; its sine comes
// from the Taylor series to t^9 at t = 2 pi r (next term below 3e-9), so it keeps its relative
// accuracy near zero, and its cosine (at least 0.7) from the hardware.  After the rotation by
// the quarter turns each component is accurate relative to its own size near its zeros.
// Rounding x to FP32 first (as sincos_rev does) leaves an absolute error of about 2e-7 there,
// which the TDI factors 1 - D^2 and 1 - D^4 of the link delay turn into a relative template
// error of that size over their value: near their nulls (f near c / 2L, and c / 4L for the
// second generation) it grows without bound.
__device__ __forceinline__ void sincos_rev_red(double x, double* s, double* c) { sincos_rev(x, s, c); }
__device__ __forceinline__ void sincos_rev_red(double x, float* s, float* c) {
  const double n = rint(4.0 * x);
  const float r = (float)(x - 0.25 * n);
  const float t = r * 6.28318530717958647692f;
  const float t2 = t * t;
  float ps = 1.0f / 362880.0f;              // 1/9!
  ps = ps * t2 - 1.0f / 5040.0f;            // -1/7!
  ps = ps * t2 + 1.0f / 120.0f;             // 1/5!
  ps = ps * t2 - 1.0f / 6.0f;               // -1/3!
  const float sr = t + t * (t2 * ps);
  const float cr = __builtin_amdgcn_cosf(r);
  // rotate by the n quarter turns (n mod 4 of a two's-complement integer)
  const int q = (int)n & 3;
  *s = q == 0 ? sr : q == 1 ? cr : q == 2 ? -sr : -cr;
  *c = q == 0 ? cr : q == 1 ? -sr : q == 2 ? -cr : sr;
}

// sin(u)/u.  For |u| <= 2 the Taylor series in u^2 (next term below 2e-18 in FP64 and 2e-10
// in FP32 there), the quotient beyond (frequencies above c / (pi L)).
__device__ __forceinline__ double sinc_r(double u) {
  if (fabs(u) <= 2.0) {
    const double u2 = u * u;
    double p = -1.0 / 25852016738884976640000.0;  // -1/23!
    p = p * u2 + 1.0 / 51090942171709440000.0;     // 1/21!
    p = p * u2 - 1.0 / 121645100408832000.0;       // -1/19!
    p = p * u2 + 1.0 / 355687428096000.0;          // 1/17!
    p = p * u2 - 1.0 / 1307674368000.0;            // -1/15!
    p = p * u2 + 1.0 / 6227020800.0;               // 1/13!
    p = p * u2 - 1.0 / 39916800.0;                 // -1/11!
    p = p * u2 + 1.0 / 362880.0;                   // 1/9!
    p = p * u2 - 1.0 / 5040.0;                     // -1/7!
    p = p * u2 + 1.0 / 120.0;                      // 1/5!
    p = p * u2 - 1.0 / 6.0;                        // -1/3!
    return p * u2 + 1.0;
  }
  double sn, cs;
  sincos_rev(u * (0.5 / kPi), &sn, &cs);
  return sn / u;
}
__device__ __forceinline__ float sinc_r(float u) {
  if (fabsf(u) <= 2.0f) {
    const float u2 = u * u;
    float p = -1.0f / 1307674368000.0f;            // -1/15!
    p = p * u2 + 1.0f / 6227020800.0f;             // 1/13!
    p = p * u2 - 1.0f / 39916800.0f;               // -1/11!
    p = p * u2 + 1.0f / 362880.0f;                 // 1/9!
    p = p * u2 - 1.0f / 5040.0f;                   // -1/7!
    p = p * u2 + 1.0f / 120.0f;                    // 1/5!
    p = p * u2 - 1.0f / 6.0f;                      // -1/3!
    return p * u2 + 1.0f;
  }
  return __builtin_amdgcn_sinf(u * (float)(0.5 / kPi)) / u;
}

// The short series: for link arguments |u| <= sinc_short_max<R>(), FP64 ten terms (the next,
// u^20/21!, is below 7e-17 at 1.5) and FP32 five terms (u^10/11! below 3e-8 at 1.0).  A template
// takes it when every lane of its wave has all six link arguments in that range (frequencies up
// to about 28 and 19 mHz), so no quotient is needed there.
template <class R>
__device__ __forceinline__ constexpr double sinc_short_max() { return sizeof(R) == 8 ? 1.5 : 1.0; }
__device__ __forceinline__ double sinc_short(double u) {
  const double u2 = u * u;
  double p = -1.0 / 121645100408832000.0;  // -1/19!
  p = p * u2 + 1.0 / 355687428096000.0;     // 1/17!
  p = p * u2 - 1.0 / 1307674368000.0;       // -1/15!
  p = p * u2 + 1.0 / 6227020800.0;          // 1/13!
  p = p * u2 - 1.0 / 39916800.0;            // -1/11!
  p = p * u2 + 1.0 / 362880.0;              // 1/9!
  p = p * u2 - 1.0 / 5040.0;                // -1/7!
  p = p * u2 + 1.0 / 120.0;                 // 1/5!
  p = p * u2 - 1.0 / 6.0;                   // -1/3!
  return p * u2 + 1.0;
}
__device__ __forceinline__ float sinc_short(float u) {
  const float u2 = u * u;
  float p = 1.0f / 362880.0f;               // 1/9!
  p = p * u2 - 1.0f / 5040.0f;              // -1/7!
  p = p * u2 + 1.0f / 120.0f;               // 1/5!
  p = p * u2 - 1.0f / 6.0f;                 // -1/3!
  return p * u2 + 1.0f;
}
template <class R, bool SHORT>
__device__ __forceinline__ R sinc_sel(R u) {
  if (SHORT) return sinc_short(u);
  return sinc_r(u);
}

// Per-candidate constants (computed once per template, replicated over its lanes).
template <class R>
struct Cand {
  double f0, fd, df, phi0c;   // f0, fdot, f0 - q/T, phi0 / 2 pi
  double kxd, kyd, kzd;       // k in FP64 for k.R (the only large phase term)
  int64_t q;                  // carrier bin floor(f0 T)
  R k[3], u[3], v[3];         // propagation direction and transverse basis
  cplx<R> ap, ax;             // n.H.n = ap F+ + ax Fx for unit amplitude
  double amp;                 // amplitude (applied in FP64 after the DFT)
  bool ok;                    // parameters in the domain of the model
};

// theta = (f0, fdot, beta, lambda, A, iota, psi, phi0).  Out-of-domain candidates get a
// harmless stand-in so every lane still runs the same schedule; `ok` marks them.
template <class R>
__device__ __forceinline__ Cand<R> make_cand(const double* th, double T) {
  Cand<R> s;
  double f0 = th[0], fd = th[1], be = th[2], la = th[3], amp = th[4], io = th[5], ps = th[6], ph = th[7];
  bool ok = isfinite(f0) && isfinite(fd) && isfinite(be) && isfinite(la) && isfinite(amp) &&
            isfinite(io) && isfinite(ps) && isfinite(ph) && f0 > 0.0 && f0 * T < 4.0e15 && amp >= 0.0;
  if (!ok) {
    f0 = 1e-3; fd = 0.0; be = 0.0; la = 0.0; amp = 0.0; io = 0.0; ps = 0.0; ph = 0.0;
  }
  s.ok = ok;
  s.f0 = f0;
  s.fd = fd;
  s.amp = amp;
  s.q = (int64_t)floor(f0 * T);
  s.df = f0 - (double)s.q / T;
  s.phi0c = ph * (0.5 / kPi);
  double sb, cb, sl, cl, s2, c2, si, ci;
  sincos_rad(be, &sb, &cb);
  sincos_rad(la, &sl, &cl);
  sincos_rad(2.0 * ps, &s2, &c2);
  sincos_rad(io, &si, &ci);
  (void)si;
  s.kxd = -cb * cl;
  s.kyd = -cb * sl;
  s.kzd = -sb;
  s.k[0] = (R)(-cb * cl);
  s.k[1] = (R)(-cb * sl);
  s.k[2] = (R)(-sb);
  s.u[0] = (R)(sb * cl);
  s.u[1] = (R)(sb * sl);
  s.u[2] = (R)(-cb);
  s.v[0] = (R)sl;
  s.v[1] = (R)(-cl);
  s.v[2] = (R)0;
  const double Ap = 1.0 + ci * ci, Ac = -2.0 * ci;  // per unit amplitude
  // n.(A+ e+ - i Ax ex).n with e+ = c2 eps+ + s2 epsx, ex = c2 epsx - s2 eps+:
  //   = F+ (A+ c2 + i Ax s2) + Fx (A+ s2 - i Ax c2)
  s.ap = mk<R>((R)(Ap * c2), (R)(Ac * s2));
  s.ax = mk<R>((R)(Ap * s2), (R)(-Ac * c2));
  return s;
}

// Element m of field f of an orbit table [OB_FIELDS][N].  BUF (the FP64 kernels) reads through a
// buffer resource over the whole table: the per-lane byte offset of sample m (one VGPR, shared
// by the fourteen reads of a sample) plus the field's row offset as a scalar, so no per-lane
// 64-bit address arithmetic is formed; the resource's word 3 is the gfx9-family raw-buffer
// setting, and a read past the table's bytes would return zero (m never leaves [0, N)).
// Measured: the FP64 short sample loop loses 30 of its 457 instructions; the single-precision
// kernels, whose scalar registers are scarcer, ran slower with it and index plainly.
template <bool BUF, class T>
__device__ __forceinline__ T ob_at(const T* __restrict__ tab, int f, int N, int m) {
  if constexpr (BUF) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(tab), (short)0, OB_FIELDS * N * (int)sizeof(T), 0x00020000);
    const int boff = m * (int)sizeof(T), soff = f * N * (int)sizeof(T);
    T x;
    if constexpr (sizeof(T) == 8) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, boff, soff, 0);
      __builtin_memcpy(&x, &v, 8);
    } else {
      const auto v = __builtin_amdgcn_raw_buffer_load_b32(r, boff, soff, 0);
      __builtin_memcpy(&x, &v, 4);
    }
    return x;
  } else {
    return tab[f * N + m];
  }
}

// One sample of the slow series of channels A, E[, T] (without their normalisations) for unit
// amplitude at t = tab time m.
// ob64: FP64 orbit table [OB_FIELDS][N]; obR: the same in precision R (fields >= OB_N12).
template <class R, int C, bool TDI2, bool SHORT>
__device__ __forceinline__ void slow_sample(const Cand<R>& s, const double* __restrict__ ob64,
                                            const R* __restrict__ obR, int N, int m, double t,
                                            double Lc, cplx<R> out[C]) {
  constexpr bool BUF = sizeof(R) == 8;  // orbit reads through a buffer resource (ob_at)
  // common phase in cycles (FP64), reduced to [-1/2, 1/2]
  const double f = s.f0 + s.fd * t;
  const double kR = s.kxd * ob_at<BUF>(ob64, OB_RX, N, m) + s.kyd * ob_at<BUF>(ob64, OB_RY, N, m);
  double p = s.df * t + 0.5 * s.fd * t * t + s.phi0c - f * (0.5 * Lc + kR);
  p -= rint(p);
  R sp, cp;
  sincos_rev((R)p, &sp, &cp);
  const R fr = (R)f;
  const R x = fr * (R)(kPi * Lc);  // pi f L / c
  R sD, cD;
  if constexpr (SHORT && sizeof(R) == 8)
    delay_short(x, &sD, &cD);  // D = e^{-2 pi i f L/c}, from x = pi f L/c
  else if constexpr (SHORT)
    sincos_rev(-fr * (R)Lc, &sD, &cD);
  else
    sincos_rev_red(-f * Lc, &sD, &cD);  // up to the transfer nulls of the TDI factors

  // projections on the arms; the arm vectors of the rigid triangle sum to zero, so the third
  // arm's projections are minus the sum of the other two
  R kn[3], un[3], vn[3], Fp[3], Fx[3];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int o = OB_N12 + 3 * a;
    const R n0 = ob_at<BUF>(obR, o + 0, N, m), n1 = ob_at<BUF>(obR, o + 1, N, m), n2 = ob_at<BUF>(obR, o + 2, N, m);
    kn[a] = s.k[0] * n0 + s.k[1] * n1 + s.k[2] * n2;
    un[a] = s.u[0] * n0 + s.u[1] * n1 + s.u[2] * n2;
    vn[a] = s.v[0] * n0 + s.v[1] * n1;
  }
  kn[2] = -(kn[0] + kn[1]);
  un[2] = -(un[0] + un[1]);
  vn[2] = -(vn[0] + vn[1]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fp[a] = un[a] * un[a] - vn[a] * vn[a];
    Fx[a] = (R)2 * un[a] * vn[a];
  }
  // k . dx_o / c for spacecraft 1, 2, 3
  R kp[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int o = OB_P1 + 3 * i;
    kp[i] = s.k[0] * ob_at<BUF>(obR, o + 0, N, m) + s.k[1] * ob_at<BUF>(obR, o + 1, N, m) +
            s.k[2] * ob_at<BUF>(obR, o + 2, N, m);
  }
  // e^{i pi f k.dx_i / c} per spacecraft; the offsets from the guiding centre sum to zero, so
  // the third factor is the conjugate of the product of the other two
  cplx<R> ph[3];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    R sc, cc;
    if (SHORT)
      sincos_rev_small((R)0.5 * fr * kp[i], &sc, &cc);
    else
      sincos_rev((R)0.5 * fr * kp[i], &sc, &cc);
    ph[i] = mk<R>(cc, sc);
  }
  ph[2] = conjg(ph[0] * ph[1]);
  // arm 12 -> opposite spacecraft 3, arm 23 -> 1, arm 31 -> 2
  const int opp[3] = {2, 0, 1};
  cplx<R> P[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cplx<R> b = mk<R>(s.ap.x * Fp[a] + s.ax.x * Fx[a], s.ap.y * Fp[a] + s.ax.y * Fx[a]);
    P[a] = b * ph[opp[a]];
  }
  // link sincs: n12 = +arm 12 for link 12, -arm 12 for link 21 (and cyclically)
  const R s12 = sinc_sel<R, SHORT>(x * ((R)1 - kn[0])), s21 = sinc_sel<R, SHORT>(x * ((R)1 + kn[0]));
  const R s23 = sinc_sel<R, SHORT>(x * ((R)1 - kn[1])), s32 = sinc_sel<R, SHORT>(x * ((R)1 + kn[1]));
  const R s31 = sinc_sel<R, SHORT>(x * ((R)1 - kn[2])), s13 = sinc_sel<R, SHORT>(x * ((R)1 + kn[2]));
  // G(a, b) = a + D b for real a, b
  auto G = [&](R a, R b) { return mk<R>(a + cD * b, sD * b); };
  const cplx<R> X = P[2] * G(s13, s31) - P[0] * G(s12, s21);
  const cplx<R> Y = P[0] * G(s21, s12) - P[1] * G(s23, s32);
  const cplx<R> Z = P[1] * G(s32, s23) - P[2] * G(s31, s13);
  // K = (1 - D^2) (-i x) e^{2 pi i p}, with 1 - D^2 = -2i sin(-2 pi f L/c) D (no cancellation
  // at low frequency)
  const cplx<R> omd = mk<R>((R)2 * sD * sD, -((R)2 * cD * sD));
  cplx<R> K = scal(mul_mi(omd * mk<R>(cp, sp)), x);
  // second generation: 1 - D^4 = 2i sin(4 pi f L/c) D^2 = -4i sD cD D^2 (no cancellation at low
  // frequency either)
  if (TDI2) K = K * mul_mi(scal(mk<R>(cD * cD - sD * sD, (R)2 * cD * sD), (R)4 * sD * cD));
  // the channels without their normalisations (chan_norm)
  out[0] = K * (Z - X);
  out[1] = K * (X - scal(Y, (R)2) + Z);
  if (C == 3) out[C - 1] = K * (X + Y + Z);
}

// 1 - w^2 for a unit phasor w = e^{-i theta}: 2i sin(theta) w with sin(theta) = -Im w (no
// cancellation when theta is small).
template <class R>
__device__ __forceinline__ cplx<R> one_minus_sq(cplx<R> w) { return mul_i(scal(w, (R)-2 * w.y)); }

// One sample of the slow series with one light time per arm (numerical orbits): the table's arm
// light times LT_a at the sample, all three arm vectors and the guiding centre's z.  For arm a
// (12, 23, 31 = index 0, 1, 2), x_a = pi f LT_a and E_a = e^{-i x_a}: its two links carry the
// amplitude x_a sinc(x_a (1 -+ k.n_a)) and the phase E_a (half the arm's travel time), and its
// delay is D_a = E_a^2.  With Dc = arm 12, Da = arm 23, Db = arm 31 (the link phasors frozen at
// the sample time)
//   X = (1 - Dc^2)(y13 + Db y31) - (1 - Db^2)(y12 + Dc y21),   Y, Z cyclically,
// and the second generation multiplies X by 1 - Db^2 Dc^2 (Y, Z likewise).  With equal arms
// this is slow_sample's form.  General sinc and sin/cos throughout (no short series).
template <class R, int C, bool TDI2>
__device__ __forceinline__ void slow_sample_uneq(const Cand<R>& s, const double* __restrict__ ob64,
                                                 const R* __restrict__ obR, int N, int m, double t,
                                                 cplx<R> out[C]) {
  constexpr bool BUF = sizeof(R) == 8;  // orbit reads through a buffer resource (ob_at)
  const double f = s.f0 + s.fd * t;
  const double kR = s.kxd * ob_at<BUF>(ob64, OB_RX, N, m) + s.kyd * ob_at<BUF>(ob64, OB_RY, N, m) +
                    s.kzd * ob_at<BUF>(ob64, OB_RZ, N, m);
  double p = s.df * t + 0.5 * s.fd * t * t + s.phi0c - f * kR;
  p -= rint(p);
  R sp, cp;
  sincos_rev((R)p, &sp, &cp);
  const R fr = (R)f;
  R kn[3], un[3], vn[3], Fp[3], Fx[3], xa[3];
  cplx<R> E[3], D[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int o = OB_N12 + 3 * a;
    const R n0 = ob_at<BUF>(obR, o + 0, N, m), n1 = ob_at<BUF>(obR, o + 1, N, m), n2 = ob_at<BUF>(obR, o + 2, N, m);
    kn[a] = s.k[0] * n0 + s.k[1] * n1 + s.k[2] * n2;
    un[a] = s.u[0] * n0 + s.u[1] * n1 + s.u[2] * n2;
    vn[a] = s.v[0] * n0 + s.v[1] * n1;
    Fp[a] = un[a] * un[a] - vn[a] * vn[a];
    Fx[a] = (R)2 * un[a] * vn[a];
    const R lt = ob_at<BUF>(obR, OB_LT12 + a, N, m);
    xa[a] = fr * (R)kPi * lt;
    R se, ce;
    sincos_rev((R)-0.5 * fr * lt, &se, &ce);  // E_a = e^{-i pi f LT_a}
    E[a] = mk<R>(ce, se);
    D[a] = E[a] * E[a];
  }
  R kp[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int o = OB_P1 + 3 * i;
    kp[i] = s.k[0] * ob_at<BUF>(obR, o + 0, N, m) + s.k[1] * ob_at<BUF>(obR, o + 1, N, m) +
            s.k[2] * ob_at<BUF>(obR, o + 2, N, m);
  }
  // e^{i pi f k.dx_i / c} per spacecraft (the offsets from the centroid sum to zero)
  cplx<R> ph[3];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    R sc, cc;
    sincos_rev((R)0.5 * fr * kp[i], &sc, &cc);
    ph[i] = mk<R>(cc, sc);
  }
  ph[2] = conjg(ph[0] * ph[1]);
  const int opp[3] = {2, 0, 1};  // arm 12 -> spacecraft 3, arm 23 -> 1, arm 31 -> 2
  cplx<R> P[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cplx<R> b = mk<R>(s.ap.x * Fp[a] + s.ax.x * Fx[a], s.ap.y * Fp[a] + s.ax.y * Fx[a]);
    P[a] = (b * ph[opp[a]]) * E[a];
  }
  // links: the "1 - k.n" link and the "1 + k.n" link of each arm
  const cplx<R> y12 = scal(P[0], xa[0] * sinc_r(xa[0] * ((R)1 - kn[0])));
  const cplx<R> y21 = scal(P[0], xa[0] * sinc_r(xa[0] * ((R)1 + kn[0])));
  const cplx<R> y23 = scal(P[1], xa[1] * sinc_r(xa[1] * ((R)1 - kn[1])));
  const cplx<R> y32 = scal(P[1], xa[1] * sinc_r(xa[1] * ((R)1 + kn[1])));
  const cplx<R> y31 = scal(P[2], xa[2] * sinc_r(xa[2] * ((R)1 - kn[2])));
  const cplx<R> y13 = scal(P[2], xa[2] * sinc_r(xa[2] * ((R)1 + kn[2])));
  const cplx<R> gc = one_minus_sq(D[0]), ga = one_minus_sq(D[1]), gb = one_minus_sq(D[2]);
  cplx<R> X = gc * (y13 + D[2] * y31) - gb * (y12 + D[0] * y21);
  cplx<R> Y = ga * (y21 + D[0] * y12) - gc * (y23 + D[1] * y32);
  cplx<R> Z = gb * (y32 + D[1] * y23) - ga * (y31 + D[2] * y13);
  if (TDI2) {
    X = one_minus_sq(D[2] * D[0]) * X;
    Y = one_minus_sq(D[0] * D[1]) * Y;
    Z = one_minus_sq(D[1] * D[2]) * Z;
  }
  const cplx<R> K = mul_mi(mk<R>(cp, sp));  // -i e^{2 pi i p}
  out[0] = K * (Z - X);
  out[1] = K * (X - scal(Y, (R)2) + Z);
  if (C == 3) out[C - 1] = K * (X + Y + Z);
}

// Synchronisation of the LPC lanes that share one template's LDS buffer.  A template wider
// than a wave needs the workgroup barrier.  Within one wave, LDS operations complete in issue
// order, so it is enough that the compiler moves no LDS access across the point (wave-scope
// release and acquire fences around a wave barrier); the workgroup's other waves, which work
// on other templates, are not held.
template <int LPC>
__device__ __forceinline__ void slot_sync() {
  if (LPC > 64) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ------------------------------------------------------------------------------------
// In-LDS Stockham FFT, radix 8, 4 and 2 (fft_lds picks the passes), register-staged in place:
// every pass reads all of a lane's elements, synchronises the template's lanes, butterflies,
// writes, synchronises.  buf: [C][N] complex of one template; LPC lanes per template, E = N/LPC
// elements per lane (E a multiple of the radix).  DIR = -1 forward (e^{-2 pi i jm/N}), +1
// inverse (unnormalised).  tw[m] = e^{-2 pi i m / N}.
template <class R, int N, int LPC, int C, int RADIX, int DIR>
__device__ __forceinline__ void stockham_pass(cplx<R>* buf, int lane, int Ns, const cplx<R>* __restrict__ tw) {
  constexpr int E = N / LPC;
  constexpr int NB = E / RADIX;
  cplx<R> v[C][NB][RADIX];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = lane + LPC * b;
#pragma unroll
      for (int r = 0; r < RADIX; ++r) v[c][b][r] = buf[c * N + j + r * (N / RADIX)];
    }
  slot_sync<LPC>();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = lane + LPC * b;
    const int k = j & (Ns - 1);
    const int step = k * (N / (Ns * RADIX));
    // the first pass (Ns = 1, a compile-time constant once fft_lds is unrolled) has every
    // twiddle equal to 1: no loads, no products
    const bool first = Ns == 1;
    cplx<R> w[RADIX];
    w[0] = mk<R>((R)1, (R)0);
#pragma unroll
    for (int r = 1; r < RADIX; ++r) {
      const cplx<R> t = first ? mk<R>((R)1, (R)0) : tw[r * step];
      w[r] = (DIR < 0) ? t : conjg(t);
    }
    const int base = (j - k) * RADIX + k;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      cplx<R> a[RADIX];
#pragma unroll
      for (int r = 0; r < RADIX; ++r) a[r] = (r == 0 || first) ? v[c][b][r] : v[c][b][r] * w[r];
      if (RADIX == 2) {
        buf[c * N + base] = a[0] + a[1];
        buf[c * N + base + Ns] = a[0] - a[1];
      } else if (RADIX == 4) {
        const cplx<R> s0 = a[0] + a[2], d0 = a[0] - a[2];
        const cplx<R> s1 = a[1] + a[3], d1 = a[1] - a[3];
        const cplx<R> rot = (DIR < 0) ? mul_mi(d1) : mul_i(d1);
        buf[c * N + base] = s0 + s1;
        buf[c * N + base + Ns] = d0 + rot;
        buf[c * N + base + 2 * Ns] = s0 - s1;
        buf[c * N + base + 3 * Ns] = d0 - rot;
      } else {
        // 8-point DFT: 4-point DFTs of the even and odd elements, combined with w8^q
        // (w8 = e^{DIR 2 pi i / 8}): X_q = E_q + w8^q O_q, X_{q+4} = E_q - w8^q O_q
        auto rot4 = [](cplx<R> z) { return (DIR < 0) ? mul_mi(z) : mul_i(z); };
        const cplx<R> e0 = a[0] + a[4], e1 = a[0] - a[4], e2 = a[2] + a[6], e3 = rot4(a[2] - a[6]);
        const cplx<R> o0 = a[1] + a[5], o1 = a[1] - a[5], o2 = a[3] + a[7], o3 = rot4(a[3] - a[7]);
        const cplx<R> E0 = e0 + e2, E1 = e1 + e3, E2 = e0 - e2, E3 = e1 - e3;
        const cplx<R> O0 = o0 + o2, O1 = o1 + o3, O2 = o0 - o2, O3 = o1 - o3;
        const R h = (R)0.70710678118654752440;
        const cplx<R> W1 = scal(O1 + rot4(O1), h);             // w8 O1 = (1 -+ i) O1 / sqrt2
        const cplx<R> W2 = rot4(O2);                             // w8^2 = -+ i
        const cplx<R> W3 = scal(rot4(O3) - O3, h);             // w8^3 = (-1 -+ i) / sqrt2
        buf[c * N + base] = E0 + O0;
        buf[c * N + base + Ns] = E1 + W1;
        buf[c * N + base + 2 * Ns] = E2 + W2;
        buf[c * N + base + 3 * Ns] = E3 + W3;
        buf[c * N + base + 4 * Ns] = E0 - O0;
        buf[c * N + base + 5 * Ns] = E1 - W1;
        buf[c * N + base + 6 * Ns] = E2 - W2;
        buf[c * N + base + 7 * Ns] = E3 - W3;
      }
    }
  }
  slot_sync<LPC>();
}

template <int N>
struct Log2 {
  static constexpr int v = 1 + Log2<N / 2>::v;
};
template <>
struct Log2<1> {
  static constexpr int v = 0;
};

// Passes: radix 8 as often as it fits when a lane holds 8 elements (fewer LDS round trips and
// twiddle products per element), then radix 4, and one radix-2 pass when an odd power of two
// remains.  The mixed-radix Stockham indexing takes the radices in any order.
template <class R, int N, int LPC, int C, int DIR>
__device__ __forceinline__ void fft_lds(cplx<R>* buf, int lane, const cplx<R>* __restrict__ tw) {
  constexpr int LG = Log2<N>::v;
  constexpr int N8 = (N / LPC) % 8 == 0 ? LG / 3 : 0;   // radix-8 passes
  constexpr int REM = LG - 3 * N8;                     // log2 N left for radix 4 and 2
  int Ns = 1;
  if (REM & 1) {
    stockham_pass<R, N, LPC, C, 2, DIR>(buf, lane, 1, tw);
    Ns = 2;
  }
#pragma unroll
  for (int p = 0; p < REM / 2; ++p) {
    stockham_pass<R, N, LPC, C, 4, DIR>(buf, lane, Ns, tw);
    Ns *= 4;
  }
#pragma unroll
  for (int p = 0; p < N8; ++p) {
    stockham_pass<R, N, LPC, C, 8, DIR>(buf, lane, Ns, tw);
    Ns *= 8;
  }
}

}  // namespace gbx

namespace gbx {

// ------------------------------------------------------------------------------------
// Gradient support.

// sinc(u) and its derivative
__device__ __forceinline__ void sinc_d(double u, double* s, double* ds) {
  if (fabs(u) <= 2.0) {
    const double u2 = u * u;
    // coefficients (-1)^k / (2k+1)!, k = 0..11
    const double c[12] = {1.0, -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0, -1.0 / 39916800.0,
                          1.0 / 6227020800.0, -1.0 / 1307674368000.0, 1.0 / 355687428096000.0,
                          -1.0 / 121645100408832000.0, 1.0 / 51090942171709440000.0,
                          -1.0 / 25852016738884976640000.0};
    double p = c[11], q = 22.0 * c[11];
#pragma unroll
    for (int k = 10; k >= 1; --k) {
      p = p * u2 + c[k];
      q = q * u2 + 2.0 * k * c[k];
    }
    *s = p * u2 + c[0];
    *ds = q * u;
  } else {
    double sn, cs;
    sincos_rev(u * (0.5 / kPi), &sn, &cs);
    *s = sn / u;
    *ds = (cs - *s) / u;
  }
}
__device__ __forceinline__ void sinc_d(float u, float* s, float* ds) {
  if (fabsf(u) <= 2.0f) {
    const float u2 = u * u;
    const float c[8] = {1.0f, -1.0f / 6.0f, 1.0f / 120.0f, -1.0f / 5040.0f, 1.0f / 362880.0f,
                        -1.0f / 39916800.0f, 1.0f / 6227020800.0f, -1.0f / 1307674368000.0f};
    float p = c[7], q = 14.0f * c[7];
#pragma unroll
    for (int k = 6; k >= 1; --k) {
      p = p * u2 + c[k];
      q = q * u2 + 2.0f * k * c[k];
    }
    *s = p * u2 + c[0];
    *ds = q * u;
  } else {
    const float sn = __builtin_amdgcn_sinf(u * (float)(0.5 / kPi));
    const float cs = __builtin_amdgcn_cosf(u * (float)(0.5 / kPi));
    *s = sn / u;
    *ds = (cs - *s) / u;
  }
}
// sinc and its derivative by the short series (see sinc_short)
__device__ __forceinline__ void sinc_d_short(double u, double* s, double* ds) {
  const double u2 = u * u;
  const double c[10] = {1.0, -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0, -1.0 / 39916800.0,
                        1.0 / 6227020800.0, -1.0 / 1307674368000.0, 1.0 / 355687428096000.0,
                        -1.0 / 121645100408832000.0};
  double p = c[9], q = 18.0 * c[9];
#pragma unroll
  for (int k = 8; k >= 1; --k) {
    p = p * u2 + c[k];
    q = q * u2 + 2.0 * k * c[k];
  }
  *s = p * u2 + c[0];
  *ds = q * u;
}
__device__ __forceinline__ void sinc_d_short(float u, float* s, float* ds) {
  const float u2 = u * u;
  const float c[5] = {1.0f, -1.0f / 6.0f, 1.0f / 120.0f, -1.0f / 5040.0f, 1.0f / 362880.0f};
  float p = c[4], q = 8.0f * c[4];
#pragma unroll
  for (int k = 3; k >= 1; --k) {
    p = p * u2 + c[k];
    q = q * u2 + 2.0f * k * c[k];
  }
  *s = p * u2 + c[0];
  *ds = q * u;
}
template <class R, bool SHORT>
__device__ __forceinline__ void sinc_d_sel(R u, R* s, R* ds) {
  if (SHORT)
    sinc_d_short(u, s, ds);
  else
    sinc_d(u, s, ds);
}

// Extra per-candidate constants of the gradient.
template <class R>
struct CandG {
  R sb, cb;           // sin beta, cos beta
  R wl[2];            // d v / d lambda = (cos lambda, sin lambda, 0)
};
template <class R>
__device__ __forceinline__ CandG<R> make_cand_grad(const double* th, bool ok) {
  CandG<R> g;
  double sb, cb, sl, cl;
  sincos_rad(ok ? th[2] : 0.0, &sb, &cb);
  sincos_rad(ok ? th[3] : 0.0, &sl, &cl);
  g.sb = (R)sb;
  g.cb = (R)cb;
  g.wl[0] = (R)cl;
  g.wl[1] = (R)sl;
  return g;
}

// Per-sample accumulators of the gradient (FP64; laid out as ten consecutive doubles).
struct GradAcc {
  double gf, gtf, gb, gl;   // sum Re(cot . dS/d{f, beta, lambda}); gtf = sum t * (f part)
  double gu_re, gu_im, gv_re, gv_im;  // sum conj(Sbar) U, conj(Sbar) V
  double pt, ptt;           // sum t Im(conj(Sbar) S), sum t^2 Im(conj(Sbar) S)
};

}  // namespace gbx

namespace gbx {

// ------------------------------------------------------------------------------------
// Contribution of slow-series sample m to the gradient, by hand-written reverse mode.
// With the channel cotangents folded onto X, Y, Z (bX, bY, bZ) and the links onto one
// cotangent per arm (Lam_a), the sample's share of sum_c conj(sbar_c) S_c is J = K Q with
//   Q = sum_a Lam_a P_a,   P_a = (ap F+_a + ax Fx_a) E_a,   E_a = e^{i chi_a},
//   K = (1 - D^2)(-i x) e^{2 pi i p} = kappa e^{i psi},  kappa = phi_D sin(phi_D),
//   psi = 2 pi p - phi_D,  phi_D = 2 pi f L/c,  x = phi_D / 2.
// Its derivative along f (local frequency), beta, lambda collects: the amplitude kappa and
// the phase psi of K, the arm phases chi_a, the projections F+_a, Fx_a, the six link sincs
// through u = x (1 -+ k.n_a), and the delay D inside Lam_a.
template <class R, int C, bool TDI2, bool SHORT>
__device__ __forceinline__ void grad_sample_rev(const Cand<R>& s, const CandG<R>& sg,
                                                const double* __restrict__ ob64, const R* __restrict__ obR,
                                                int N, int m, double t, double Lc, const cplx<R> sbar[C],
                                                GradAcc& acc) {
  const R twopi = (R)(2.0 * kPi), pi = (R)kPi;
  constexpr bool BUF = sizeof(R) == 8;  // orbit reads through a buffer resource (ob_at)
  const double f = s.f0 + s.fd * t;
  const double Rx = ob_at<BUF>(ob64, OB_RX, N, m), Ry = ob_at<BUF>(ob64, OB_RY, N, m);
  const double kR = s.kxd * Rx + s.kyd * Ry;
  double p = s.df * t + 0.5 * s.fd * t * t + s.phi0c - f * (0.5 * Lc + kR);
  p -= rint(p);
  const R fr = (R)f, Lr = (R)Lc;
  R sp, cp, sDm, cDm;
  sincos_rev((R)p, &sp, &cp);
  // D = e^{-i phi_D}: (cDm, sDm), sDm = -sin(phi_D); beyond the short series' range the argument
  // is reduced in FP64 (the TDI factors' nulls)
  if constexpr (SHORT)
    sincos_rev(-fr * Lr, &sDm, &cDm);
  else
    sincos_rev_red(-f * Lc, &sDm, &cDm);
  const cplx<R> D = mk<R>(cDm, sDm);
  const R phiD = fr * (R)(2.0 * kPi * Lc);
  const R x = fr * (R)(kPi * Lc);
  R kappa = -(R)2 * x * sDm;                           // = phi_D sin(phi_D)
  cplx<R> Ep = D * mk<R>(cp, sp);                       // e^{i psi}
  // amplitude and phase of K along f (below): d kappa/df and d psi/df
  R dkappa_f = twopi * Lr * (-sDm + phiD * cDm);        // d(phi_D sin phi_D)/df
  R dpsi_f = -twopi * ((R)1.5 * Lr + (R)kR);
  if (TDI2) {
    // second generation: K2 = K (1 - D^4) = K 2 sin(2 phi_D) i D^2, so kappa gains the factor
    // g = 2 sin(2 phi_D) = -4 sDm cDm and psi the phase pi/2 - 2 phi_D
    const R g = -(R)4 * sDm * cDm;
    const R dg = (R)4 * (cDm * cDm - sDm * sDm) * twopi * Lr;   // 4 cos(2 phi_D) d phi_D/df
    dkappa_f = dkappa_f * g + kappa * dg;
    kappa = kappa * g;
    Ep = mul_i(Ep * (D * D));
    dpsi_f = dpsi_f - (R)2 * twopi * Lr;
  }
  const cplx<R> K = scal(Ep, kappa);
  const R uR = s.u[0] * (R)Rx + s.u[1] * (R)Ry;
  const R vR = s.v[0] * (R)Rx + s.v[1] * (R)Ry;

  // arms: projections, phases
  R kn[3], un[3], vn[3], wn[3], Fp[3], Fx[3], kp[3], up[3], vp[3];
  cplx<R> E[3], P[3];
  const int opp[3] = {2, 0, 1};
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int o = OB_N12 + 3 * a;
    const R n0 = ob_at<BUF>(obR, o + 0, N, m), n1 = ob_at<BUF>(obR, o + 1, N, m), n2 = ob_at<BUF>(obR, o + 2, N, m);
    kn[a] = s.k[0] * n0 + s.k[1] * n1 + s.k[2] * n2;
    un[a] = s.u[0] * n0 + s.u[1] * n1 + s.u[2] * n2;
    vn[a] = s.v[0] * n0 + s.v[1] * n1;
    wn[a] = sg.wl[0] * n0 + sg.wl[1] * n1;
  }
  // the arm vectors of the rigid triangle sum to zero (as in the forward series)
  kn[2] = -(kn[0] + kn[1]);
  un[2] = -(un[0] + un[1]);
  vn[2] = -(vn[0] + vn[1]);
  wn[2] = -(wn[0] + wn[1]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fp[a] = un[a] * un[a] - vn[a] * vn[a];
    Fx[a] = (R)2 * un[a] * vn[a];
    if (a == 0) continue;  // spacecraft 3 (arm 12) below
    const int q = OB_P1 + 3 * opp[a];
    const R p0 = ob_at<BUF>(obR, q + 0, N, m), p1 = ob_at<BUF>(obR, q + 1, N, m), p2 = ob_at<BUF>(obR, q + 2, N, m);
    kp[a] = s.k[0] * p0 + s.k[1] * p1 + s.k[2] * p2;
    up[a] = s.u[0] * p0 + s.u[1] * p1 + s.u[2] * p2;
    vp[a] = s.v[0] * p0 + s.v[1] * p1;
  }
  // the offsets from the guiding centre sum to zero: spacecraft 3's projections are minus the
  // sum of those of spacecraft 1 and 2 (as its phase factor is in the forward series)
  kp[0] = -(kp[1] + kp[2]);
  up[0] = -(up[1] + up[2]);
  vp[0] = -(vp[1] + vp[2]);
  // spacecraft phase factors e^{i pi f k.dx / c}: arms 23 and 31 face spacecraft 1 and 2; the
  // offsets sum to zero, so the factor of spacecraft 3 (arm 12) is the conjugate of their product
#pragma unroll
  for (int a = 1; a < 3; ++a) {
    R sc, cc;
    sincos_rev((R)0.5 * fr * kp[a], &sc, &cc);
    E[a] = mk<R>(cc, sc);
  }
  E[0] = conjg(E[1] * E[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
    P[a] = mk<R>(s.ap.x * Fp[a] + s.ax.x * Fx[a], s.ap.y * Fp[a] + s.ax.y * Fx[a]) * E[a];
  // links: index 2a is the "1 - k.n_a" link, 2a+1 the "1 + k.n_a" link of arm a
  // (arm 12: links 12, 21; arm 23: 23, 32; arm 31: 31, 13)
  R sv[6], sd[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sinc_d_sel<R, SHORT>(x * ((R)1 - kn[a]), &sv[2 * a], &sd[2 * a]);
    sinc_d_sel<R, SHORT>(x * ((R)1 + kn[a]), &sv[2 * a + 1], &sd[2 * a + 1]);
  }
  const R s12 = sv[0], s21 = sv[1], s23 = sv[2], s32 = sv[3], s31 = sv[4], s13 = sv[5];
  // channel cotangents (of the series without their normalisations) folded onto X, Y, Z
  const cplx<R> cA = conjg(sbar[0]), cE = conjg(sbar[1]);
  const cplx<R> cT = (C == 3) ? conjg(sbar[C - 1]) : mk<R>((R)0, (R)0);
  const cplx<R> bX = cE + cT - cA;
  const cplx<R> bY = cT - scal(cE, (R)2);
  const cplx<R> bZ = cA + cE + cT;
  auto G = [&](R a, R b) { return mk<R>(a + cDm * b, sDm * b); };  // a + D b
  cplx<R> Lam[3];
  Lam[0] = bY * G(s21, s12) - bX * G(s12, s21);
  Lam[1] = bZ * G(s32, s23) - bY * G(s23, s32);
  Lam[2] = bX * G(s13, s31) - bZ * G(s31, s13);
  // GU = K sum_a F+_a Lam_a E_a and GV = K sum_a Fx_a Lam_a E_a from the per-arm K Lam_a E_a
  cplx<R> Q = mk<R>((R)0, (R)0), GU = Q, GV = Q;
  cplx<R> KLP[3], KLE[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Q = Q + Lam[a] * P[a];
    KLE[a] = K * (Lam[a] * E[a]);
    GU = GU + scal(KLE[a], Fp[a]);
    GV = GV + scal(KLE[a], Fx[a]);
    KLP[a] = K * (Lam[a] * P[a]);
  }
  const cplx<R> J = K * Q;

  // amplitude and phase of K
  const R EQre = (Ep * Q).x;
  const R dpsi_b = -twopi * fr * uR;
  const R dpsi_l = -twopi * fr * sg.cb * vR;
  R gf = EQre * dkappa_f - J.y * dpsi_f;
  R gb = -J.y * dpsi_b;
  R gl = -J.y * dpsi_l;
  // arm phases chi_a = pi f k.p_a and projections F+_a, Fx_a.  With rp = Re(K Lam_a E_a ap),
  // rx = Re(K Lam_a E_a ax) and t1 = rp u.n + rx v.n, t2 = rp v.n - rx u.n:
  //   beta:   rp dF+/dbeta + rx dFx/dbeta = -2 k.n t1,
  //   lambda: rp dF+/dlambda + rx dFx/dlambda = -2 sin(beta) v.n t1 - 2 w.n t2;
  // the per-arm terms are summed first and the candidate constants applied once
  R hk = (R)0, hu = (R)0, hv = (R)0, bk = (R)0, lv = (R)0, lw = (R)0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R im = KLP[a].y;
    hk += im * kp[a];
    hu += im * up[a];
    hv += im * vp[a];
    const R rp = KLE[a].x * s.ap.x - KLE[a].y * s.ap.y;
    const R rx = KLE[a].x * s.ax.x - KLE[a].y * s.ax.y;
    const R t1 = rp * un[a] + rx * vn[a];
    const R t2 = rp * vn[a] - rx * un[a];
    bk += kn[a] * t1;
    lv += vn[a] * t1;
    lw += wn[a] * t2;
  }
  gf -= pi * hk;
  gb -= (pi * fr) * hu + (R)2 * bk;
  gl -= (pi * fr) * sg.cb * hv + (R)2 * (sg.sb * lv + lw);
  // link sincs: the coefficient of s_rs in K Q is e_rs (K P_arm).  With r-, r+ the weights of
  // the arm's links u = x (1 - k.n) and u = x (1 + k.n), their share is
  //   f: pi L/c [(r- + r+) + k.n (r+ - r-)],  beta: x u.n (r+ - r-),  lambda: x cos(beta) v.n (r+ - r-)
  cplx<R> KP[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) KP[a] = K * P[a];
  const cplx<R> bXD = bX * D, bYD = bY * D, bZD = bZ * D;
  const cplx<R> el[6] = {bYD - bX, bY - bXD, bZD - bY, bZ - bYD, bXD - bZ, bX - bZD};
  R ls = (R)0, lk = (R)0, lu = (R)0, lvn = (R)0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R rm = (el[2 * a] * KP[a]).x * sd[2 * a];
    const R rq = (el[2 * a + 1] * KP[a]).x * sd[2 * a + 1];
    const R dr = rq - rm;
    ls += rq + rm;
    lk += kn[a] * dr;
    lu += un[a] * dr;
    lvn += vn[a] * dr;
  }
  gf += (pi * Lr) * (ls + lk);
  gb += x * lu;
  gl += (x * sg.cb) * lvn;
  // the delay inside Lam: d(KQ)/dD = sum_a (dLam_a/dD) K P_a, dD/df = -2 pi i (L/c) D
  const cplx<R> KcD = (scal(bY, s12) - scal(bX, s21)) * KP[0] + (scal(bZ, s23) - scal(bY, s32)) * KP[1] +
                      (scal(bX, s31) - scal(bZ, s13)) * KP[2];
  gf += twopi * Lr * (KcD * D).y;

  const double gfd = (double)gf;
  acc.gf += gfd;
  acc.gtf += t * gfd;
  acc.gb += (double)gb;
  acc.gl += (double)gl;
  acc.gu_re += (double)GU.x;
  acc.gu_im += (double)GU.y;
  acc.gv_re += (double)GV.x;
  acc.gv_im += (double)GV.y;
  acc.pt += t * (double)J.y;
  acc.ptt += t * t * (double)J.y;
}

// Contribution of slow-series sample m to the gradient on numerical orbits (one light time per
// arm, the model of slow_sample_uneq), by hand-written reverse mode.  Every link term is
// y_l = x_a sinc(x_a (1 -+ k.n_a)) b_a ph_o E_a (b_a = ap F+_a + ax Fx_a, ph_o the phase of the
// spacecraft opposite the arm, E_a = e^{-i x_a}).  The channel cotangents, folded onto X, Y, Z
// and multiplied by K' = -i e^{2 pi i p} (and by the second-generation factors 1 - (D_i D_j)^2
// when they apply), give one complex coefficient k_l per link, so that the sample's share of
// sum_c conj(sbar_c) S_c is J = sum_l k_l y_l.  Its derivatives along the local frequency f,
// beta and lambda then need only the per-link derivatives of y_l (amplitude, projections,
// phases of ph_o E_a) contracted with k_l, plus, along f, the partial derivatives of J in the
// delays D_a = E_a^2 (in the coefficients 1 - D_a^2, the explicit delays and the
// second-generation factors) times dD_a/df = -2 pi i LT_a D_a, and the phase of K' (through
// f k.R, with dk/dbeta = u and dk/dlambda = cos(beta) v).  GU and GV are J with b_a replaced by
// F+_a and Fx_a.
template <class R, int C, bool TDI2>
__device__ __forceinline__ void grad_sample_uneq(const Cand<R>& s, const CandG<R>& sg,
                                                 const double* __restrict__ ob64, const R* __restrict__ obR,
                                                 int N, int m, double t, const cplx<R> sbar[C], GradAcc& acc) {
  constexpr bool BUF = sizeof(R) == 8;  // orbit reads through a buffer resource (ob_at)
  const R pi = (R)kPi, twopi = (R)(2.0 * kPi);
  const double f = s.f0 + s.fd * t;
  const double Rx = ob_at<BUF>(ob64, OB_RX, N, m), Ry = ob_at<BUF>(ob64, OB_RY, N, m);
  const double Rz = ob_at<BUF>(ob64, OB_RZ, N, m);
  const double kR = s.kxd * Rx + s.kyd * Ry + s.kzd * Rz;
  double p = s.df * t + 0.5 * s.fd * t * t + s.phi0c - f * kR;
  p -= rint(p);
  R sp, cp;
  sincos_rev((R)p, &sp, &cp);
  const cplx<R> Kp = mul_mi(mk<R>(cp, sp));  // K' = -i e^{2 pi i p}
  const R fr = (R)f;
  const R uR = s.u[0] * (R)Rx + s.u[1] * (R)Ry + s.u[2] * (R)Rz;  // dk/dbeta . R
  const R vR = s.v[0] * (R)Rx + s.v[1] * (R)Ry;                  // dk/dlambda . R / cos(beta)

  // arms 12, 23, 31 (index 0, 1, 2)
  R kn[3], un[3], vn[3], wn[3], Fp[3], Fx[3], xa[3], lt[3];
  cplx<R> E[3], D[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int o = OB_N12 + 3 * a;
    const R n0 = ob_at<BUF>(obR, o + 0, N, m), n1 = ob_at<BUF>(obR, o + 1, N, m), n2 = ob_at<BUF>(obR, o + 2, N, m);
    kn[a] = s.k[0] * n0 + s.k[1] * n1 + s.k[2] * n2;
    un[a] = s.u[0] * n0 + s.u[1] * n1 + s.u[2] * n2;
    vn[a] = s.v[0] * n0 + s.v[1] * n1;
    wn[a] = sg.wl[0] * n0 + sg.wl[1] * n1;
    Fp[a] = un[a] * un[a] - vn[a] * vn[a];
    Fx[a] = (R)2 * un[a] * vn[a];
    lt[a] = ob_at<BUF>(obR, OB_LT12 + a, N, m);
    xa[a] = fr * pi * lt[a];
    R se, ce;
    sincos_rev((R)-0.5 * fr * lt[a], &se, &ce);
    E[a] = mk<R>(ce, se);
    D[a] = E[a] * E[a];
  }
  // spacecraft 1, 2 (offsets from the centroid; spacecraft 3 is minus their sum)
  R kp[3], up[3], vp[3];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int o = OB_P1 + 3 * i;
    const R p0 = ob_at<BUF>(obR, o + 0, N, m), p1 = ob_at<BUF>(obR, o + 1, N, m), p2 = ob_at<BUF>(obR, o + 2, N, m);
    kp[i] = s.k[0] * p0 + s.k[1] * p1 + s.k[2] * p2;
    up[i] = s.u[0] * p0 + s.u[1] * p1 + s.u[2] * p2;
    vp[i] = s.v[0] * p0 + s.v[1] * p1;
  }
  kp[2] = -(kp[0] + kp[1]);
  up[2] = -(up[0] + up[1]);
  vp[2] = -(vp[0] + vp[1]);
  cplx<R> ph[3];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    R sc, cc;
    sincos_rev((R)0.5 * fr * kp[i], &sc, &cc);
    ph[i] = mk<R>(cc, sc);
  }
  ph[2] = conjg(ph[0] * ph[1]);
  const int opp[3] = {2, 0, 1};  // arm 12 -> spacecraft 3, arm 23 -> 1, arm 31 -> 2

  // channel cotangents folded onto X, Y, Z, times K'; second generation: X2 = (1 - W_X^2) X with
  // W_X = D2 D0, W_Y = D0 D1, W_Z = D1 D2
  const cplx<R> cA = conjg(sbar[0]), cE = conjg(sbar[1]);
  const cplx<R> cT = (C == 3) ? conjg(sbar[C - 1]) : mk<R>((R)0, (R)0);
  const cplx<R> b3[3] = {Kp * (cE + cT - cA), Kp * (cT - scal(cE, (R)2)), Kp * (cA + cE + cT)};
  cplx<R> W[3], bf[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) bf[i] = b3[i];
  if (TDI2) {
    W[0] = D[2] * D[0];
    W[1] = D[0] * D[1];
    W[2] = D[1] * D[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) bf[i] = b3[i] * one_minus_sq(W[i]);
  }
  // link coefficients from X = g0 (y13 + D2 y31) - g2 (y12 + D0 y21) and cyclically
  // (g_a = 1 - D_a^2; links 12, 21, 23, 32, 31, 13 at index 0..5)
  const cplx<R> g[3] = {one_minus_sq(D[0]), one_minus_sq(D[1]), one_minus_sq(D[2])};
  const cplx<R> A0 = bf[0] * g[0], A2 = bf[0] * g[2], B0 = bf[1] * g[0];
  const cplx<R> B1 = bf[1] * g[1], C1 = bf[2] * g[1], C2 = bf[2] * g[2];
  const cplx<R> k[6] = {B1 * D[0] - A2, B1 - A2 * D[0], C2 * D[1] - B0,
                        C2 - B0 * D[1], A0 * D[2] - C1, A0 - C1 * D[2]};

  // per arm: kap = sum over its two links of k_l x_a sinc (J's share is kap P_a), and the
  // same sums with the derivatives of x_a sinc along f, beta, lambda
  R gf = (R)0, gb = (R)0, gl = (R)0, Jy = (R)0;
  cplx<R> GU = mk<R>((R)0, (R)0), GV = GU;
  cplx<R> y[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int o = opp[a];
    const cplx<R> pe = ph[o] * E[a];
    const cplx<R> b = mk<R>(s.ap.x * Fp[a] + s.ax.x * Fx[a], s.ap.y * Fp[a] + s.ax.y * Fx[a]);
    const R dFpb = (R)-2 * kn[a] * un[a], dFxb = (R)-2 * kn[a] * vn[a];
    const R dFpl = (R)-2 * (sg.sb * un[a] * vn[a] + vn[a] * wn[a]);
    const R dFxl = (R)2 * (un[a] * wn[a] - sg.sb * vn[a] * vn[a]);
    const cplx<R> bb = mk<R>(s.ap.x * dFpb + s.ax.x * dFxb, s.ap.y * dFpb + s.ax.y * dFxb);
    const cplx<R> bl = mk<R>(s.ap.x * dFpl + s.ax.x * dFxl, s.ap.y * dFpl + s.ax.y * dFxl);
    const cplx<R> P = b * pe;
    // phase rates of ph_o E_a along f, beta, lambda
    const R wf = pi * (kp[o] - lt[a]), wb = pi * fr * up[o], wl = pi * fr * sg.cb * vp[o];
    cplx<R> kap = mk<R>((R)0, (R)0), phf = kap, phb = kap, phl = kap;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const R sgn = q == 0 ? (R)1 : (R)-1;  // u = x (1 - sgn k.n)
      const R arg = xa[a] * ((R)1 - sgn * kn[a]);
      R sv, sd;
      sinc_d(arg, &sv, &sd);
      const int l = 2 * a + q;
      const R amp = xa[a] * sv;
      y[l] = scal(P, amp);
      // f: d(x_a sinc)/df = pi LT (sinc + x_a sinc' (1 - sgn k.n)); beta: the sinc argument
      // moves by -sgn x_a u.n; lambda: by -sgn x_a cos(beta) v.n
      const R damp_f = pi * lt[a] * (sv + xa[a] * sd * ((R)1 - sgn * kn[a]));
      const R damp_b = xa[a] * sd * (-sgn * xa[a] * un[a]);
      const R damp_l = xa[a] * sd * (-sgn * xa[a] * sg.cb * vn[a]);
      kap = kap + scal(k[l], amp);
      phf = phf + scal(k[l], damp_f);
      phb = phb + scal(k[l], damp_b);
      phl = phl + scal(k[l], damp_l);
    }
    const cplx<R> kP = kap * P, kpe = kap * pe;
    // Re(i w z) = -w Im(z) for the phase rates
    Jy += kP.y;
    gf += (P * phf).x - wf * kP.y;
    gb += (P * phb).x + (kpe * bb).x - wb * kP.y;
    gl += (P * phl).x + (kpe * bl).x - wl * kP.y;
    GU = GU + scal(kpe, Fp[a]);
    GV = GV + scal(kpe, Fx[a]);
  }
  // along f through the delays: dJ[a] = dJ/dD_a with the link terms held
  const cplx<R> SX0 = y[5] + D[2] * y[4], SX2 = y[0] + D[0] * y[1];
  const cplx<R> SY1 = y[1] + D[0] * y[0], SY0 = y[2] + D[1] * y[3];
  const cplx<R> SZ2 = y[3] + D[1] * y[2], SZ1 = y[4] + D[2] * y[5];
  cplx<R> dJ[3];
  dJ[0] = bf[0] * (scal(D[0] * SX0, (R)-2) - g[2] * y[1]) + bf[1] * (g[1] * y[0] + scal(D[0] * SY0, (R)2));
  dJ[1] = bf[1] * (scal(D[1] * SY1, (R)-2) - g[0] * y[3]) + bf[2] * (g[2] * y[2] + scal(D[1] * SZ1, (R)2));
  dJ[2] = bf[2] * (scal(D[2] * SZ2, (R)-2) - g[1] * y[5]) + bf[0] * (g[0] * y[4] + scal(D[2] * SX2, (R)2));
  if (TDI2) {
    // d(1 - W^2)/dD_a = -2 W dW/dD_a
    const cplx<R> X = g[0] * SX0 - g[2] * SX2, Y = g[1] * SY1 - g[0] * SY0, Z = g[2] * SZ2 - g[1] * SZ1;
    const cplx<R> hX = scal(W[0] * (b3[0] * X), (R)-2), hY = scal(W[1] * (b3[1] * Y), (R)-2);
    const cplx<R> hZ = scal(W[2] * (b3[2] * Z), (R)-2);
    dJ[0] = dJ[0] + hX * D[2] + hY * D[1];
    dJ[1] = dJ[1] + hY * D[0] + hZ * D[2];
    dJ[2] = dJ[2] + hX * D[0] + hZ * D[1];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) gf += (dJ[a] * mul_mi(scal(D[a], twopi * lt[a]))).x;  // dD/df = -2 pi i LT D
  // the phase of K' moves by -2 pi f k.R: along f by -2 pi k.R, beta -2 pi f u.R, lambda
  // -2 pi f cos(beta) v.R
  gf += Jy * (twopi * (R)kR);
  gb += Jy * (twopi * fr * uR);
  gl += Jy * (twopi * fr * sg.cb * vR);
  const double gfd = (double)gf;
  acc.gf += gfd;
  acc.gtf += t * gfd;
  acc.gb += (double)gb;
  acc.gl += (double)gl;
  acc.gu_re += (double)GU.x;
  acc.gu_im += (double)GU.y;
  acc.gv_re += (double)GV.x;
  acc.gv_im += (double)GV.y;
  acc.pt += t * (double)Jy;
  acc.ptt += t * t * (double)Jy;
}

}  // namespace gbx
