// CPU oracle for the batched Galactic-binary log-likelihood -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, scalar FP64.  Only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark load this library; the product path never does.  It shares no
// code with the HIP library.
//
// What it computes (paper: Strub et al., arXiv:2307.03763):
//  * logL = -1/2 <d - s | d - s>                       (Sec. II, log-likelihood equation)
//  * <x|y> = 4 Re int x y* / S df, summed over channels (Sec. II, scalar-product and
//    channel-sum equations), discretised on the bins of the padded frequency window
//    (Sec. III D restricts the integral to that segment): sum_k w_k Re(x_k y_k*), w = 4/(T S)
//  * channels A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3 (Sec. II)
//  * the eight parameters (A, lambda, beta, f, fdot, iota, phi0, psi) of Sec. III.
// The paper names the parameters but defers the signal model to the literature, so the
// model below is this project's reading: a plane wave with + and x polarisations,
// a rigid equal-arm triangle on the classic first-order heliocentric orbit, the
// single-link response for light travel L/c, first- or second-generation equal-arm
// Michelson TDI, and the fast/slow evaluation (slow series on N samples, N-point DFT, heterodyne by the
// carrier bin q = floor(f0 T)).  Every convention is listed in the design notes.
//
// Gradients: every step is written once over a scalar type R; R = double gives values,
// R = Dual (eight tangent directions) gives the exact derivative of the same numbers.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

const double kPi = 3.14159265358979323846;
const double kC = 299792458.0;  // m/s

// ------------------------------------------------------------------ dual numbers
struct Dual {
  double v;
  double d[8];
  Dual() : v(0.0), d{} {}
  Dual(double x) : v(x), d{} {}  // a constant: zero tangents
};

inline Dual mk(double v) { return Dual(v); }
inline Dual operator+(const Dual& a, const Dual& b) {
  Dual r;
  r.v = a.v + b.v;
  for (int i = 0; i < 8; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
inline Dual operator-(const Dual& a, const Dual& b) {
  Dual r;
  r.v = a.v - b.v;
  for (int i = 0; i < 8; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
inline Dual operator-(const Dual& a) {
  Dual r;
  r.v = -a.v;
  for (int i = 0; i < 8; ++i) r.d[i] = -a.d[i];
  return r;
}
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r;
  r.v = a.v * b.v;
  for (int i = 0; i < 8; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r;
  r.v = a.v / b.v;
  for (int i = 0; i < 8; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + mk(b); }
inline Dual operator+(double a, const Dual& b) { return mk(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - mk(b); }
inline Dual operator-(double a, const Dual& b) { return mk(a) - b; }
inline Dual operator*(const Dual& a, double b) {
  Dual r;
  r.v = a.v * b;
  for (int i = 0; i < 8; ++i) r.d[i] = a.d[i] * b;
  return r;
}
inline Dual operator*(double a, const Dual& b) { return b * a; }
inline Dual operator/(const Dual& a, double b) { return a * (1.0 / b); }
inline Dual sin(const Dual& a) {
  Dual r;
  r.v = std::sin(a.v);
  double c = std::cos(a.v);
  for (int i = 0; i < 8; ++i) r.d[i] = c * a.d[i];
  return r;
}
inline Dual cos(const Dual& a) {
  Dual r;
  r.v = std::cos(a.v);
  double s = -std::sin(a.v);
  for (int i = 0; i < 8; ++i) r.d[i] = s * a.d[i];
  return r;
}
inline double value(double x) { return x; }
inline double value(const Dual& x) { return x.v; }
inline Dual seed(double v, int dir) {
  Dual r = mk(v);
  r.d[dir] = 1.0;
  return r;
}

using std::cos;
using std::sin;

// ------------------------------------------------------------------ complex numbers
template <class R>
struct Cx {
  R re, im;
};
template <class R>
Cx<R> cx(R re, R im) {
  Cx<R> z;
  z.re = re;
  z.im = im;
  return z;
}
template <class R>
Cx<R> operator+(const Cx<R>& a, const Cx<R>& b) { return cx<R>(a.re + b.re, a.im + b.im); }
template <class R>
Cx<R> operator-(const Cx<R>& a, const Cx<R>& b) { return cx<R>(a.re - b.re, a.im - b.im); }
template <class R>
Cx<R> operator*(const Cx<R>& a, const Cx<R>& b) {
  return cx<R>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class R>
Cx<R> scale(const Cx<R>& a, const R& s) { return cx<R>(a.re * s, a.im * s); }
template <class R>
Cx<R> scaled(const Cx<R>& a, double s) { return cx<R>(a.re * s, a.im * s); }
template <class R>
Cx<R> expi(const R& ph) { return cx<R>(cos(ph), sin(ph)); }

// ------------------------------------------------------------------ geometry
struct Params {
  double T;       // observation time, s
  double P_orb;   // orbital period of the guiding centre, s
  double L;       // arm length, m
  double AU;      // orbital radius, m
  int tdi;        // TDI generation, 1 or 2
};

struct V3 {
  double x, y, z;
};
inline V3 v3(double x, double y, double z) { return V3{x, y, z}; }
inline V3 add(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
inline V3 sub(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
inline V3 mul(V3 a, double s) { return v3(a.x * s, a.y * s, a.z * s); }
inline V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Rigid equilateral triangle of side L, centred on the guiding centre R(t) on a circle
// of radius AU, plane tilted by 60 degrees to the ecliptic, rotating once per orbit
// against the orbital sense ("cartwheel").  Guiding-centre phase 0 at t = 0.
// Numerical orbits (optional): spacecraft positions on the uniform time grid t_j = t0 + j dt,
// interpolated by the cubic through four neighbouring nodes (Lagrange form; nodes j-1 .. j+2
// around t, moved inwards at the ends of the grid).  With a grid set, every arm has its own
// length |x_r - x_s| at the sample time and the TDI takes one delay per arm; without one, the
// rigid equal-arm triangle below.
struct OrbitGrid {
  std::vector<double> pos;  // [n][3 spacecraft][3 coordinates], m
  int n = 0;
  double t0 = 0.0, dt = 0.0;
};
OrbitGrid g_orbit;

void spacecraft_grid(double t, V3 x[3]) {
  const double u = (t - g_orbit.t0) / g_orbit.dt;
  int j = (int)std::floor(u) - 1;
  if (j < 0) j = 0;
  if (j > g_orbit.n - 4) j = g_orbit.n - 4;
  const double s = u - (double)j;
  const double w[4] = {-(s - 1.0) * (s - 2.0) * (s - 3.0) / 6.0, s * (s - 2.0) * (s - 3.0) / 2.0,
                       -s * (s - 1.0) * (s - 3.0) / 2.0, s * (s - 1.0) * (s - 2.0) / 6.0};
  for (int i = 0; i < 3; ++i) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 4; ++q)
      for (int k = 0; k < 3; ++k) acc[k] += w[q] * g_orbit.pos[((size_t)(j + q) * 3 + i) * 3 + k];
    x[i] = v3(acc[0], acc[1], acc[2]);
  }
}

inline double dist(V3 a, V3 b) {
  const V3 d = sub(a, b);
  return std::sqrt(d.x * d.x + d.y * d.y + d.z * d.z);
}

void spacecraft(double t, const Params& p, V3 x[3]) {
  if (g_orbit.n > 0) {
    spacecraft_grid(t, x);
    return;
  }
  const double a = 2.0 * kPi * t / p.P_orb;
  const V3 rhat = v3(std::cos(a), std::sin(a), 0.0);
  const V3 phat = v3(-std::sin(a), std::cos(a), 0.0);
  const V3 ncar = sub(v3(0.0, 0.0, 0.5), mul(rhat, std::sqrt(3.0) / 2.0));
  const V3 what = cross(ncar, phat);
  const V3 R = mul(rhat, p.AU);
  for (int i = 0; i < 3; ++i) {
    const double th = a - 2.0 * kPi * i / 3.0;
    x[i] = add(R, mul(add(mul(what, std::cos(th)), mul(phat, std::sin(th))), p.L / std::sqrt(3.0)));
  }
}

// ------------------------------------------------------------------ source
template <class R>
struct Source {
  R f0, fdot, beta, lam, amp, iota, psi, phi0;
  R k[3];        // propagation direction
  R ep[3][3];    // e_plus  (rotated by psi)
  R ec[3][3];    // e_cross (rotated by psi)
  R Ap, Ac;      // A_+ = A (1 + cos^2 iota), A_x = -2 A cos iota
};

template <class R>
Source<R> make_source(const R th[8]) {
  Source<R> s;
  s.f0 = th[0];
  s.fdot = th[1];
  s.beta = th[2];
  s.lam = th[3];
  s.amp = th[4];
  s.iota = th[5];
  s.psi = th[6];
  s.phi0 = th[7];
  const R cb = cos(s.beta), sb = sin(s.beta), cl = cos(s.lam), sl = sin(s.lam);
  // k = -(cos b cos l, cos b sin l, sin b): the wave travels away from the sky position
  s.k[0] = -(cb * cl);
  s.k[1] = -(cb * sl);
  s.k[2] = -sb;
  // transverse basis u, v with (u, v, k) right-handed
  const R u[3] = {sb * cl, sb * sl, -cb};
  const R v[3] = {sl, -cl, R(0.0) * cl};
  const R c2 = cos(2.0 * s.psi), s2 = sin(2.0 * s.psi);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const R epl = u[i] * u[j] - v[i] * v[j];
      const R ecr = u[i] * v[j] + v[i] * u[j];
      s.ep[i][j] = c2 * epl + s2 * ecr;
      s.ec[i][j] = c2 * ecr - s2 * epl;
    }
  const R ci = cos(s.iota);
  s.Ap = s.amp * (1.0 + ci * ci);
  s.Ac = -2.0 * s.amp * ci;
  return s;
}

template <class R>
R quad(const R e[3][3], const double n[3]) {
  R acc = R(0.0) * e[0][0];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) acc = acc + e[i][j] * (n[i] * n[j]);
  return acc;
}

template <class R>
R sinc(const R& x) {
  if (std::fabs(value(x)) < 1e-4) {
    const R x2 = x * x;
    return 1.0 - x2 / 6.0 + x2 * x2 / 120.0;
  }
  return sin(x) / x;
}

// Complex slow-time response of link s -> r at time t (sample of the slow series),
// carrier removed: the real link signal is Re[z e^{2 pi i q t / T}].
template <class R>
Cx<R> link(const Source<R>& s, const V3 x[3], int r, int snd, double t, const R& dfreq, const Params& p) {
  const double L = g_orbit.n > 0 ? dist(x[r], x[snd]) : p.L;  // this link's arm length
  const double n[3] = {(x[r].x - x[snd].x) / L, (x[r].y - x[snd].y) / L, (x[r].z - x[snd].z) / L};
  const R kn = s.k[0] * n[0] + s.k[1] * n[1] + s.k[2] * n[2];
  const R f = s.f0 + s.fdot * t;
  const R u = kPi * f * L * (1.0 - kn) / kC;
  // n.H.n for the complex field H = A+ e+ - i Ax ex
  const Cx<R> nhn = cx<R>(s.Ap * quad(s.ep, n), -(s.Ac * quad(s.ec, n)));
  const double mid[3] = {0.5 * (x[r].x + x[snd].x), 0.5 * (x[r].y + x[snd].y), 0.5 * (x[r].z + x[snd].z)};
  const R kmid = s.k[0] * mid[0] + s.k[1] * mid[1] + s.k[2] * mid[2];
  // Phi(t) - 2 pi q t / T = 2 pi (df t + fdot t^2 / 2) + phi0, then the travel-time phase
  const R phase = 2.0 * kPi * (dfreq * t + 0.5 * s.fdot * t * t) + s.phi0 -
                  2.0 * kPi * f * (0.5 * L + kmid) / kC;
  const R amp = kPi * f * L / kC * sinc(u);
  // z = -i amp nhn e^{i phase}
  const Cx<R> e = expi(phase);
  const Cx<R> z = nhn * e;
  return cx<R>(z.im * amp, -(z.re * amp));
}

// One sample of the slow series of the A, E, T channels at time t: the TDI response
// with the carrier e^{2 pi i q t / T} taken out (ch[0..2] = A, E, T).
template <class R>
void slow_sample(const Source<R>& s, double t, const R& dfreq, const Params& p, Cx<R> ch[3]) {
  V3 x[3];
  spacecraft(t, p, x);
  // links (0-based spacecraft 0,1,2 = the usual 1,2,3); y_rs is received at r from s
  const Cx<R> z12 = link(s, x, 0, 1, t, dfreq, p), z21 = link(s, x, 1, 0, t, dfreq, p);
  const Cx<R> z13 = link(s, x, 0, 2, t, dfreq, p), z31 = link(s, x, 2, 0, t, dfreq, p);
  const Cx<R> z23 = link(s, x, 1, 2, t, dfreq, p), z32 = link(s, x, 2, 1, t, dfreq, p);
  const R f = s.f0 + s.fdot * t;
  const Cx<R> one = cx<R>(R(1.0) + 0.0 * f, R(0.0) * f);
  if (g_orbit.n > 0) {
    // unequal arms, each delay at the local frequency: arm 12 (c), 23 (a), 31 (b).  With the
    // link phasors frozen at t, X1 = y13 + D_b y31 + D_b^2 y12 + D_b^2 D_c y21 - y12 - D_c y21
    // - D_c^2 y13 - D_c^2 D_b y31 = (1 - D_c^2)(y13 + D_b y31) - (1 - D_b^2)(y12 + D_c y21);
    // Y, Z cyclically; the second generation multiplies X by 1 - D_b^2 D_c^2 (X1(t) minus X1
    // delayed by both arms twice), Y and Z likewise.
    const Cx<R> Dc = expi(-(2.0 * kPi * f * dist(x[0], x[1]) / kC));
    const Cx<R> Da = expi(-(2.0 * kPi * f * dist(x[1], x[2]) / kC));
    const Cx<R> Db = expi(-(2.0 * kPi * f * dist(x[2], x[0]) / kC));
    const Cx<R> ga = one - Da * Da, gb = one - Db * Db, gc = one - Dc * Dc;
    Cx<R> X = gc * (z13 + Db * z31) - gb * (z12 + Dc * z21);
    Cx<R> Y = ga * (z21 + Dc * z12) - gc * (z23 + Da * z32);
    Cx<R> Z = gb * (z32 + Da * z23) - ga * (z31 + Db * z13);
    if (p.tdi == 2) {
      X = (one - (Db * Db) * (Dc * Dc)) * X;
      Y = (one - (Dc * Dc) * (Da * Da)) * Y;
      Z = (one - (Da * Da) * (Db * Db)) * Z;
    }
    ch[0] = scaled(Z - X, 1.0 / std::sqrt(2.0));
    ch[1] = scaled((X - scaled(Y, 2.0)) + Z, 1.0 / std::sqrt(6.0));
    ch[2] = scaled((X + Y) + Z, 1.0 / std::sqrt(3.0));
    return;
  }
  const Cx<R> D = expi(-(2.0 * kPi * f * p.L / kC));  // one-arm delay at the local frequency
  const Cx<R> g = one - D * D;
  // X(t) = y13 + y31(t-L) + y12(t-2L) + y21(t-3L) - y12 - y21(t-L) - y13(t-2L) - y31(t-3L);
  // a delay by L multiplies the slowly varying link phasor by D; Y, Z by cyclic relabelling
  Cx<R> X = g * ((z13 + D * z31) - (z12 + D * z21));
  Cx<R> Y = g * ((z21 + D * z12) - (z23 + D * z32));
  Cx<R> Z = g * ((z32 + D * z23) - (z31 + D * z13));
  if (p.tdi == 2) {
    // second generation: the eight further links of X2 (delays 4L .. 7L) are the four-arm-delayed
    // copy of X with the opposite sign when the arms are equal, X2(t) = X(t) - X(t - 4L)
    const Cx<R> D2 = D * D;
    const Cx<R> g2 = one - D2 * D2;
    X = g2 * X;
    Y = g2 * Y;
    Z = g2 * Z;
  }
  ch[0] = scaled(Z - X, 1.0 / std::sqrt(2.0));                   // A
  ch[1] = scaled((X - scaled(Y, 2.0)) + Z, 1.0 / std::sqrt(6.0));  // E
  ch[2] = scaled((X + Y) + Z, 1.0 / std::sqrt(3.0));              // T
}

// Radix-2 decimation-in-time DFT, X_j = sum_m x_m e^{-2 pi i j m / n}, n a power of two.
template <class R>
void dft_forward(std::vector<Cx<R>>& a) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    for (size_t i = 0; i < n; i += len)
      for (size_t j = 0; j < len / 2; ++j) {
        const double ang = -2.0 * kPi * (double)j / (double)len;
        const Cx<R> w = cx<R>(R(std::cos(ang)) + 0.0 * a[0].re, R(std::sin(ang)) + 0.0 * a[0].re);
        const Cx<R> u0 = a[i + j];
        const Cx<R> v0 = a[i + j + len / 2] * w;
        a[i + j] = u0 + v0;
        a[i + j + len / 2] = u0 - v0;
      }
  }
}

// Template on bins first_bin .. first_bin + N - 1 for C channels (A, E[, T]):
// h[c][i] = T / (2N) * DFT_N[S_c][(i - N/2) mod N], first_bin = q - N/2.
template <class R>
int64_t waveform(const R th[8], int N, int C, const Params& p, std::vector<Cx<R>> h[3]) {
  const Source<R> s = make_source(th);
  const double f0v = value(s.f0);
  const int64_t q = (int64_t)std::floor(f0v * p.T);
  const R dfreq = s.f0 - (double)q / p.T;
  for (int c = 0; c < C; ++c) h[c].assign(N, cx<R>(R(0.0) * s.f0, R(0.0) * s.f0));
  std::vector<Cx<R>> S[3];
  for (int c = 0; c < 3; ++c) S[c].assign(N, cx<R>(R(0.0) * s.f0, R(0.0) * s.f0));
  for (int m = 0; m < N; ++m) {
    const double t = p.T * (double)m / (double)N;
    Cx<R> ch[3];
    slow_sample(s, t, dfreq, p, ch);
    for (int c = 0; c < 3; ++c) S[c][m] = ch[c];
  }
  const double norm = p.T / (2.0 * (double)N);
  for (int c = 0; c < C; ++c) {
    dft_forward(S[c]);
    for (int i = 0; i < N; ++i) {
      const int j = (i - N / 2 + N) % N;
      h[c][i] = scaled(S[c][j], norm);
    }
  }
  return q - N / 2;
}

// logL and components over the window bins k0..k0+W-1 of C channels.
template <class R>
R loglik_one(const R th[8], int64_t k0, int W, int N, int C, const double* d, const double* w,
             const Params& p, double* dh_out, double* hh_out) {
  std::vector<Cx<R>> h[3];
  const int64_t fb = waveform(th, N, C, p, h);
  R acc = R(0.0) * th[0];
  double dh = 0.0, hh = 0.0;
  for (int c = 0; c < C; ++c)
    for (int k = 0; k < W; ++k) {
      const int64_t i = k0 + k - fb;
      Cx<R> hk = cx<R>(R(0.0) * th[0], R(0.0) * th[0]);
      if (i >= 0 && i < N) hk = h[c][(size_t)i];
      const double dre = d[2 * ((size_t)c * W + k)], dim = d[2 * ((size_t)c * W + k) + 1];
      const double wk = w[(size_t)c * W + k];
      const R rre = dre - hk.re, rim = dim - hk.im;
      acc = acc + wk * (rre * rre + rim * rim);
      dh += wk * (dre * value(hk.re) + dim * value(hk.im));
      hh += wk * (value(hk.re) * value(hk.re) + value(hk.im) * value(hk.im));
    }
  if (dh_out) *dh_out = dh;
  if (hh_out) *hh_out = hh;
  return -0.5 * acc;
}

Params mkp(double T, double P_orb, double L, double AU, int tdi) {
  Params p;
  p.T = T;
  p.P_orb = P_orb;
  p.L = L;
  p.AU = AU;
  p.tdi = tdi;
  return p;
}

int threads(int n) {
#ifdef _OPENMP
  return n > 0 ? n : omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

}  // namespace

extern "C" {

// Threads the OpenMP loops over candidates would use for nthreads <= 0.
int gbo_max_threads(void) { return threads(0); }

// Numerical orbits for every later call: positions pos[n][3][3] (spacecraft, xyz; m) at
// t_j = t0 + j dt (n >= 4, dt > 0); returns 0, or -1 on bad arguments.  gbo_clear_orbit()
// returns to the analytic rigid triangle.  Not for use while other calls run.
int gbo_set_orbit(const double* pos, int n, double t0, double dt) {
  if (!pos || n < 4 || !(dt > 0.0)) return -1;
  g_orbit.pos.assign(pos, pos + (size_t)n * 9);
  g_orbit.n = n;
  g_orbit.t0 = t0;
  g_orbit.dt = dt;
  return 0;
}
void gbo_clear_orbit(void) { g_orbit = OrbitGrid(); }

// Spacecraft positions x[3][3] (m) at time t.
void gbo_spacecraft(double t, double P_orb, double L, double AU, double* x_out) {
  Params p = mkp(1.0, P_orb, L, AU, 1);
  V3 x[3];
  spacecraft(t, p, x);
  for (int i = 0; i < 3; ++i) {
    x_out[3 * i] = x[i].x;
    x_out[3 * i + 1] = x[i].y;
    x_out[3 * i + 2] = x[i].z;
  }
}

// Forward DFT of n complex values (interleaved), in place; n a power of two.
void gbo_dft(double* z, int n) {
  std::vector<Cx<double>> a(n);
  for (int i = 0; i < n; ++i) a[i] = cx<double>(z[2 * i], z[2 * i + 1]);
  dft_forward(a);
  for (int i = 0; i < n; ++i) {
    z[2 * i] = a[i].re;
    z[2 * i + 1] = a[i].im;
  }
}

// Slow series S_c(t_m) (before the DFT) of one source: out[c][m] complex, c < 3.
void gbo_slow_series(const double* theta, int N, double T, double P_orb, double L, double AU, int tdi, double* out) {
  Params p = mkp(T, P_orb, L, AU, tdi);
  const Source<double> s = make_source(theta);
  const int64_t q = (int64_t)std::floor(theta[0] * T);
  const double dfreq = theta[0] - (double)q / T;
  for (int m = 0; m < N; ++m) {
    Cx<double> ch[3];
    slow_sample(s, T * (double)m / (double)N, dfreq, p, ch);
    for (int c = 0; c < 3; ++c) {
      out[2 * ((size_t)c * N + m)] = ch[c].re;
      out[2 * ((size_t)c * N + m) + 1] = ch[c].im;
    }
  }
}

// Templates of B sources: h_out[B][C][N] complex (interleaved), first_bin[B].
void gbo_waveform(const double* theta, int64_t B, int N, int C, double T, double P_orb, double L,
                  double AU, int tdi, double* h_out, int64_t* first_bin, int nthreads) {
  Params p = mkp(T, P_orb, L, AU, tdi);
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads(nthreads))
  for (int64_t b = 0; b < B; ++b) {
    std::vector<Cx<double>> h[3];
    first_bin[b] = waveform(theta + 8 * b, N, C, p, h);
    for (int c = 0; c < C; ++c)
      for (int i = 0; i < N; ++i) {
        h_out[2 * (((size_t)b * C + c) * N + i)] = h[c][i].re;
        h_out[2 * (((size_t)b * C + c) * N + i) + 1] = h[c][i].im;
      }
  }
}

// logL of B candidates on one window (d: [C][W] complex interleaved, w: [C][W]);
// comps (may be null): [B][2] = <d|h>, <h|h>.
void gbo_loglik(const double* theta, int64_t B, int64_t k0, int W, int N, int C, const double* d,
                const double* w, double T, double P_orb, double L, double AU, int tdi, double* logL,
                double* comps, int nthreads) {
  Params p = mkp(T, P_orb, L, AU, tdi);
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads(nthreads))
  for (int64_t b = 0; b < B; ++b) {
    double dh = 0.0, hh = 0.0;
    logL[b] = loglik_one<double>(theta + 8 * b, k0, W, N, C, d, w, p, &dh, &hh);
    if (comps) {
      comps[2 * b] = dh;
      comps[2 * b + 1] = hh;
    }
  }
}

// logL and its gradient [B][8] with respect to (f0, fdot, beta, lambda, A, iota, psi, phi0),
// by forward-mode dual numbers through every step above (q held fixed).
void gbo_loglik_grad(const double* theta, int64_t B, int64_t k0, int W, int N, int C, const double* d,
                     const double* w, double T, double P_orb, double L, double AU, int tdi, double* logL,
                     double* grad, int nthreads) {
  Params p = mkp(T, P_orb, L, AU, tdi);
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads(nthreads))
  for (int64_t b = 0; b < B; ++b) {
    Dual th[8];
    for (int i = 0; i < 8; ++i) th[i] = seed(theta[8 * b + i], i);
    const Dual l = loglik_one<Dual>(th, k0, W, N, C, d, w, p, nullptr, nullptr);
    logL[b] = l.v;
    for (int i = 0; i < 8; ++i) grad[8 * b + i] = l.d[i];
  }
}

// Jacobian of the template: jac[8][C][N] complex = d h / d theta_i (same bins as gbo_waveform).
int64_t gbo_waveform_jacobian(const double* theta, int N, int C, double T, double P_orb, double L,
                              double AU, int tdi, double* jac) {
  Params p = mkp(T, P_orb, L, AU, tdi);
  Dual th[8];
  for (int i = 0; i < 8; ++i) th[i] = seed(theta[i], i);
  std::vector<Cx<Dual>> h[3];
  const int64_t fb = waveform(th, N, C, p, h);
  for (int i = 0; i < 8; ++i)
    for (int c = 0; c < C; ++c)
      for (int m = 0; m < N; ++m) {
        jac[2 * (((size_t)i * C + c) * N + m)] = h[c][m].re.d[i];
        jac[2 * (((size_t)i * C + c) * N + m) + 1] = h[c][m].im.d[i];
      }
  return fb;
}

// Fisher matrix F_ij = sum_c sum_k w Re(d_i h conj(d_j h)) over window bins k0..k0+W-1
// (Sec. III G; the garbled "partial p(d|theta)" read as the template derivative).
void gbo_fisher(const double* theta, int64_t k0, int W, int N, int C, const double* w, double T,
                double P_orb, double L, double AU, int tdi, double* F) {
  std::vector<double> jac((size_t)16 * C * N);
  const int64_t fb = gbo_waveform_jacobian(theta, N, C, T, P_orb, L, AU, tdi, jac.data());
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      double acc = 0.0;
      for (int c = 0; c < C; ++c)
        for (int k = 0; k < W; ++k) {
          const int64_t m = k0 + k - fb;
          if (m < 0 || m >= N) continue;
          const double* a = &jac[2 * (((size_t)i * C + c) * N + m)];
          const double* b = &jac[2 * (((size_t)j * C + c) * N + m)];
          acc += w[(size_t)c * W + k] * (a[0] * b[0] + a[1] * b[1]);
        }
      F[8 * i + j] = acc;
    }
}

// Independent-proposal Metropolis-Hastings chain (Algorithm 4, acceptance equation of
// Sec. III G).  Given logL_i = ln p(d|theta_i), log_g_i = ln g(theta_i) and uniforms u_i:
// start at sample 0; for i = 1..n-1 accept with probability
//   alpha = min(1, [L_i / L_c * g_c / g_i]^(1/T)).
// "u_i < alpha" is evaluated in logarithms as  pi_c < pi_i - T ln u_i  with
// pi = ln L - ln g (equivalent for T > 0; u_i = 0 always accepts).
// chain[i] = index of the state after step i (chain[0] = 0); returns the accept count.
int64_t gbo_mh_chain(const double* logL, const double* log_g, const double* u, int64_t n,
                     double temperature, int32_t* chain) {
  if (n <= 0) return 0;
  int64_t c = 0, acc = 0;
  chain[0] = 0;
  double pic = logL[0] - log_g[0];
  for (int64_t i = 1; i < n; ++i) {
    const double pii = logL[i] - log_g[i];
    const double tau = pii - temperature * std::log(u[i]);
    if (pic < tau) {
      c = i;
      pic = pii;
      ++acc;
    }
    chain[i] = (int32_t)c;
  }
  return acc;
}

}  // extern "C"
