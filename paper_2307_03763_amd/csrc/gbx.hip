// C ABI of the Galactic-binary likelihood (see include/gbx.h): contexts, plans, dispatch.
#include "../../include/gbx.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gbx_kernels.h"
#include "gbx_chain.h"
#include "gbx_post.h"
#include "gbx_noise.h"
#include "gbx_noise_global.h"
#include "gbx_de.h"
#include "gbx_variants.h"

using namespace gbx;


// ------------------------------------------------------------------------------- errors
static thread_local std::string g_err;

static gb_status fail(gb_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) return fail(GB_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------------------- set-up kernels
// Spacecraft of a rigid equilateral triangle (side L) around the guiding centre R(t) on a
// circle of radius AU; plane tilted by 60 degrees, turning once per orbit against the orbital
// sense (the classic first-order free-fall constellation).  Guiding-centre phase 0 at t = 0.
__global__ void k_orbit_table(double* ob64, float* ob32, int N, double T, double P, double L, double AU) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const double t = T * (double)m / (double)N;
  double sa, ca;
  sincospi(2.0 * t / P, &sa, &ca);
  const double r3 = sqrt(3.0);
  // in-plane unit vectors: phi = (-sin a, cos a, 0), w = n_c x phi = (-cos a / 2, -sin a / 2, -sqrt3/2)
  const double ph[3] = {-sa, ca, 0.0};
  const double wv[3] = {-0.5 * ca, -0.5 * sa, -0.5 * r3};
  double dx[3][3];
  for (int i = 0; i < 3; ++i) {
    double st, ct;
    sincospi(2.0 * t / P - 2.0 * i / 3.0, &st, &ct);
    for (int k = 0; k < 3; ++k) dx[i][k] = L / r3 * (ct * wv[k] + st * ph[k]);
  }
  double v[OB_FIELDS];
  v[OB_RX] = AU * ca / kC;
  v[OB_RY] = AU * sa / kC;
  for (int k = 0; k < 3; ++k) {
    v[OB_N12 + k] = (dx[0][k] - dx[1][k]) / L;
    v[OB_N23 + k] = (dx[1][k] - dx[2][k]) / L;
    v[OB_N31 + k] = (dx[2][k] - dx[0][k]) / L;
    v[OB_P1 + k] = dx[0][k] / kC;
    v[OB_P2 + k] = dx[1][k] / kC;
    v[OB_P3 + k] = dx[2][k] / kC;
  }
  v[OB_RZ] = 0.0;
  v[OB_LT12] = v[OB_LT23] = v[OB_LT31] = L / kC;
  for (int f = 0; f < OB_FIELDS; ++f) {
    ob64[f * N + m] = v[f];
    ob32[f * N + m] = (float)v[f];
  }
}

// The same table from numerical orbits: spacecraft positions pos[n][3][3] (m) on the grid
// t_j = t0 + j dt, interpolated at t_m = T m / N by the cubic through four neighbouring nodes
// (Lagrange form, nodes j-1 .. j+2 around t, moved inwards at the ends of the grid).  The
// guiding centre is the centroid; every arm gets its own unit vector and light time.
__global__ void k_orbit_table_grid(double* ob64, float* ob32, int N, double T, const double* __restrict__ pos,
                                   int n, double t0, double dt) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const double u = (T * (double)m / (double)N - t0) / dt;
  int j = (int)floor(u) - 1;
  j = j < 0 ? 0 : (j > n - 4 ? n - 4 : j);
  const double s = u - (double)j;
  const double w[4] = {-(s - 1.0) * (s - 2.0) * (s - 3.0) / 6.0, s * (s - 2.0) * (s - 3.0) / 2.0,
                       -s * (s - 1.0) * (s - 3.0) / 2.0, s * (s - 1.0) * (s - 2.0) / 6.0};
  double x[3][3];
  for (int i = 0; i < 3; ++i)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int q = 0; q < 4; ++q) acc += w[q] * pos[((size_t)(j + q) * 3 + i) * 3 + k];
      x[i][k] = acc;
    }
  double v[OB_FIELDS];
  double cen[3];
  for (int k = 0; k < 3; ++k) cen[k] = (x[0][k] + x[1][k] + x[2][k]) / 3.0;
  v[OB_RX] = cen[0] / kC;
  v[OB_RY] = cen[1] / kC;
  v[OB_RZ] = cen[2] / kC;
  const int r[3] = {0, 1, 2}, q[3] = {1, 2, 0};  // arms 12, 23, 31: (x_r - x_q) / |.|
  const int nf[3] = {OB_N12, OB_N23, OB_N31}, lf[3] = {OB_LT12, OB_LT23, OB_LT31};
  for (int a = 0; a < 3; ++a) {
    double d[3], l2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      d[k] = x[r[a]][k] - x[q[a]][k];
      l2 += d[k] * d[k];
    }
    const double l = sqrt(l2);
    for (int k = 0; k < 3; ++k) v[nf[a] + k] = d[k] / l;
    v[lf[a]] = l / kC;
  }
  for (int k = 0; k < 3; ++k) {
    v[OB_P1 + k] = (x[0][k] - cen[k]) / kC;
    v[OB_P2 + k] = (x[1][k] - cen[k]) / kC;
    v[OB_P3 + k] = (x[2][k] - cen[k]) / kC;
  }
  for (int f = 0; f < OB_FIELDS; ++f) {
    ob64[f * N + m] = v[f];
    ob32[f * N + m] = (float)v[f];
  }
}

__global__ void k_twiddles(double* tw64, float* tw32, int N) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  double s, c;
  sincospi(-2.0 * (double)m / (double)N, &s, &c);
  tw64[2 * m] = c;
  tw64[2 * m + 1] = s;
  tw32[2 * m] = (float)c;
  tw32[2 * m + 1] = (float)s;
}

// <d|d> of every window: one workgroup per window.
__global__ void __launch_bounds__(256) k_prepare(DevWin* wins, const double* d, const double* w) {
  const DevWin win = wins[blockIdx.x];
  const int64_t n = (int64_t)win.C * win.W;
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int64_t g = win.data_off + e;
    const double re = d[2 * g], im = d[2 * g + 1];
    acc += w[g] * (re * re + im * im);
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x / 64] = acc;
  __syncthreads();
  if (threadIdx.x == 0) wins[blockIdx.x].dd = part[0] + part[1] + part[2] + part[3];
}

// ------------------------------------------------------------------------------- variants
namespace {

const VariantList& all_variants() {
  static std::vector<Variant> v;
  static VariantList list{nullptr, 0};
  if (!list.v) {
    for (VariantList (*f)() : {gbx_variants_f64_loglik, gbx_variants_mixed_loglik, gbx_variants_mixed_grad,
                               gbx_variants_waveform}) {
      const VariantList l = f();
      v.insert(v.end(), l.v, l.v + l.n);
    }
    list.v = v.data();
    list.n = (int)v.size();
  }
  return list;
}

const Variant* find_variant(int prec, int N, int C, int mode) {
  const VariantList& l = all_variants();
  for (int i = 0; i < l.n; ++i) {
    const Variant& v = l.v[i];
    if (v.prec == prec && v.N == N && v.C == C && v.mode == mode) return &v;
  }
  return nullptr;
}

size_t lds_bytes(const Variant& v) {
  const size_t cpb = (size_t)v.WPB * 64 / v.LPC;
  return cpb * v.C * v.N * (v.prec == GB_FP64 ? 16 : 8);
}

bool pow2_in_range(int N) { return N >= 64 && N <= 1024 && (N & (N - 1)) == 0; }
int n_index(int N) {
  int i = 0;
  while ((64 << i) < N) ++i;
  return i;
}

}  // namespace

// ------------------------------------------------------------------------------- context
struct NTab {
  double* ob64 = nullptr;
  float* ob32 = nullptr;
  double* tw64 = nullptr;
  float* tw32 = nullptr;
};

struct gb_ctx {
  gb_config cfg;
  int device = 0;
  int n_cu = 256;
  NTab tab[5];
  const Variant* choice[2][5][2][3] = {};  // autotuned variant per precision, N, C, mode
  int uneq = 0;                              // numerical orbits set (gb_set_orbit)
};

static const Variant* pick_variant(const gb_ctx* c, int prec, int N, int C, int mode) {
  const Variant* v = (c && mode <= MODE_GRAD) ? c->choice[prec][n_index(N)][C - 2][mode] : nullptr;
  return v ? v : find_variant(prec, N, C, mode);
}

extern "C" const char* gb_last_error(void) { return g_err.c_str(); }

extern "C" gb_status gb_create(const gb_config* cfg, gb_ctx** out) {
  if (!out) return fail(GB_EINVAL, "gb_create: null output pointer");
  *out = nullptr;
  if (!cfg) return fail(GB_EINVAL, "gb_create: null config");
  if (!(cfg->T > 0) || !(cfg->orbit_period > 0) || !(cfg->arm_length > 0) || !(cfg->au > 0) ||
      !std::isfinite(cfg->T) || !std::isfinite(cfg->arm_length) || !std::isfinite(cfg->au))
    return fail(GB_EINVAL, "gb_create: T, orbit_period, arm_length and au must be positive and finite");
  if (cfg->tdi_generation < 0 || cfg->tdi_generation > 2 || cfg->reserved != 0)
    return fail(GB_EINVAL, "gb_create: tdi_generation must be 1 or 2 (0 means 1) and reserved 0");
  gb_ctx* c = new gb_ctx();
  c->cfg = *cfg;
  if (c->cfg.tdi_generation == 0) c->cfg.tdi_generation = 1;
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device);
  for (int i = 0; i < 5 && e == hipSuccess; ++i) {
    const int N = 64 << i;
    NTab& t = c->tab[i];
    e = hipMalloc(&t.ob64, sizeof(double) * OB_FIELDS * N);
    if (e == hipSuccess) e = hipMalloc(&t.ob32, sizeof(float) * OB_FIELDS * N);
    if (e == hipSuccess) e = hipMalloc(&t.tw64, sizeof(double) * 2 * N);
    if (e == hipSuccess) e = hipMalloc(&t.tw32, sizeof(float) * 2 * N);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_orbit_table, dim3((N + 63) / 64), dim3(64), 0, 0, t.ob64, t.ob32, N, cfg->T,
                       cfg->orbit_period, cfg->arm_length, cfg->au);
    hipLaunchKernelGGL(k_twiddles, dim3((N + 63) / 64), dim3(64), 0, 0, t.tw64, t.tw32, N);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    gb_destroy(c);
    return fail(e == hipErrorOutOfMemory ? GB_ENOMEM : GB_EHIP, "gb_create: %s", hipGetErrorString(e));
  }
  *out = c;
  return GB_OK;
}

extern "C" void gb_destroy(gb_ctx* c) {
  if (!c) return;
  for (NTab& t : c->tab) {
    (void)hipFree(t.ob64);
    (void)hipFree(t.ob32);
    (void)hipFree(t.tw64);
    (void)hipFree(t.tw32);
  }
  delete c;
}

static BatchArgs base_args(const gb_ctx* c, int N, int prec) {
  BatchArgs a;
  std::memset(&a, 0, sizeof a);
  const NTab& t = c->tab[n_index(N)];
  a.ob64 = t.ob64;
  a.obR = prec == GB_FP64 ? (const void*)t.ob64 : (const void*)t.ob32;
  a.tw = prec == GB_FP64 ? (const void*)t.tw64 : (const void*)t.tw32;
  a.T = c->cfg.T;
  a.Lc = c->cfg.arm_length / kC;
  a.tdi2 = c->cfg.tdi_generation == 2;
  return a;
}

static gb_status launch(const Variant* v, dim3 grid, BatchArgs& a, hipStream_t st) {
  void* args[] = {&a};
  HIPCHK(hipLaunchKernel(v->fn, grid, dim3(v->WPB * 64), args, lds_bytes(*v), st));
  return GB_OK;
}

extern "C" gb_status gb_waveform(gb_ctx* c, const double* theta, int64_t B, int N, int C,
                                 gb_precision prec, double* h_out, int64_t* first_bin, void* stream) {
  if (!c) return fail(GB_EINVAL, "gb_waveform: null context");
  if (B < 0) return fail(GB_EINVAL, "gb_waveform: B = %lld < 0", (long long)B);
  if (!pow2_in_range(N)) return fail(GB_EINVAL, "gb_waveform: N = %d is not a power of two in [64, 1024]", N);
  if (C != 2 && C != 3) return fail(GB_EINVAL, "gb_waveform: C = %d (must be 2 or 3)", C);
  if (prec != GB_FP64 && prec != GB_MIXED) return fail(GB_EINVAL, "gb_waveform: bad precision %d", (int)prec);
  if (B == 0) return GB_OK;
  if (!theta || !h_out || !first_bin) return fail(GB_EINVAL, "gb_waveform: null array");
  const Variant* v = pick_variant(c, prec, N, C, c->uneq ? MODE_WAVEFORM_UNEQ : MODE_WAVEFORM);
  if (!v) return fail(GB_EUNSUPPORTED, "gb_waveform: no variant for N=%d C=%d", N, C);
  BatchArgs a = base_args(c, N, prec);
  a.theta = theta;
  a.B = B;
  a.h_out = h_out;
  a.first_bin = first_bin;
  const int64_t cpb = (int64_t)v->WPB * 64 / v->LPC;
  const int64_t blocks = (B + cpb - 1) / cpb;
  if (blocks > 0x7fffffff) return fail(GB_EINVAL, "gb_waveform: B too large");
  return launch(v, dim3((unsigned)blocks), a, (hipStream_t)stream);
}

// ------------------------------------------------------------------------------- channels
// The rule of Sec. II: A, E below f*/2 = c / (4 pi L), A, E, T at and above, at the window centre.
static int paper_channels(const gb_ctx* c, int64_t k0, int32_t W) {
  const double f = ((double)k0 + 0.5 * (double)W) / c->cfg.T;
  return f >= kC / (4.0 * kPi * c->cfg.arm_length) ? 3 : 2;
}

extern "C" gb_status gb_set_orbit(gb_ctx* c, const double* pos, int32_t n_pts, double t0, double dt) {
  if (!c) return fail(GB_EINVAL, "gb_set_orbit: null context");
  const double T = c->cfg.T;
  if (!pos && n_pts == 0) {  // back to the analytic orbits
    for (int i = 0; i < 5; ++i) {
      const int N = 64 << i;
      hipLaunchKernelGGL(k_orbit_table, dim3((N + 63) / 64), dim3(64), 0, 0, c->tab[i].ob64, c->tab[i].ob32, N, T,
                         c->cfg.orbit_period, c->cfg.arm_length, c->cfg.au);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipDeviceSynchronize());
    c->uneq = 0;
    return GB_OK;
  }
  if (!pos) return fail(GB_EINVAL, "gb_set_orbit: null positions with n_pts = %d", n_pts);
  if (n_pts < 4 || n_pts > (1 << 24)) return fail(GB_EINVAL, "gb_set_orbit: n_pts = %d outside [4, 2^24]", n_pts);
  if (!std::isfinite(t0) || !std::isfinite(dt) || !(dt > 0.0))
    return fail(GB_EINVAL, "gb_set_orbit: t0 and dt must be finite, dt > 0");
  if (t0 > 0.0 || t0 + (double)(n_pts - 1) * dt < T)
    return fail(GB_EINVAL, "gb_set_orbit: the grid [%g, %g] s does not cover the observation [0, %g] s", t0,
                t0 + (double)(n_pts - 1) * dt, T);
  for (int64_t j = 0; j < n_pts; ++j) {
    const double* x = pos + 9 * j;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(x[k])) return fail(GB_EINVAL, "gb_set_orbit: position %lld is not finite", (long long)j);
    for (int a = 0; a < 3; ++a) {
      const double* p0 = x + 3 * a;
      const double* p1 = x + 3 * ((a + 1) % 3);
      const double l = std::sqrt((p0[0] - p1[0]) * (p0[0] - p1[0]) + (p0[1] - p1[1]) * (p0[1] - p1[1]) +
                                 (p0[2] - p1[2]) * (p0[2] - p1[2]));
      if (!(l > 0.0)) return fail(GB_EINVAL, "gb_set_orbit: two spacecraft coincide at node %lld", (long long)j);
    }
  }
  double* d_pos = nullptr;
  hipError_t e = hipMalloc(&d_pos, sizeof(double) * 9 * (size_t)n_pts);
  if (e == hipSuccess) e = hipMemcpy(d_pos, pos, sizeof(double) * 9 * (size_t)n_pts, hipMemcpyHostToDevice);
  for (int i = 0; i < 5 && e == hipSuccess; ++i) {
    const int N = 64 << i;
    hipLaunchKernelGGL(k_orbit_table_grid, dim3((N + 63) / 64), dim3(64), 0, 0, c->tab[i].ob64, c->tab[i].ob32, N, T,
                       d_pos, (int)n_pts, t0, dt);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(d_pos);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? GB_ENOMEM : GB_EHIP, "gb_set_orbit: %s", hipGetErrorString(e));
  c->uneq = 1;
  return GB_OK;
}

extern "C" gb_status gb_channels(const gb_ctx* c, int64_t k0, int32_t W, int32_t* C) {
  if (!c || !C) return fail(GB_EINVAL, "gb_channels: null argument");
  if (W < 1) return fail(GB_EINVAL, "gb_channels: W = %d < 1", W);
  *C = paper_channels(c, k0, W);
  return GB_OK;
}

// ------------------------------------------------------------------------------- plans
namespace {
struct Bucket {
  int prec, N, C;
  const Variant* v[6];  // per mode (MODE_*): logL, gradient and their numerical-orbit kernels used
  int grid[6];
  Tile* d_tiles = nullptr;
  int n_tiles = 0;
  unsigned* d_ctr = nullptr;  // [2]
};
}  // namespace

struct gb_plan {
  gb_ctx* ctx = nullptr;
  std::vector<gb_window> wins;
  DevWin* d_wins = nullptr;
  ChainWin* d_cw = nullptr;  // chain scratch of every window (max-tree, binary-lifting tables)
  double* d_tree = nullptr;
  int32_t* d_jump = nullptr;
  std::vector<Bucket> buckets;
  const double* prep_d = nullptr;
  const double* prep_w = nullptr;
  int64_t rows = 0;
};

extern "C" void gb_plan_destroy(gb_plan* p) {
  if (!p) return;
  (void)hipFree(p->d_wins);
  (void)hipFree(p->d_cw);
  (void)hipFree(p->d_tree);
  (void)hipFree(p->d_jump);
  for (Bucket& b : p->buckets) {
    (void)hipFree(b.d_tiles);
    (void)hipFree(b.d_ctr);
  }
  delete p;
}

static const int kTileIters = 4;  // workgroup passes per tile

extern "C" gb_status gb_plan_create(gb_ctx* c, const gb_window* windows, int n_win, gb_precision prec,
                                    gb_plan** out) {
  if (!out) return fail(GB_EINVAL, "gb_plan_create: null output pointer");
  *out = nullptr;
  if (!c) return fail(GB_EINVAL, "gb_plan_create: null context");
  if (n_win < 0 || (n_win > 0 && !windows)) return fail(GB_EINVAL, "gb_plan_create: bad window array");
  if (prec != GB_FP64 && prec != GB_MIXED && prec != GB_PER_WINDOW)
    return fail(GB_EINVAL, "gb_plan_create: bad precision %d", (int)prec);
  std::vector<DevWin> dw(n_win);
  int64_t rows = 0;
  std::vector<gb_window> resolved(windows, windows + n_win);
  for (int i = 0; i < n_win; ++i) {
    gb_window& w = resolved[i];
    const int wp = prec == GB_PER_WINDOW ? w.precision : (int)prec;
    if (!pow2_in_range(w.N)) return fail(GB_EINVAL, "window %d: N = %d is not a power of two in [64, 1024]", i, w.N);
    if (w.W < 1) return fail(GB_EINVAL, "window %d: W = %d < 1", i, w.W);
    if (w.C == 0) w.C = paper_channels(c, w.k0, w.W);
    if (w.C != 2 && w.C != 3) return fail(GB_EINVAL, "window %d: C = %d (must be 2, 3, or 0 for the rule)", i, w.C);
    if (w.k0 < 0) return fail(GB_EINVAL, "window %d: k0 < 0", i);
    if (w.data_off < 0 || w.cand_off < 0 || w.n_cand < 0)
      return fail(GB_EINVAL, "window %d: negative offset or count", i);
    if (w.n_cand > 0x7fffffffLL) return fail(GB_EINVAL, "window %d: more than 2^31 candidates", i);
    if (wp != GB_FP64 && wp != GB_MIXED) return fail(GB_EINVAL, "window %d: bad precision %d", i, wp);
    dw[i].k0 = w.k0;
    dw[i].data_off = w.data_off;
    dw[i].cand_off = w.cand_off;
    dw[i].n_cand = w.n_cand;
    dw[i].dd = 0.0;
    dw[i].W = w.W;
    dw[i].N = w.N;
    dw[i].C = w.C;
    dw[i].prec = wp;
    rows = std::max(rows, w.cand_off + w.n_cand);
  }
  gb_plan* p = new gb_plan();
  p->ctx = c;
  p->wins = resolved;
  p->rows = rows;
  // group by (N, C, precision); larger N first (longest work first)
  std::vector<int> order(n_win);
  for (int i = 0; i < n_win; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (dw[a].N != dw[b].N) return dw[a].N > dw[b].N;
    if (dw[a].C != dw[b].C) return dw[a].C > dw[b].C;
    return dw[a].prec < dw[b].prec;
  });
  hipError_t e = hipSuccess;
  for (size_t s = 0; s < order.size();) {
    size_t t = s;
    const DevWin& w0 = dw[order[s]];
    while (t < order.size() && dw[order[t]].N == w0.N && dw[order[t]].C == w0.C && dw[order[t]].prec == w0.prec) ++t;
    Bucket b;
    b.prec = w0.prec;
    b.N = w0.N;
    b.C = w0.C;
    for (int m = 0; m < 6; ++m) {
      b.v[m] = (m == MODE_WAVEFORM || m == MODE_WAVEFORM_UNEQ) ? nullptr : pick_variant(c, b.prec, b.N, b.C, m);
      b.grid[m] = 0;
    }
    if (!b.v[MODE_LOGLIK]) {
      gb_plan_destroy(p);
      return fail(GB_EUNSUPPORTED, "no kernel variant for N=%d C=%d", b.N, b.C);
    }
    // tiles hold a whole number of workgroup passes of the tuned likelihood and gradient kernels
    // (the counts are powers of two, so the larger is a multiple of the other); the kernel of
    // numerical orbits takes the same tiles in passes of its own width
    int cpb = 0;
    for (int m = 1; m < 3; ++m)
      if (b.v[m]) cpb = std::max(cpb, b.v[m]->WPB * 64 / b.v[m]->LPC);
    const int tsz = cpb * kTileIters;
    std::vector<Tile> tiles;
    for (size_t k = s; k < t; ++k) {
      const int wi = order[k];
      for (int64_t c0 = 0; c0 < dw[wi].n_cand; c0 += tsz) {
        Tile tl;
        tl.win = wi;
        tl.n = (int32_t)std::min<int64_t>(tsz, dw[wi].n_cand - c0);
        tl.c0 = c0;
        tiles.push_back(tl);
      }
    }
    b.n_tiles = (int)tiles.size();
    for (int m = 1; m < 6; ++m) {
      if (!b.v[m]) continue;
      int nb = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, b.v[m]->fn, b.v[m]->WPB * 64, lds_bytes(*b.v[m]));
      if (e != hipSuccess) break;
      b.grid[m] = std::max(1, std::min(b.n_tiles, std::max(1, nb) * c->n_cu));
    }
    if (e == hipSuccess && b.n_tiles > 0) {
      e = hipMalloc(&b.d_tiles, sizeof(Tile) * tiles.size());
      if (e == hipSuccess) e = hipMemcpy(b.d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMalloc(&b.d_ctr, 2 * sizeof(unsigned));
      if (e == hipSuccess) e = hipMemset(b.d_ctr, 0, 2 * sizeof(unsigned));
    }
    p->buckets.push_back(b);
    if (e != hipSuccess) break;
    s = t;
  }
  if (e == hipSuccess && n_win > 0) {
    e = hipMalloc(&p->d_wins, sizeof(DevWin) * n_win);
    if (e == hipSuccess) e = hipMemcpy(p->d_wins, dw.data(), sizeof(DevWin) * n_win, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && n_win > 0) {
    // chain scratch: per window a max-tree of 2P doubles and K levels of n + 1 jump entries
    std::vector<ChainWin> cw(n_win);
    int64_t toff = 0, joff = 0;
    for (int i = 0; i < n_win; ++i) {
      const int64_t n = dw[i].n_cand;
      int64_t P = 1;
      while (P < n) P <<= 1;
      int K = 1;
      while (((int64_t)1 << K) <= n) ++K;
      cw[i].tree_off = toff;
      cw[i].jump_off = joff;
      cw[i].P = P;
      cw[i].K = K;
      cw[i].pad = 0;
      toff += 2 * P;
      joff += (int64_t)K * (n + 1);
    }
    e = hipMalloc(&p->d_cw, sizeof(ChainWin) * n_win);
    if (e == hipSuccess) e = hipMemcpy(p->d_cw, cw.data(), sizeof(ChainWin) * n_win, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->d_tree, sizeof(double) * (size_t)toff);
    if (e == hipSuccess) e = hipMalloc(&p->d_jump, sizeof(int32_t) * (size_t)joff);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    gb_plan_destroy(p);
    return fail(e == hipErrorOutOfMemory ? GB_ENOMEM : GB_EHIP, "gb_plan_create: %s", hipGetErrorString(e));
  }
  *out = p;
  return GB_OK;
}

extern "C" gb_status gb_plan_info(const gb_plan* p, int64_t* rows, int* n_win, int64_t* data_len) {
  if (!p) return fail(GB_EINVAL, "gb_plan_info: null plan");
  if (rows) *rows = p->rows;
  if (n_win) *n_win = (int)p->wins.size();
  if (data_len) {
    int64_t m = 0;
    for (const gb_window& w : p->wins) m = std::max(m, w.data_off + (int64_t)w.C * w.W);
    *data_len = m;
  }
  return GB_OK;
}

extern "C" gb_status gb_window_prepare(gb_plan* p, const double* d, const double* w, void* stream) {
  if (!p) return fail(GB_EINVAL, "gb_window_prepare: null plan");
  if (p->wins.empty()) {
    p->prep_d = d;
    p->prep_w = w;
    return GB_OK;
  }
  if (!d || !w) return fail(GB_EINVAL, "gb_window_prepare: null data or weights");
  hipLaunchKernelGGL(k_prepare, dim3((unsigned)p->wins.size()), dim3(256), 0, (hipStream_t)stream, p->d_wins, d, w);
  HIPCHK(hipGetLastError());
  p->prep_d = d;
  p->prep_w = w;
  return GB_OK;
}

static gb_status run_batch(gb_plan* p, int mode, const double* d, const double* w, const double* theta,
                           double* logL, double* comps, double* grad, hipStream_t st, const char* who) {
  if (!p) return fail(GB_EINVAL, "%s: null plan", who);
  if (p->rows == 0) return GB_OK;
  if (!d || !w || !theta || !logL) return fail(GB_EINVAL, "%s: null array", who);
  if (d != p->prep_d || w != p->prep_w)
    return fail(GB_EINVAL, "%s: data/weights differ from the ones passed to gb_window_prepare", who);
  if (mode == MODE_GRAD && !grad) return fail(GB_EINVAL, "%s: null gradient array", who);
  // numerical orbits take the kernels of one light time per arm, chosen at launch so that plans
  // built before gb_set_orbit follow it
  if (p->ctx->uneq) mode = mode == MODE_GRAD ? MODE_GRAD_UNEQ : MODE_LOGLIK_UNEQ;
  // every bucket must have a kernel before any is launched, so a refused call writes nothing
  for (const Bucket& b : p->buckets) {
    if (b.n_tiles == 0 || b.v[mode]) continue;
    if ((mode == MODE_GRAD || mode == MODE_GRAD_UNEQ) && b.prec == GB_FP64)
      return fail(GB_EUNSUPPORTED,
                  "%s: the FP64 gradient is switched off (its kernels faulted on the GPU; cause not yet known); "
                  "use GB_MIXED", who);
    return fail(GB_EUNSUPPORTED, "%s: no kernel variant for N=%d C=%d", who, b.N, b.C);
  }
  for (Bucket& b : p->buckets) {
    if (b.n_tiles == 0) continue;
    const Variant* v = b.v[mode];
    BatchArgs a = base_args(p->ctx, b.N, b.prec);
    a.wins = p->d_wins;
    a.tiles = b.d_tiles;
    a.n_tiles = b.n_tiles;
    a.ctr = b.d_ctr;
    a.d = d;
    a.w = w;
    a.theta = theta;
    a.logL = logL;
    a.comps = comps;
    a.grad = grad;
    gb_status s = launch(v, dim3(b.grid[mode]), a, st);
    if (s != GB_OK) return s;
  }
  return GB_OK;
}

extern "C" gb_status gb_loglik(gb_plan* p, const double* d, const double* w, const double* theta, double* logL,
                               double* comps, void* stream) {
  return run_batch(p, MODE_LOGLIK, d, w, theta, logL, comps, nullptr, (hipStream_t)stream, "gb_loglik");
}

extern "C" gb_status gb_loglik_grad(gb_plan* p, const double* d, const double* w, const double* theta,
                                    double* logL, double* grad, void* stream) {
  return run_batch(p, MODE_GRAD, d, w, theta, logL, nullptr, grad, (hipStream_t)stream, "gb_loglik_grad");
}

extern "C" gb_status gb_mh_step(gb_plan* p, const double* d, const double* w, const double* theta,
                                const double* log_g, const double* u, double temperature, double* logL,
                                int32_t* chain, int64_t* n_accept, void* stream) {
  if (!p) return fail(GB_EINVAL, "gb_mh_step: null plan");
  if (!(temperature > 0) || !std::isfinite(temperature))
    return fail(GB_EINVAL, "gb_mh_step: temperature must be positive and finite");
  if (p->wins.empty()) return GB_OK;
  if (!log_g || !u || !chain || !n_accept) return fail(GB_EINVAL, "gb_mh_step: null array");
  gb_status s = run_batch(p, MODE_LOGLIK, d, w, theta, logL, nullptr, nullptr, (hipStream_t)stream, "gb_mh_step");
  if (s != GB_OK) return s;
  hipLaunchKernelGGL(k_mh_chain, dim3((unsigned)p->wins.size()), dim3(1024), 0, (hipStream_t)stream, p->d_wins,
                     p->d_cw, logL, log_g, u, temperature, p->d_tree, p->d_jump, chain, n_accept);
  HIPCHK(hipGetLastError());
  return GB_OK;
}

// ------------------------------------------------------------------------------- posterior helpers
extern "C" gb_status gb_fisher(gb_ctx* c, const double* theta, const double* steps, int n, const gb_window* windows,
                               const double* w, double* F, void* stream) {
  if (!c) return fail(GB_EINVAL, "gb_fisher: null context");
  if (n < 0 || (n > 0 && (!windows || !theta || !steps || !w || !F))) return fail(GB_EINVAL, "gb_fisher: bad arguments");
  if (n == 0) return GB_OK;
  std::vector<FisherWin> fw(n);
  for (int i = 0; i < n; ++i) {
    const gb_window& g = windows[i];
    if (!pow2_in_range(g.N)) return fail(GB_EINVAL, "gb_fisher: source %d: N = %d is not a power of two in [64, 1024]", i, g.N);
    if (g.C != 2 && g.C != 3) return fail(GB_EINVAL, "gb_fisher: source %d: C = %d (must be 2 or 3)", i, g.C);
    if (g.W < 1 || g.k0 < 0 || g.data_off < 0) return fail(GB_EINVAL, "gb_fisher: source %d: bad window", i);
    fw[i].k0 = g.k0;
    fw[i].data_off = g.data_off;
    fw[i].W = g.W;
    fw[i].pad = 0;
  }
  hipStream_t st = (hipStream_t)stream;
  FisherWin* d_fw = nullptr;
  int32_t* d_idx = nullptr;
  double *d_th = nullptr, *d_h = nullptr;
  int64_t* d_fb = nullptr;
  hipError_t e = hipMalloc(&d_fw, sizeof(FisherWin) * n);
  if (e == hipSuccess) e = hipMemcpyAsync(d_fw, fw.data(), sizeof(FisherWin) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMalloc(&d_idx, sizeof(int32_t) * n);
  gb_status status = GB_OK;
  // one (N, C) group at a time: templates of its 17 points per source, then the reduction
  std::vector<char> done(n, 0);
  for (int i0 = 0; i0 < n && e == hipSuccess && status == GB_OK; ++i0) {
    if (done[i0]) continue;
    const int N = windows[i0].N, C = windows[i0].C;
    std::vector<int32_t> idx;
    for (int i = i0; i < n; ++i)
      if (!done[i] && windows[i].N == N && windows[i].C == C) {
        idx.push_back(i);
        done[i] = 1;
      }
    const int m = (int)idx.size();
    const int64_t B = (int64_t)m * kFdPoints;
    e = hipMemcpyAsync(d_idx, idx.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_th);
    (void)hipFree(d_h);
    (void)hipFree(d_fb);
    d_th = d_h = nullptr;
    d_fb = nullptr;
    if (e == hipSuccess) e = hipMalloc(&d_th, sizeof(double) * 8 * B);
    if (e == hipSuccess) e = hipMalloc(&d_h, sizeof(double) * 2 * C * N * B);
    if (e == hipSuccess) e = hipMalloc(&d_fb, sizeof(int64_t) * B);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(k_fisher_points, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, theta, steps, d_idx, m, d_th);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    status = gb_waveform(c, d_th, B, N, C, GB_FP64, d_h, d_fb, stream);
    if (status != GB_OK) break;
    hipLaunchKernelGGL(k_fisher_reduce, dim3((unsigned)m), dim3(256), 0, st, d_h, d_fb, d_idx, m, d_fw, w, steps, N, C, F);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (void* q : {(void*)d_fw, (void*)d_idx, (void*)d_th, (void*)d_h, (void*)d_fb}) (void)hipFree(q);
  if (status != GB_OK) return status;
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? GB_ENOMEM : GB_EHIP, "gb_fisher: %s", hipGetErrorString(e));
  return GB_OK;
}

extern "C" gb_status gb_add_templates(gb_ctx* c, const gb_window* windows, int n_win, const double* theta,
                                      const int32_t* src_win, int n_src, double sign, const double* d_in,
                                      double* d_out, void* stream) {
  if (!c) return fail(GB_EINVAL, "gb_add_templates: null context");
  if (n_win < 0 || n_src < 0 || (n_win > 0 && (!windows || !d_in || !d_out)) || (n_src > 0 && (!theta || !src_win)))
    return fail(GB_EINVAL, "gb_add_templates: bad arguments");
  if (n_win == 0) return GB_OK;
  for (int i = 0; i < n_win; ++i) {
    const gb_window& g = windows[i];
    if (!pow2_in_range(g.N) || (g.C != 2 && g.C != 3) || g.W < 1 || g.k0 < 0 || g.data_off < 0)
      return fail(GB_EINVAL, "gb_add_templates: window %d: bad N, C, W, k0 or offset", i);
  }
  for (int s = 0; s < n_src; ++s)
    if (src_win[s] < 0 || src_win[s] >= n_win) return fail(GB_EINVAL, "gb_add_templates: source %d: bad window index", s);
  hipStream_t st = (hipStream_t)stream;
  // (N, C) groups of windows; per group the list of its sources and their templates
  std::vector<AddWin> aw(n_win);
  std::vector<void*> bufs;
  std::vector<std::vector<int32_t>> win_src(n_win);
  std::vector<int32_t> pos_in_group(n_src, -1);
  hipError_t e = hipSuccess;
  gb_status status = GB_OK;
  std::vector<char> done(n_win, 0);
  for (int w0 = 0; w0 < n_win && e == hipSuccess && status == GB_OK; ++w0) {
    if (done[w0]) continue;
    const int N = windows[w0].N, C = windows[w0].C;
    std::vector<int32_t> gsrc;  // sources of this group, in input order
    for (int s = 0; s < n_src; ++s)
      if (windows[src_win[s]].N == N && windows[src_win[s]].C == C) {
        pos_in_group[s] = (int32_t)gsrc.size();
        gsrc.push_back(s);
      }
    double* d_th = nullptr;
    double* d_h = nullptr;
    int64_t* d_fb = nullptr;
    int32_t* d_src = nullptr;
    const int m = (int)gsrc.size();
    std::vector<int32_t> lists;  // per window of the group: its sources (group positions)
    std::vector<int> win_of_group;
    for (int w = w0; w < n_win; ++w)
      if (!done[w] && windows[w].N == N && windows[w].C == C) {
        done[w] = 1;
        win_of_group.push_back(w);
      }
    for (int s : gsrc) win_src[src_win[s]].push_back(pos_in_group[s]);
    std::vector<int64_t> starts;
    for (int w : win_of_group) {
      starts.push_back((int64_t)lists.size());
      lists.insert(lists.end(), win_src[w].begin(), win_src[w].end());
    }
    int32_t* d_gidx = nullptr;
    if (m > 0) {
      // gather the group's parameters
      e = hipMalloc(&d_th, sizeof(double) * 8 * m);
      if (e == hipSuccess) e = hipMalloc(&d_gidx, sizeof(int32_t) * m);
      if (e == hipSuccess) e = hipMemcpyAsync(d_gidx, gsrc.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((8 * m + 255) / 256)), dim3(256), 0, st, theta, d_gidx, m, d_th);
        e = hipGetLastError();
      }
      if (e == hipSuccess) e = hipMalloc(&d_h, sizeof(double) * 2 * (size_t)C * N * m);
      if (e == hipSuccess) e = hipMalloc(&d_fb, sizeof(int64_t) * m);
      if (e == hipSuccess) status = gb_waveform(c, d_th, m, N, C, GB_FP64, d_h, d_fb, stream);
    }
    if (e == hipSuccess && !lists.empty()) {
      e = hipMalloc(&d_src, sizeof(int32_t) * lists.size());
      if (e == hipSuccess) e = hipMemcpyAsync(d_src, lists.data(), sizeof(int32_t) * lists.size(), hipMemcpyHostToDevice, st);
    }
    for (void* b : {(void*)d_th, (void*)d_h, (void*)d_fb, (void*)d_src, (void*)d_gidx})
      if (b) bufs.push_back(b);
    for (size_t q = 0; q < win_of_group.size(); ++q) {
      const int w = win_of_group[q];
      aw[w].k0 = windows[w].k0;
      aw[w].data_off = windows[w].data_off;
      aw[w].h = d_h;
      aw[w].fb = d_fb;
      aw[w].src = d_src ? d_src + starts[q] : nullptr;
      aw[w].W = windows[w].W;
      aw[w].N = N;
      aw[w].C = C;
      aw[w].n_src = (int32_t)win_src[w].size();
    }
  }
  AddWin* d_aw = nullptr;
  if (e == hipSuccess && status == GB_OK) e = hipMalloc(&d_aw, sizeof(AddWin) * n_win);
  if (e == hipSuccess && status == GB_OK)
    e = hipMemcpyAsync(d_aw, aw.data(), sizeof(AddWin) * n_win, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && status == GB_OK) {
    hipLaunchKernelGGL(k_add_templates, dim3((unsigned)n_win), dim3(256), 0, st, d_aw, sign, d_in, d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_aw);
  for (void* b : bufs) (void)hipFree(b);
  if (status != GB_OK) return status;
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? GB_ENOMEM : GB_EHIP, "gb_add_templates: %s", hipGetErrorString(e));
  return GB_OK;
}

extern "C" gb_status gb_noise_estimate(const gb_window* windows, int n_win, const double* d, double T, double* w,
                                       double* S, void* stream) {
  if (n_win < 0 || (n_win > 0 && (!windows || !d || !w)) || !(T > 0.0) || !std::isfinite(T))
    return fail(GB_EINVAL, "gb_noise_estimate: bad arguments");
  if (n_win == 0) return GB_OK;
  std::vector<NoiseWin> nw(n_win);
  for (int i = 0; i < n_win; ++i) {
    const gb_window& g = windows[i];
    if (g.W < 1 || g.W > kNoiseMaxW || (g.C != 2 && g.C != 3) || g.data_off < 0)
      return fail(GB_EINVAL, "gb_noise_estimate: window %d: W must be 1..%d, C 2 or 3, offset >= 0", i, kNoiseMaxW);
    nw[i].data_off = g.data_off;
    nw[i].W = g.W;
    nw[i].C = g.C;
  }
  hipStream_t st = (hipStream_t)stream;
  NoiseWin* d_nw = nullptr;
  hipError_t e = hipMalloc(&d_nw, sizeof(NoiseWin) * n_win);
  if (e == hipSuccess) e = hipMemcpyAsync(d_nw, nw.data(), sizeof(NoiseWin) * n_win, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_noise_median, dim3((unsigned)n_win, 3), dim3(1024), 0, st, d_nw, d, T, w, S);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(d_nw);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? GB_ENOMEM : GB_EHIP, "gb_noise_estimate: %s", hipGetErrorString(e));
  return GB_OK;
}

// ------------------------------------------------------------------------------- global noise estimate
namespace {

template <int NF>
void launch_ifft_a(const double* Y, double* Z, const double* tw, int64_t M1, hipStream_t st) {
  hipLaunchKernelGGL(k_ifft_a<NF>, dim3((unsigned)M1), dim3(NF / 8), 0, st, Y, Z, tw, M1);
}

constexpr int kIfftM1 = 2048;  // pass-B length of the four-step inverse DFT

}  // namespace

extern "C" gb_status gb_noise_global(const gb_window* windows, const int64_t* seg, int n_win, const double* d,
                                     double T, const gb_noise_global_config* cfg, double* w, double* S,
                                     double* welch, double* smooth, void* stream) {
  if (!cfg || !windows || !seg || !d || !w || n_win < 1 || n_win > 65535)
    return fail(GB_EINVAL, "gb_noise_global: null arguments or n_win outside 1..65535");
  const double dt = cfg->dt;
  if (!(T > 0.0) || !std::isfinite(T) || !(dt > 0.0) || !std::isfinite(dt))
    return fail(GB_EINVAL, "gb_noise_global: T and dt must be positive and finite");
  const int64_t M = (int64_t)std::llround(T / dt);
  if (M < (1 << 20) || M > (1 << 22) || (M & (M - 1)) || std::fabs((double)M * dt - T) > 1e-9 * T)
    return fail(GB_EINVAL, "gb_noise_global: T / dt must be a power of two in [2^20, 2^22]");
  const int L = cfg->nperseg;
  if (L != 8192 && L != 16384) return fail(GB_EINVAL, "gb_noise_global: nperseg must be 8192 or 16384");
  if (cfg->clip_width < 1 || cfg->clip_width > 64 || cfg->clip_stride < 1 || cfg->sg_short < 1 ||
      cfg->sg_long < 1 || !(cfg->f_switch >= 0.0) || cfg->reserved != 0)
    return fail(GB_EINVAL, "gb_noise_global: clip width 1..64, stride >= 1, filter lengths >= 1, f_switch >= 0");
  const int NF = L / 2;
  const int64_t M2 = M / kIfftM1;
  const int K = (int)(2 * M / L - 1);
  const int64_t pitch = NF + 1;
  // windows, segments, bands
  std::vector<SegWin> sw(n_win);
  int64_t band_lo[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, band_hi[3] = {0, 0, 0};
  int64_t max_cw = 0;
  for (int i = 0; i < n_win; ++i) {
    const gb_window& g = windows[i];
    const int64_t lo = seg[2 * i], hi = seg[2 * i + 1];
    if ((g.C != 2 && g.C != 3) || g.W < 1 || g.data_off < 0 || g.k0 < 0)
      return fail(GB_EINVAL, "gb_noise_global: window %d: C must be 2 or 3, W >= 1, offsets >= 0", i);
    if (!(lo < hi) || lo < g.k0 || hi > g.k0 + g.W || lo < 1 || hi > M / 2)
      return fail(GB_EINVAL, "gb_noise_global: window %d: segment [%lld, %lld) must lie inside the window and "
                  "inside [1, M/2)", i, (long long)lo, (long long)hi);
    sw[i] = SegWin{g.k0, g.data_off, lo, hi, g.W, g.C};
    max_cw = std::max(max_cw, (int64_t)g.C * g.W);
    for (int c = 0; c < g.C; ++c) {
      band_lo[c] = std::min(band_lo[c], lo);
      band_hi[c] = std::max(band_hi[c], hi);
    }
  }
  // the segments of one channel must not overlap (each bin has one owner)
  for (int c = 0; c < 3; ++c) {
    std::vector<std::pair<int64_t, int64_t>> r;
    for (const SegWin& x : sw)
      if (c < x.C) r.emplace_back(x.lo, x.hi);
    std::sort(r.begin(), r.end());
    for (size_t k = 1; k < r.size(); ++k)
      if (r[k].first < r[k - 1].second) return fail(GB_EINVAL, "gb_noise_global: overlapping segments in channel %d", c);
  }
  int h_lo[3] = {0, 0, 0}, h_n[3] = {0, 0, 0};
  const int wl_max = std::max(std::max(cfg->sg_short, cfg->sg_long), 3);
  for (int c = 0; c < 3; ++c) {
    if (band_hi[c] == 0) continue;
    const int64_t j_lo = (band_lo[c] * L + M - 1) / M, j_hi = ((band_hi[c] - 1) * L) / M;
    h_lo[c] = (int)j_lo;
    h_n[c] = (int)(j_hi - j_lo + 1);
    if (h_n[c] < wl_max) return fail(GB_EINVAL, "gb_noise_global: channel %d: the band holds %d Welch bins, fewer "
                                     "than the filter window %d", c, h_n[c], wl_max);
  }
  // Hann window and its sum of squares (periodic: w_n = 1/2 - 1/2 cos(2 pi n / L))
  std::vector<double> hann(L);
  double ssq = 0.0;
  for (int n = 0; n < L; ++n) {
    hann[n] = 0.5 - 0.5 * std::cos(2.0 * kPi * (double)n / (double)L);
    ssq += hann[n] * hann[n];
  }
  hipStream_t st = (hipStream_t)stream;
  double *Y = nullptr, *Z = nullptr, *x = nullptr, *Pseg = nullptr, *P = nullptr, *Pc = nullptr, *Sm = nullptr,
         *mm = nullptr, *dg = nullptr, *twA = nullptr, *twB = nullptr, *twW = nullptr, *d_hann = nullptr;
  SegWin* d_sw = nullptr;
  int *d_lo = nullptr, *d_n = nullptr;
  hipError_t e = hipSuccess;
  auto mal = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  mal((void**)&Y, sizeof(double) * 2 * M);
  mal((void**)&Z, sizeof(double) * 2 * M);
  mal((void**)&x, sizeof(double) * M);
  mal((void**)&Pseg, sizeof(double) * (size_t)K * pitch);
  for (double** q : {&P, &Pc, &Sm, &mm, &dg}) mal((void**)q, sizeof(double) * 3 * pitch);
  mal((void**)&twA, sizeof(double) * 2 * M2);
  mal((void**)&twB, sizeof(double) * 2 * kIfftM1);
  mal((void**)&twW, sizeof(double) * 2 * NF);
  mal((void**)&d_hann, sizeof(double) * L);
  mal((void**)&d_sw, sizeof(SegWin) * n_win);
  mal((void**)&d_lo, sizeof(int) * 3);
  mal((void**)&d_n, sizeof(int) * 3);
  if (e == hipSuccess) e = hipMemcpyAsync(d_hann, hann.data(), sizeof(double) * L, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sw, sw.data(), sizeof(SegWin) * n_win, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_lo, h_lo, sizeof(h_lo), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_n, h_n, sizeof(h_n), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_twiddle64, dim3((unsigned)((M2 + 255) / 256)), dim3(256), 0, st, twA, (int)M2);
    hipLaunchKernelGGL(k_twiddle64, dim3(kIfftM1 / 256), dim3(256), 0, st, twB, kIfftM1);
    hipLaunchKernelGGL(k_twiddle64, dim3((unsigned)(NF / 256)), dim3(256), 0, st, twW, NF);
    for (double* q : {P, Sm})
      hipLaunchKernelGGL(k_fill_zero, dim3(64), dim3(256), 0, st, q, (int64_t)3 * pitch);
    e = hipGetLastError();
  }
  for (int c = 0; c < 3 && e == hipSuccess; ++c) {
    if (h_n[c] == 0) continue;
    hipLaunchKernelGGL(k_fill_zero, dim3(1024), dim3(256), 0, st, Y, 2 * M);
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)n_win), dim3(256), 0, st, d_sw, d, c, M, Y);
    if (M2 == 512) launch_ifft_a<512>(Y, Z, twA, kIfftM1, st);
    else if (M2 == 1024) launch_ifft_a<1024>(Y, Z, twA, kIfftM1, st);
    else launch_ifft_a<2048>(Y, Z, twA, kIfftM1, st);
    hipLaunchKernelGGL(k_ifft_b<kIfftM1>, dim3((unsigned)M2), dim3(kIfftM1 / 8), 0, st, Z, x, twB, M2, 1.0 / T);
    if (NF == 8192)
      hipLaunchKernelGGL(k_welch_seg<8192>, dim3((unsigned)K), dim3(1024), 0, st, x, d_hann, twW, Pseg);
    else
      hipLaunchKernelGGL(k_welch_seg<4096>, dim3((unsigned)K), dim3(512), 0, st, x, d_hann, twW, Pseg);
    hipLaunchKernelGGL(k_welch_mean, dim3((unsigned)((pitch + 255) / 256)), dim3(256), 0, st, Pseg, K, (int)pitch,
                       2.0 * dt / ssq, P + c * pitch);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int nmax = std::max(h_n[0], std::max(h_n[1], h_n[2]));
    hipLaunchKernelGGL(k_median_clip, dim3(3), dim3(64), 0, st, P, Pc, pitch, d_lo, d_n, cfg->clip_width,
                       cfg->clip_stride);
    hipLaunchKernelGGL(k_savgol, dim3((unsigned)((nmax + 255) / 256), 3), dim3(256), 0, st, Pc, Sm, pitch, d_lo, d_n,
                       L, dt, cfg->f_switch, cfg->sg_short, cfg->sg_long);
    hipLaunchKernelGGL(k_spline_m, dim3(3), dim3(64), 0, st, Sm, mm, dg, pitch, d_lo, d_n);
    hipLaunchKernelGGL(k_spline_eval, dim3((unsigned)((max_cw + 255) / 256), (unsigned)n_win), dim3(256), 0, st, d_sw,
                       Sm, mm, pitch, d_lo, d_n, (int64_t)(M / L), T, w, S);
    e = hipGetLastError();
  }
  if (e == hipSuccess && welch) e = hipMemcpyAsync(welch, P, sizeof(double) * 3 * pitch, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && smooth) e = hipMemcpyAsync(smooth, Sm, sizeof(double) * 3 * pitch, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (void* q : {(void*)Y, (void*)Z, (void*)x, (void*)Pseg, (void*)P, (void*)Pc, (void*)Sm, (void*)mm, (void*)dg,
                  (void*)twA, (void*)twB, (void*)twW, (void*)d_hann, (void*)d_sw, (void*)d_lo, (void*)d_n})
    (void)hipFree(q);
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? GB_ENOMEM : GB_EHIP, "gb_noise_global: %s", hipGetErrorString(e));
  return GB_OK;
}

// ------------------------------------------------------------------------------- allocation-free noise estimate
// gb_noise_estimate_noalloc stages its window list in this file-scope device array instead of
// a per-call allocation.  Every GPU the library runs on holds its own copy until the process
// ends.  In host code the array's name is only a stand-in: host code reaches the memory through
// the per-device address that hipGetSymbolAddress returns (noise_scratch below).
constexpr int kNoiseNoallocMaxWin = 16384;  // 16 B per window: 256 KiB per device
static __device__ __align__(256) NoiseWin scratch[kNoiseNoallocMaxWin];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static NoiseWin* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's staging array, looked up once per device (with that
// device current) and kept.
static gb_status noise_scratch(NoiseWin** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(GB_EUNSUPPORTED, "gb_noise_estimate_noalloc: device %d >= %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GB_EHIP, "gb_noise_estimate_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<NoiseWin*>(p);
  }
  *out = g_scratch_ptr[dev];
  return GB_OK;
}

extern "C" gb_status gb_noise_estimate_noalloc(const gb_window* windows, int n_win, const double* d, double T,
                                               double* w, double* S, void* stream) {
  if (n_win < 0 || (n_win > 0 && (!windows || !d || !w)) || !(T > 0.0) || !std::isfinite(T))
    return fail(GB_EINVAL, "gb_noise_estimate_noalloc: bad arguments");
  if (n_win > kNoiseNoallocMaxWin)
    return fail(GB_EINVAL, "gb_noise_estimate_noalloc: %d windows exceed the staging limit of %d", n_win,
                kNoiseNoallocMaxWin);
  if (n_win == 0) return GB_OK;
  for (int i = 0; i < n_win; ++i) {
    const gb_window& g = windows[i];
    if (g.W < 1 || g.W > kNoiseMaxW || (g.C != 2 && g.C != 3) || g.data_off < 0)
      return fail(GB_EINVAL, "gb_noise_estimate_noalloc: window %d: W must be 1..%d, C 2 or 3, offset >= 0", i,
                  kNoiseMaxW);
  }
  NoiseWin* stage = nullptr;
  gb_status s = noise_scratch(&stage);
  if (s != GB_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  // the window list goes to the device in chunks through a small host buffer on the stack; the
  // stream is drained after each copy, so the buffer can be refilled
  constexpr int kChunk = 256;
  NoiseWin host[kChunk];
  for (int i0 = 0; i0 < n_win; i0 += kChunk) {
    const int n = std::min(kChunk, n_win - i0);
    for (int i = 0; i < n; ++i) {
      host[i].data_off = windows[i0 + i].data_off;
      host[i].W = windows[i0 + i].W;
      host[i].C = windows[i0 + i].C;
    }
    HIPCHK(hipMemcpyAsync(stage + i0, host, sizeof(NoiseWin) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  hipLaunchKernelGGL(k_noise_median, dim3((unsigned)n_win, 3), dim3(1024), 0, st, stage, d, T, w, S);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  return GB_OK;
}

extern "C" gb_status gb_de_trial(int n_win, int pop, const double* lo, const double* hi, const double* x,
                                 const double* u_idx, const double* u_cross, const double* u_j, const double* F,
                                 const int32_t* base, double cr, double amp, double* trial_x, double* trial_theta,
                                 void* stream) {
  if (n_win < 0 || pop < 4 || !(cr >= 0.0 && cr <= 1.0)) return fail(GB_EINVAL, "gb_de_trial: bad sizes or rate");
  if (n_win == 0) return GB_OK;
  if (!lo || !hi || !x || !u_idx || !u_cross || !u_j || !F || !trial_x || !trial_theta)
    return fail(GB_EINVAL, "gb_de_trial: null array");
  const int64_t n = (int64_t)n_win * pop;
  if ((n + 255) / 256 > 0x7fffffff) return fail(GB_EINVAL, "gb_de_trial: population too large");
  hipLaunchKernelGGL(k_de_trial, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n_win, pop, lo,
                     hi, x, u_idx, u_cross, u_j, F, base, cr, amp, trial_x, trial_theta);
  HIPCHK(hipGetLastError());
  return GB_OK;
}

extern "C" gb_status gb_de_select(int n_win, int pop, const double* comps, double* x, double* s,
                                  const double* trial_x, double* best, int32_t* best_idx, void* stream) {
  if (n_win < 0 || pop < 1) return fail(GB_EINVAL, "gb_de_select: bad sizes");
  if (n_win == 0) return GB_OK;
  if (!comps || !x || !s || !trial_x || !best) return fail(GB_EINVAL, "gb_de_select: null array");
  hipLaunchKernelGGL(k_de_select, dim3((unsigned)n_win), dim3(256), 0, (hipStream_t)stream, pop, comps, x, s, trial_x,
                     best, best_idx);
  HIPCHK(hipGetLastError());
  return GB_OK;
}

extern "C" gb_status gb_kde_logpdf(const double* pts, const double* wts, int n_sets, int n_pairs, int64_t m,
                                   const double* chol, const double* x, int64_t q, double* out, void* stream) {
  if (n_sets < 0 || n_sets > 65535 || n_pairs < 1 || m < 0 || q < 0) return fail(GB_EINVAL, "gb_kde_logpdf: bad sizes");
  if (q == 0 || n_sets == 0) return GB_OK;
  if (!pts || !wts || !chol || !x || !out) return fail(GB_EINVAL, "gb_kde_logpdf: null array");
  if ((q + 255) / 256 > 0x7fffffff) return fail(GB_EINVAL, "gb_kde_logpdf: too many queries");
  hipLaunchKernelGGL(k_kde_logpdf, dim3((unsigned)((q + 255) / 256), (unsigned)n_sets), dim3(256), 0,
                     (hipStream_t)stream, pts, wts, n_pairs, m, chol, x, q, out);
  HIPCHK(hipGetLastError());
  return GB_OK;
}

extern "C" gb_status gb_select_variant(gb_ctx* c, gb_precision prec, int mode, int N, int C, int lpc, int wpb,
                                       int occ) {
  if (!c) return fail(GB_EINVAL, "gb_select_variant: null context");
  if ((prec != GB_FP64 && prec != GB_MIXED) || (mode != MODE_LOGLIK && mode != MODE_GRAD) || !pow2_in_range(N) ||
      (C != 2 && C != 3))
    return fail(GB_EINVAL, "gb_select_variant: bad precision, mode, N or C");
  const VariantList& l = all_variants();
  for (int i = 0; i < l.n; ++i) {
    const Variant& v = l.v[i];
    if (v.prec == (int)prec && v.mode == mode && v.N == N && v.C == C && v.LPC == lpc && v.WPB == wpb && v.occ == occ) {
      c->choice[prec][n_index(N)][C - 2][mode] = &v;
      return GB_OK;
    }
  }
  return fail(GB_EINVAL, "gb_select_variant: no compiled variant k_batch<%s,%d,%d,%d,%d,%d,%d>",
              prec == GB_FP64 ? "double" : "float", N, lpc, C, wpb, mode, occ);
}

// Mean time of `reps` launches of variant v over a.tiles (after one warm-up launch) on the null
// stream, with the persistent grid a plan would give it.
static hipError_t time_variant(const gb_ctx* c, const Variant& v, BatchArgs& a, int reps, hipEvent_t e0,
                               hipEvent_t e1, float* ms) {
  int nb = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, v.fn, v.WPB * 64, lds_bytes(v));
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)std::max(1, std::min(a.n_tiles, std::max(1, nb) * c->n_cu)));
  if (launch(&v, grid, a, 0) != GB_OK) return hipErrorLaunchFailure;  // warm-up
  e = hipEventRecord(e0, 0);
  for (int r = 0; r < reps && e == hipSuccess; ++r)
    if (launch(&v, grid, a, 0) != GB_OK) e = hipErrorLaunchFailure;
  if (e == hipSuccess) e = hipEventRecord(e1, 0);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  *ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  *ms /= (float)reps;
  return e;
}

// One line of a tuning report.
static std::string tune_line(int prec, int mode, int N, int C, const Variant& v, float ms, int64_t n, int tried) {
  char line[256];
  std::snprintf(line, sizeof line,
                "%s %s N=%d C=%d: lanes/template=%d min waves/SIMD=%d %.4f ms / %lld (%d variants) "
                "kernel=k_batch<%s,%d,%d,%d,%d,%d,%d>\n",
                prec == GB_FP64 ? "fp64 " : "mixed", mode == MODE_GRAD ? "grad  " : "loglik", N, C, v.LPC, v.occ,
                ms, (long long)n, tried, prec == GB_FP64 ? "double" : "float", N, v.LPC, C, v.WPB, mode, v.occ);
  return line;
}

// Time every compiled variant of each (precision, N, C, mode) family on synthetic candidates
// (one window of W = N bins at 8 mHz, 16384 candidates) and keep the fastest in the context.
extern "C" gb_status gb_autotune(gb_ctx* c, int reps, char* report, size_t report_len) {
  if (!c) return fail(GB_EINVAL, "gb_autotune: null context");
  if (reps < 1) reps = 1;
  const int B = 16384;
  std::string rep;
  // synthetic candidates (deterministic linear congruential draws), data and weights
  std::vector<double> th(8 * (size_t)B);
  uint64_t st = 0x9E3779B97F4A7C15ull;
  auto uni = [&]() {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(st >> 11) * (1.0 / 9007199254740992.0);
  };
  const double f = 8e-3, T = c->cfg.T;
  for (int i = 0; i < B; ++i) {
    double* t = &th[8 * (size_t)i];
    t[0] = f + (uni() - 0.5) * 64.0 / T;
    t[1] = 1e-16;
    t[2] = std::asin(2.0 * uni() - 1.0);
    t[3] = (2.0 * uni() - 1.0) * kPi;
    t[4] = 1e-22;
    t[5] = std::acos(2.0 * uni() - 1.0);
    t[6] = uni() * kPi;
    t[7] = uni() * 2.0 * kPi;
  }
  double *d_th = nullptr, *d_d = nullptr, *d_w = nullptr, *d_l = nullptr, *d_g = nullptr;
  DevWin* d_win = nullptr;
  Tile* d_tiles = nullptr;
  unsigned* d_ctr = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int Wmax = 1024, Cmax = 3;
  hipError_t e = hipMalloc(&d_th, sizeof(double) * th.size());
  if (e == hipSuccess) e = hipMemcpy(d_th, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&d_d, sizeof(double) * 2 * Wmax * Cmax);
  if (e == hipSuccess) e = hipMemset(d_d, 0, sizeof(double) * 2 * Wmax * Cmax);
  std::vector<double> wv((size_t)Wmax * Cmax, 1e40);
  if (e == hipSuccess) e = hipMalloc(&d_w, sizeof(double) * wv.size());
  if (e == hipSuccess) e = hipMemcpy(d_w, wv.data(), sizeof(double) * wv.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&d_l, sizeof(double) * B);
  if (e == hipSuccess) e = hipMalloc(&d_g, sizeof(double) * 8 * B);
  if (e == hipSuccess) e = hipMalloc(&d_win, sizeof(DevWin));
  if (e == hipSuccess) e = hipMalloc(&d_tiles, sizeof(Tile) * B);
  if (e == hipSuccess) e = hipMalloc(&d_ctr, 2 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(d_ctr, 0, 2 * sizeof(unsigned));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const VariantList& all = all_variants();
  for (int prec = 0; prec < 2 && e == hipSuccess; ++prec)
    for (int ni = 0; ni < 5 && e == hipSuccess; ++ni)
      for (int C = 2; C <= 3 && e == hipSuccess; ++C)
        for (int mode = MODE_LOGLIK; mode <= MODE_GRAD && e == hipSuccess; ++mode) {
          const int N = 64 << ni;
          DevWin w;
          std::memset(&w, 0, sizeof w);
          w.k0 = (int64_t)std::floor(f * T) - N / 2;
          w.W = N;
          w.N = N;
          w.C = C;
          w.prec = prec;
          w.n_cand = B;
          w.dd = 0.0;
          e = hipMemcpy(d_win, &w, sizeof w, hipMemcpyHostToDevice);
          const Variant* best = nullptr;
          float best_ms = 0.0f;
          int tried = 0;
          for (int i = 0; i < all.n && e == hipSuccess; ++i) {
            const Variant& v = all.v[i];
            if (v.prec != prec || v.N != N || v.C != C || v.mode != mode) continue;
            const int tsz = v.WPB * 64 / v.LPC * kTileIters;
            std::vector<Tile> tiles;
            for (int c0 = 0; c0 < B; c0 += tsz) tiles.push_back(Tile{0, std::min(tsz, B - c0), c0});
            e = hipMemcpy(d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice);
            if (e != hipSuccess) break;
            BatchArgs a = base_args(c, N, prec);
            a.wins = d_win;
            a.tiles = d_tiles;
            a.n_tiles = (int)tiles.size();
            a.ctr = d_ctr;
            a.d = d_d;
            a.w = d_w;
            a.theta = d_th;
            a.logL = d_l;
            a.grad = d_g;
            float ms = 0.0f;
            e = time_variant(c, v, a, reps, e0, e1, &ms);
            if (e != hipSuccess) break;
            ++tried;
            if (!best || ms < best_ms) {
              best = &v;
              best_ms = ms;
            }
          }
          if (best) {
            c->choice[prec][ni][C - 2][mode] = best;
            rep += tune_line(prec, mode, N, C, *best, best_ms, B, tried);
          }
        }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void* p : {(void*)d_th, (void*)d_d, (void*)d_w, (void*)d_l, (void*)d_g, (void*)d_win, (void*)d_tiles, (void*)d_ctr})
    (void)hipFree(p);
  if (e != hipSuccess) return fail(GB_EHIP, "gb_autotune: %s", hipGetErrorString(e));
  if (report && report_len) std::snprintf(report, report_len, "%s", rep.c_str());
  return GB_OK;
}

static const int64_t kTuneMaxCand = 1 << 19;  // candidates timed per (N, C) group of gb_autotune_windows

// Time every compiled variant on the (N, C) groups of the given windows, in both precisions, with
// their own data, weights and candidates; keep the fastest of each (precision, N, C, mode) family
// in the context.  Each group is timed over its windows' candidates, in window order, up to
// kTuneMaxCand of them (whole tiles).
extern "C" gb_status gb_autotune_windows(gb_ctx* c, const gb_window* windows, int n_win, const double* d,
                                         const double* w, const double* theta, int reps, char* report,
                                         size_t report_len) {
  if (!c) return fail(GB_EINVAL, "gb_autotune_windows: null context");
  if (n_win < 0 || (n_win > 0 && !windows)) return fail(GB_EINVAL, "gb_autotune_windows: bad window array");
  if (n_win > 0 && (!d || !w || !theta)) return fail(GB_EINVAL, "gb_autotune_windows: null array");
  if (reps < 1) reps = 1;
  std::string rep;
  const VariantList& all = all_variants();
  double *d_l = nullptr, *d_g = nullptr;
  Tile* d_tiles = nullptr;
  size_t tile_cap = 0;
  unsigned* d_ctr = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&d_ctr, 2 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(d_ctr, 0, 2 * sizeof(unsigned));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  gb_status st = GB_OK;
  for (int prec = GB_FP64; prec <= GB_MIXED && e == hipSuccess && st == GB_OK && n_win > 0; ++prec) {
    gb_plan* p = nullptr;
    st = gb_plan_create(c, windows, n_win, (gb_precision)prec, &p);
    if (st != GB_OK) break;
    if (!d_l && p->rows > 0) {
      e = hipMalloc(&d_l, sizeof(double) * p->rows);
      if (e == hipSuccess) e = hipMalloc(&d_g, sizeof(double) * 8 * p->rows);
    }
    // (N, C) groups of the windows that hold candidates, in window order
    std::vector<std::vector<int>> groups(5 * 2);
    for (int i = 0; i < n_win; ++i)
      if (p->wins[i].n_cand > 0) groups[n_index(p->wins[i].N) * 2 + p->wins[i].C - 2].push_back(i);
    for (int gi = 0; gi < 10 && e == hipSuccess; ++gi) {
      if (groups[gi].empty()) continue;
      const int N = 64 << (gi / 2), C = 2 + gi % 2;
      for (int mode = MODE_LOGLIK; mode <= MODE_GRAD && e == hipSuccess; ++mode) {
        const Variant* best = nullptr;
        float best_ms = 0.0f;
        int64_t best_n = 0;
        int tried = 0;
        for (int i = 0; i < all.n && e == hipSuccess; ++i) {
          const Variant& v = all.v[i];
          if (v.prec != prec || v.N != N || v.C != C || v.mode != mode) continue;
          const int tsz = v.WPB * 64 / v.LPC * kTileIters;
          std::vector<Tile> tiles;
          int64_t n = 0;
          for (int wi : groups[gi]) {
            for (int64_t c0 = 0; c0 < p->wins[wi].n_cand && n < kTuneMaxCand; c0 += tsz) {
              const int32_t k = (int32_t)std::min<int64_t>(tsz, p->wins[wi].n_cand - c0);
              tiles.push_back(Tile{wi, k, c0});
              n += k;
            }
            if (n >= kTuneMaxCand) break;
          }
          if (tiles.size() > tile_cap) {
            (void)hipFree(d_tiles);
            d_tiles = nullptr;
            tile_cap = tiles.size();
            e = hipMalloc(&d_tiles, sizeof(Tile) * tile_cap);
          }
          if (e == hipSuccess)
            e = hipMemcpy(d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice);
          if (e != hipSuccess) break;
          BatchArgs a = base_args(c, N, prec);
          a.wins = p->d_wins;
          a.tiles = d_tiles;
          a.n_tiles = (int)tiles.size();
          a.ctr = d_ctr;
          a.d = d;
          a.w = w;
          a.theta = theta;
          a.logL = d_l;
          a.grad = d_g;
          float ms = 0.0f;
          e = time_variant(c, v, a, reps, e0, e1, &ms);
          if (e != hipSuccess) break;
          ++tried;
          if (!best || ms < best_ms) {
            best = &v;
            best_ms = ms;
            best_n = n;
          }
        }
        if (best && e == hipSuccess) {
          c->choice[prec][gi / 2][C - 2][mode] = best;
          rep += tune_line(prec, mode, N, C, *best, best_ms, best_n, tried);
        }
      }
    }
    gb_plan_destroy(p);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void* q : {(void*)d_l, (void*)d_g, (void*)d_tiles, (void*)d_ctr}) (void)hipFree(q);
  if (st != GB_OK) return st;
  if (e != hipSuccess) return fail(GB_EHIP, "gb_autotune_windows: %s", hipGetErrorString(e));
  if (report && report_len) std::snprintf(report, report_len, "%s", rep.c_str());
  return GB_OK;
}
