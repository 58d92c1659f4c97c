/*
 * gbx -- batched Galactic-binary log-likelihood on AMD MI355X (gfx950).
 *
 * C ABI of the hot path of Strub et al., arXiv:2307.03763: the log-likelihood of many
 * eight-parameter Galactic-binary candidates against LISA TDI data in narrow frequency
 * windows, its gradient, and the independent-proposal Metropolis-Hastings step that
 * consumes it.
 *
 * Conventions shared by every call
 *  - theta rows are 8 doubles (f0 [Hz], fdot [Hz/s], beta, lambda [rad], amplitude,
 *    iota, psi, phi0 [rad]) -- the parameter set of Sec. III.
 *  - Frequency bins are absolute: bin k sits at f = k / T.  Data and weights of a window
 *    are stored channel-major, [C][W]; channels are A, E (C = 2) or A, E, T (C = 3), the
 *    combinations of Sec. II.  Complex values are two doubles (re, im).
 *  - Unless stated otherwise every array argument is a DEVICE pointer owned by the caller
 *    (for example a torch tensor); gb_config and gb_window arrays are HOST memory.
 *  - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL = the null
 *    stream).  The hot calls (gb_waveform, gb_loglik, gb_loglik_grad, gb_mh_step,
 *    gb_window_prepare) allocate nothing, copy nothing between host and device and never
 *    synchronise, so they may be captured in a HIP graph.
 *  - Return status covers argument validation and launch errors.  Faults during execution
 *    surface at the caller's next synchronisation.  gb_last_error() returns a message for
 *    the last non-OK status of the calling thread.
 *  - Candidates whose theta is not finite, whose amplitude is negative, or whose f0 is not
 *    in (0, 4e15 / T) get NaN outputs; the rest of the batch is unaffected.
 *  - A plan may be used by one stream at a time (its work queues are per plan).
 */
#ifndef GBX_H
#define GBX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GB_OK = 0,
  GB_EINVAL = -1,        /* bad argument (message in gb_last_error) */
  GB_EHIP = -2,          /* a HIP runtime call failed */
  GB_ENOMEM = -3,        /* device allocation failed (set-up calls only) */
  GB_EUNSUPPORTED = -4   /* no kernel variant for the requested shape */
} gb_status;

typedef enum {
  GB_FP64 = 0,           /* every step in FP64 */
  GB_MIXED = 1,          /* phase (in cycles) and all accumulations in FP64; response,
                            slow series and FFT in FP32 with hardware sin/cos */
  GB_PER_WINDOW = 2      /* plan only: take each window's `precision` field */
} gb_precision;

/* Observation and constellation constants (set-up; host memory). */
typedef struct {
  double T;              /* observation time, s; bin width 1/T */
  double orbit_period;   /* period of the guiding centre, s (sidereal year) */
  double arm_length;     /* L, m (half transfer frequency 1/(4 pi L) = 9.55 mHz for 2.5e9 m, Sec. II) */
  double au;             /* radius of the guiding-centre orbit, m */
  int32_t tdi_generation;/* 1 (or 0): first-generation equal-arm Michelson X, Y, Z, from which
                            the A, E, T of Sec. II are formed; 2: second generation, which for
                            equal arms is the first-generation combination minus its copy
                            delayed by four arm lengths (a factor 1 - D^4, D = e^{-2 pi i f L/c}) */
  int32_t reserved;      /* must be 0 */
} gb_config;

/* One frequency window: the padded segment of Sec. III B over which the scalar product is
 * summed (Sec. III D).  Host memory. */
typedef struct {
  int64_t k0;            /* absolute index of the first bin */
  int32_t W;             /* number of bins, >= 1 */
  int32_t N;             /* slow-series samples per template: power of two in [64, 1024] */
  int32_t C;             /* channels, 2 (A, E) or 3 (A, E, T); 0 in gb_plan_create: the rule of
                            Sec. II, resolved from the window's centre (see gb_channels) */
  int32_t precision;     /* gb_precision of this window when the plan is GB_PER_WINDOW */
  int64_t data_off;      /* element offset of the window's [C][W] block in d and in w */
  int64_t cand_off;      /* first candidate row of this window in theta and the outputs */
  int64_t n_cand;        /* number of candidates (rows) of this window, >= 0 */
} gb_window;

typedef struct gb_ctx gb_ctx;     /* device tables for one gb_config (orbit, twiddles) */
typedef struct gb_plan gb_plan;   /* work lists and launch shapes for a set of windows */

/* Create a context on the current HIP device: builds the per-sample orbit tables and the
 * DFT twiddles for N = 64..1024 (device memory owned by the context).  Every template,
 * likelihood and gradient of the context uses its TDI generation.  Synchronous.
 * GB_EINVAL for non-positive constants or a generation other than 0, 1, 2.  *ctx is NULL on
 * failure. */
gb_status gb_create(const gb_config* cfg, gb_ctx** ctx);
void gb_destroy(gb_ctx* ctx);

/* Message of the calling thread's last non-OK status ("" if none). */
const char* gb_last_error(void);

/* Templates of B sources (Sec. III parameters; the TDI response of Sec. II channels).
 * h_out: complex128 [B][C][N]; element i of channel c is the template on bin
 * first_bin[b] + i; first_bin: int64 [B], = floor(f0 T) - N/2.  The template is
 * (T / 2N) * DFT_N of the carrier-free slow series sampled at t_m = m T / N.
 * GB_EINVAL: B < 0, N not a power of two in [64, 1024], C not 2 or 3, null pointers. */
gb_status gb_waveform(gb_ctx* ctx, const double* theta, int64_t B, int N, int C,
                      gb_precision precision, double* h_out, int64_t* first_bin, void* stream);

/* The channel count the rule of Sec. II gives a window: the T channel is used at and above half
 * the transfer frequency, f >= f* / 2 = c / (4 pi L) (9.55 mHz for L = 2.5e9 m, the context's arm
 * length), decided at the window's centre f = (k0 + W/2) / T; *C = 3 there and 2 below.  Callers
 * that pass C = 0 to gb_plan_create lay out their data with this count.  GB_EINVAL: null
 * pointers, W < 1. */
gb_status gb_channels(const gb_ctx* ctx, int64_t k0, int32_t W, int32_t* C);

/* Numerical orbits (eccentric or simulated): the paper leaves the orbit model to its references,
 * and the context's default is the rigid equal-arm triangle.  pos: host double
 * [n_pts][3 spacecraft][3 ecliptic coordinates] in metres at the times t_j = t0 + j dt, the
 * grid covering the observation (t0 <= 0, t0 + (n_pts - 1) dt >= T); positions between nodes
 * come from the cubic through four neighbouring nodes.  Every arm then has its own light time
 * and unit vector at each sample (the centroid is the guiding centre), each link takes its own
 * arm in the transfer function, and the TDI one delay per arm:
 *   X = (1 - D12^2)(y13 + D31 y31) - (1 - D31^2)(y12 + D12 y21), Y and Z cyclically,
 * times (1 - D31^2 D12^2) for the second generation (and cyclically), with the link phasors
 * taken at the sample time.  Applies to gb_waveform, gb_loglik, gb_loglik_grad (mixed
 * precision, as on the analytic orbits), gb_mh_step, gb_fisher and gb_add_templates of this
 * context from the next call on, plans already built included (they read the context's tables
 * and pick the kernels of this model at launch); not to calls in flight or already captured in
 * a graph.  pos = NULL with n_pts = 0 returns to the analytic orbits.  Synchronous; allocates a temporary device copy.  GB_EINVAL:
 * n_pts outside [4, 2^24], dt <= 0, a grid that does not cover [0, T], positions not finite, two
 * spacecraft at one point. */
gb_status gb_set_orbit(gb_ctx* ctx, const double* pos, int32_t n_pts, double t0, double dt);

/* Build a plan for `n_win` windows (host array, copied): validates every window, groups the
 * windows by (N, C, precision), splits their candidates into tiles ordered by cost and
 * uploads the work lists (device memory owned by the plan).  Also reserves the scratch of
 * gb_mh_step's chain: per window 2P doubles (P = smallest power of two >= n_cand) and
 * K (n_cand + 1) int32 (2^K > n_cand), about 90 bytes per candidate.  Synchronous;
 * allocates.  GB_EINVAL on a bad window (message names it); GB_ENOMEM. */
gb_status gb_plan_create(gb_ctx* ctx, const gb_window* windows, int n_win,
                         gb_precision precision, gb_plan** plan);
void gb_plan_destroy(gb_plan* plan);

/* Sizes a plan's calls read and write (host outputs; any may be NULL): rows = the largest
 * cand_off + n_cand (the length of theta's first axis and of the per-candidate outputs),
 * n_win = the number of windows (length of gb_mh_step's n_accept), data_len = the largest
 * data_off + C W (elements of d and w the plan reads).  For callers that check their arrays
 * before a call: the library cannot, as it receives raw pointers.  GB_EINVAL: null plan. */
gb_status gb_plan_info(const gb_plan* plan, int64_t* rows, int* n_win, int64_t* data_len);

/* <d|d> of every window (sum over channels and bins of w |d|^2), kept in the plan.  Must be
 * called after the data or weights change and before gb_loglik / gb_loglik_grad /
 * gb_mh_step, which reject other d, w pointers than the prepared ones.
 * d: complex128, w: float64 (w = 4 / (T S), the discretised weight of the scalar product of
 * Sec. II), both indexed by gb_window.data_off. */
gb_status gb_window_prepare(gb_plan* plan, const double* d, const double* w, void* stream);

/* logL = -1/2 sum_c sum_{k in window} w_k |d_k - h_k|^2 of every candidate
 * (Sec. II log-likelihood and scalar product; Sec. III D window).  theta: [rows][8] where
 * window i owns rows cand_off .. cand_off + n_cand - 1.  logL: [rows].  comps (may be NULL):
 * [rows][2] = <d|h>, <h|h>, from which rho = <d|h>/sqrt<h|h> and A_max = A <d|h>/<h|h>
 * (Sec. III SNR and amplitude equations).  Rows that no window owns are not written. */
gb_status gb_loglik(gb_plan* plan, const double* d, const double* w, const double* theta,
                    double* logL, double* comps, void* stream);

/* logL and its gradient grad: [rows][8], d logL / d theta in the order of theta (the
 * carrier bin floor(f0 T) held fixed): the derivative of the log-likelihood of Sec. II.
 * Hand-written adjoint: inverse DFT of the weighted residual, then the slow-series
 * derivative contracted with it by reverse mode.  Windows must be GB_MIXED: the FP64
 * gradient returns GB_EUNSUPPORTED (switched off in this version). */
gb_status gb_loglik_grad(gb_plan* plan, const double* d, const double* w, const double* theta,
                         double* logL, double* grad, void* stream);

/* One stage of Algorithm 4 for every window of the plan (one window = one source): the
 * logL of its n_cand proposals in parallel, then the independent-proposal chain
 * (acceptance equation of Sec. III G, with temperature T):
 *   start at proposal 0; for i = 1 .. n-1 accept with probability
 *   min(1, [L_i / L_c * g_c / g_i]^(1/T)), evaluated as  pi_c < pi_i - T ln u_i  with
 *   pi = logL - log_g (u_i = 0 always accepts; NaN logL never accepted).
 * log_g, u: [rows] (proposal log-density and uniforms in [0, 1)); outputs logL: [rows],
 * chain: int32 [rows] (index within the window of the state after each step, chain[0] = 0),
 * n_accept: int64 [n_win].  The chain is resolved in logarithmic depth, one workgroup per
 * window (next accepted proposal of every state from a max-tree of pi_i - T ln u_i, then
 * binary lifting), with the same comparisons as the step-by-step loop; it uses the plan's
 * chain scratch, so calls on one plan must not overlap.
 * GB_EINVAL: temperature <= 0 or not finite. */
gb_status gb_mh_step(gb_plan* plan, const double* d, const double* w, const double* theta,
                     const double* log_g, const double* u, double temperature,
                     double* logL, int32_t* chain, int64_t* n_accept, void* stream);

/* Choose the launch shape (lanes per template, waves per workgroup) of every (N, C,
 * precision) group by timing the compiled variants on synthetic candidates; the choice is
 * kept in the context and used by plans created afterwards.  Synchronous; allocates.
 * `report` (host, may be NULL) receives a text summary of at most report_len bytes. */
gb_status gb_autotune(gb_ctx* ctx, int reps, char* report, size_t report_len);

/* As gb_autotune, but timed on real work: the windows' (N, C) groups, in both precisions, with
 * the data d, weights w and candidates theta laid out as for gb_loglik (d, w, theta: device,
 * covering every window's data_off + C W bins and cand_off + n_cand rows; windows: host [n_win],
 * their precision field ignored, C = 0 resolved by the rule of Sec. II).  Each group is timed
 * over its windows' candidates in window order, up to 2^19 of them.  Families that no window
 * exercises keep their previous choice.  The choice is kept in the context and used by plans
 * created afterwards (existing plans keep theirs).  Synchronous on the null stream; allocates;
 * the outputs of the timed launches go to scratch of its own.  `report` as in gb_autotune (the
 * count after "ms /" is the candidates timed).  GB_EINVAL: bad window (as gb_plan_create) or
 * null array. */
gb_status gb_autotune_windows(gb_ctx* ctx, const gb_window* windows, int n_win, const double* d,
                              const double* w, const double* theta, int reps, char* report,
                              size_t report_len);

/* Set the launch shape of one (precision, mode, N, C) group by hand, as gb_autotune would:
 * for repeating a tuned configuration exactly (for example in a profiling run).  mode:
 * 1 = likelihood, 2 = gradient.  The shape must be one of the compiled variants (the
 * autotuner's report names them as k_batch<R,N,lanes,C,waves,mode,min waves per SIMD>).
 * Affects plans created afterwards.  GB_EINVAL: no such compiled variant. */
gb_status gb_select_variant(gb_ctx* ctx, gb_precision precision, int mode, int N, int C,
                            int lanes_per_template, int waves_per_block, int min_waves_per_simd);

/* Fisher information matrix of n sources, F_ij = <d_i h | d_j h> at theta (Sec. III G FIM
 * equation; the derivatives of the template, as the paper's reading of its garbled
 * "d_i p(d|theta)"), in Table I coordinates u (sin beta, log10 A and cos iota in place of
 * beta, A, iota), by second-order forward differences
 *   d_i h = (-3 h(u) + 4 h(u + e_i) - h(u + 2 e_i)) / (2 e_i)
 * with per-source steps e (the paper takes 1e-9 of the prior widths; e_i = 0 leaves row and
 * column i zero).  The templates are FP64 (gb_waveform) and the scalar product is summed over
 * the C channels and the bins of the source's window with weights w, as in gb_loglik.
 * theta, steps: device [n][8]; windows: host [n] (k0, W, N, C and data_off are used; one
 * window per source); w: device, indexed by data_off; F: device [n][8][8].  Synchronous;
 * allocates 17 templates of C x N per source of the largest (N, C) group.  GB_EINVAL on a
 * bad window. */
gb_status gb_fisher(gb_ctx* ctx, const double* theta, const double* steps, int n, const gb_window* windows,
                    const double* w, double* F, void* stream);

/* d_out = d_in + sign * (sum of the templates of the listed sources, each placed in its own
 * window): the residuals of the search (Algorithm 2: data minus the signals found so far) and
 * of the posterior stage.  FP64 templates at the window's N and C (gb_waveform); bins outside the
 * window are dropped; within a window the sources are added in their listed order, so the
 * result is deterministic.  theta: device [n_src][8]; src_win: HOST int32 [n_src], the window
 * (index into windows) of each source; windows: host [n_win] (k0, W, N, C and data_off are
 * used); d_in, d_out: device complex128 indexed by data_off, d_out may equal d_in; every
 * window's block of d_out is written (a copy of d_in where the window has no source).
 * Synchronous; allocates the templates.  GB_EINVAL on a bad window or window index. */
gb_status gb_add_templates(gb_ctx* ctx, const gb_window* windows, int n_win, const double* theta,
                           const int32_t* src_win, int n_src, double sign, const double* d_in, double* d_out,
                           void* stream);

/* Local noise estimate of every window and channel (Sec. III, noise within a frequency
 * segment): S = the median over the window's W bins of the one-sided periodogram 2 |d_k|^2 / T
 * (the paper's 2 |A|^2 / (N f_sample) for DFT values A, written for continuous-transform data
 * d = dt A), and the scalar-product weights w_k = 4 / (T S), constant along the channel.  The
 * median of an even count is the mean of the two middle values.  windows: host [n_win] (W,
 * C and data_off are used; W at most 4096); d: device complex128 indexed by data_off (the
 * residual the estimate follows); w: device float64, each window's C x W block overwritten;
 * S: device [n_win][3] (channel levels; entries of absent channels untouched) or NULL.  A
 * window whose median is 0 gets infinite weights.  Synchronous; allocates the window list.
 * GB_EINVAL on a bad window, T <= 0 or null arrays. */
gb_status gb_noise_estimate(const gb_window* windows, int n_win, const double* d, double T, double* w, double* S,
                            void* stream);

/* Settings of the global noise estimate (host memory); the values of Sec. III F in brackets. */
typedef struct {
  double dt;             /* sampling interval of the data's time series, s; M = T / dt samples,
                            a power of two in [2^20, 2^22] [15 s] */
  double f_switch;       /* Savitzky-Golay switch frequency, Hz [0.8e-3] */
  int32_t nperseg;       /* Welch segment length L: 8192 or 16384 [16384: 2 M / L - 1 = 511
                            segments at M = 2^22, the paper's 500 windows] */
  int32_t clip_width;    /* median-clip window, Welch bins, at most 64 [30] */
  int32_t clip_stride;   /* its shift [15] */
  int32_t sg_short;      /* Savitzky-Golay window length below f_switch [10] */
  int32_t sg_long;       /* and above [70; 50 for T = 0.5 yr] */
  int32_t reserved;      /* must be 0 */
} gb_noise_global_config;

/* Global noise estimate of Sec. III F from a residual d (the data minus the recovered signals;
 * with d - s_partial sum s, Sec. III G, the partial-residual estimate), for every window and
 * channel at once:
 *  1. per channel, the one-sided spectrum of the band assembled from the segments seg (host
 *     int64 [n_win][2], absolute bins [lo, hi) inside the window and inside [1, M/2); the
 *     segments of a channel must not overlap; zero where none is), transformed to the time
 *     series x_n = (1/T) sum_k d_k e^{2 pi i k n / M} (inverse of the convention of the
 *     templates) by a four-step inverse DFT;
 *  2. Welch's method: periodic Hann windows of L = nperseg samples at 50% overlap (2M/L - 1
 *     segments), one-sided density P_j = 2 dt / sum w^2 * mean |DFT(w x)_j|^2 (DC and Nyquist not
 *     doubled) at f_j = j / (L dt);
 *  3. over the channel's band (the Welch bins inside its segments), the median clip: windows of
 *     clip_width bins shifted by clip_stride, in order, values above twice the window's median set
 *     to twice the median;
 *  4. Savitzky-Golay of order 1: window sg_short below f_switch and sg_long above (interior: the
 *     window mean; the first and last length/2 points from the line fitted to the end windows);
 *  5. the natural cubic spline through the smoothed band, evaluated at every bin of every window
 *     (held at its end values outside the band), S, and the weights w = 4 / (T S).
 * windows: host [n_win] (k0, W, C, data_off used; at most 65535); d: device complex128; w: device
 * float64 (d's layout, every window's C x W block written); S: device, same layout, or NULL;
 * welch, smooth: device [3][L/2 + 1] or NULL (step 2 and step 4 of each channel; smooth is zero
 * outside the band; rows of absent channels zero).  All FP64.  Synchronous; allocates about
 * 40 M bytes of temporaries.  GB_EINVAL on a bad setting, window, segment or a band narrower than
 * the filter windows. */
gb_status gb_noise_global(const gb_window* windows, const int64_t* seg, int n_win, const double* d, double T,
                          const gb_noise_global_config* cfg, double* w, double* S, double* welch, double* smooth,
                          void* stream);

/* gb_noise_estimate without any device allocation, for callers that cannot allocate device
 * memory (tight search loops that re-estimate the noise after every found signal, code that
 * must not call hipMalloc).  Same arguments, results and synchronous behaviour as
 * gb_noise_estimate.  The window list is staged in a fixed device array of the library (one
 * per GPU, 16384 windows of 16 bytes = 256 KiB, held until the process ends), filled through a
 * small host buffer on the stack.  Every call on one GPU shares that array, so calls that
 * overlap on one GPU (several host threads or streams) race: serialise them.
 * GB_EINVAL: more than 16384 windows (the staging limit), and the cases of gb_noise_estimate. */
gb_status gb_noise_estimate_noalloc(const gb_window* windows, int n_win, const double* d, double T, double* w,
                                    double* S, void* stream);

/* One generation of the differential-evolution search (DE/best/1/bin or DE/rand/1/bin of Storn
 * and Price, the optimiser the paper's search uses, Sec. III), trial step, for n_win windows with pop members
 * each (pop >= 4), over the seven searched Table I coordinates in the order f0, fdot, sin(beta),
 * lambda, cos(iota), psi, phi0 (the amplitude is not searched: the SNR does not depend on it).
 * For member i of window w:
 *   donors a, b, c: distinct and different from i, uniform; from u_idx[w][i][0..2] in [0, 1):
 *     a = floor(u0 (pop-1)), then b = floor(u1 (pop-2)), c = floor(u2 (pop-3)), each stepped
 *     past the indices already taken, in increasing order;
 *   mutant m = x_a + F[w] (x_b - x_c) (DE/rand/1; base NULL), or m = x_base[w] + F[w] (x_a - x_b)
 *     (DE/best/1, the window's best member as the base: base is a device int32 [n_win], for
 *     instance gb_de_select's best_idx; an index outside [0, pop) is clamped into it), each
 *     product and sum rounded separately; lambda, psi
 *     and phi0 wrap into [lo, hi) (exact remainder), the others reflect at the walls and are
 *     clipped to [lo, hi];
 *   trial coordinate k = m_k where u_cross[w][i][k] < cr or k = floor(u_j[w][i] 7), else x_i,k.
 * lo, hi: device [n_win][7] (the window's box); x: device [n_win][pop][7], the population;
 * u_idx: device [n_win][pop][3]; u_cross: device [n_win][pop][7]; u_j: device [n_win][pop];
 * F: device [n_win]; outputs trial_x [n_win][pop][7] and trial_theta [n_win * pop][8] (the
 * parameters of each trial with amplitude `amp`, ready for gb_loglik).  Asynchronous;
 * allocates nothing.  GB_EINVAL on pop < 4, cr outside [0, 1] or null arrays. */
gb_status gb_de_trial(int n_win, int pop, const double* lo, const double* hi, const double* x, const double* u_idx,
                      const double* u_cross, const double* u_j, const double* F, const int32_t* base, double cr,
                      double amp, double* trial_x, double* trial_theta, void* stream);

/* Selection step of the same generation: rho = <d|h>/sqrt(<h|h>) of every trial from its
 * gb_loglik components (comps: device [n_win * pop][2]; a rho that is not a finite number counts
 * as -inf); where rho exceeds s[w][i], the trial replaces member i of x and rho replaces s.
 * best: device [n_win], the largest s of each window afterwards; best_idx: device int32 [n_win]
 * or NULL, the smallest member index holding it.  x and trial_x may be the same array (scoring
 * an initial population with s = -inf).  Asynchronous; allocates nothing. */
gb_status gb_de_select(int n_win, int pop, const double* comps, double* x, double* s, const double* trial_x,
                       double* best, int32_t* best_idx, void* stream);

/* Log density of weighted 2-D Gaussian kernel density estimates (the pairwise KDE proposals
 * of Sec. III G: (A, iota), (lambda, beta), (f, fdot)), summed over n_pairs pairs, for
 * n_sets independent sets (one per source, so that many sources' annealing stages share a
 * launch):
 *   out[s][i] = sum_p log sum_j wts[s][p][j] N(x[s][i][p]; pts[s][p][j], L_sp L_sp^T)
 * pts: device [n_sets][n_pairs][m][2]; wts: device [n_sets][n_pairs][m] (each pair's weights
 * sum to one; zero weights allowed, so sets with fewer points are padded to m); chol: device
 * [n_sets][n_pairs][3] = (l00, l10, l11), the lower Cholesky factor of each bandwidth matrix
 * (l00, l11 > 0); x: device [n_sets][q][n_pairs][2]; out: device [n_sets][q].  FP64,
 * log-sum-exp (no underflow in the tails).  GB_EINVAL on bad sizes (n_sets above 65535) or
 * null arrays. */
gb_status gb_kde_logpdf(const double* pts, const double* wts, int n_sets, int n_pairs, int64_t m, const double* chol,
                        const double* x, int64_t q, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GBX_H */
