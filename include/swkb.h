/*
 * swkb.h -- C ABI of the screened-WKB (S-WKB) propagation library for AMD
 * MI355X (gfx950).
 *
 * The library carries a time-harmonic field across a sequence of planar
 * screens for the 2D Helmholtz problem  Delta u + k^2 eps(x,z) u = 0
 * (Bruno & Maas, "WKB across caustics: the screened-WKB method", Sec. 2,
 * eq. helmholtz_3D), x the range and z the height.  One screen step
 * (Algorithm 1, "Screened WKB") is:
 *   1. a vertical FFT of the field on screen x_q (Sec. 2.1.1, eqs. fft_eq,
 *      ifft_eq, fourier_psi), keeping the M modes n in [-M/2, M/2);
 *   2. per mode, WKB across the screen: RK4 rays of the characteristic
 *      system for the eikonal phase and the transport amplitude
 *      (Sec. 2.1.2 and Appendix A, eqs. charsys, charsys_s), marched in x;
 *   3. interpolation of phase and amplitude onto the grid of screen x_{q+1}
 *      (Sec. 2.1.2) and
 *   4. the sum over modes (eq. ray_bundle_q_plus_1), then the next screen.
 *
 * Conventions for every entry point:
 *   - Pointers named "device" are HIP device pointers; "host" pointers are
 *     ordinary CPU memory.  Complex data are interleaved (re, im) doubles
 *     (complex128), contiguous.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued asynchronously unless the description says "synchronises".
 *   - The caller owns every buffer it passes; the library never frees
 *     caller memory.  The plan lives in a caller-provided device workspace.
 *   - Every call returns swkb_status; no C++ exception crosses the ABI.
 *     swkb_last_error() gives a message for the last failure on the
 *     calling thread, swkb_plan_error() the last failure on a plan.
 *   - A plan is used from one stream at a time.  A call on a plan returns
 *     SWKB_ERR_BUSY, without doing anything, while another thread is inside
 *     a call on the same plan, or when it names a stream other than the
 *     previous call's and that call's work has not finished.
 */
#ifndef SWKB_H
#define SWKB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum swkb_status {
  SWKB_OK = 0,
  SWKB_ERR_ARG = 1,     /* invalid parameter, size or pointer                     */
  SWKB_ERR_NOMEM = 2,   /* workspace smaller than swkb_workspace_bytes()          */
  SWKB_ERR_DEVICE = 3,  /* a HIP runtime call or kernel launch failed             */
  SWKB_ERR_CAUSTIC = 4, /* a mode above caustic_tol crossed a caustic in a screen */
  SWKB_ERR_STATE = 5,   /* call out of order (e.g. continue without a field)      */
  SWKB_ERR_EVANESCENT = 6, /* a mode above caustic_tol had no live ray: every ray of
                              it was evanescent (p^2 <= p2_floor) at launch or on
                              the way, so its contribution was lost                */
  SWKB_ERR_BUSY = 7     /* the plan is in use: another host thread is inside a
                           call on it, or its previous call's work is still
                           running on another stream (a plan is single-stream)  */
} swkb_status;

/* Arithmetic of a plan.  SWKB_FP64: every step in FP64.  SWKB_MIXED: the
 * FFT, each mode's range phase frac(pbar dx / lambda), the sums across mode
 * groups, the ray-tube variations Z_s, Q_s (accumulated in FP64 from FP32
 * RK4 increments) and the transport amplitude sqrt(p0 / (p Z_s)) (its Z_s
 * factor in FP64) in FP64; the ray state (z - s, q - xi, phase deviation),
 * the medium read from the per-screen table (built from FP64 node values),
 * the interpolation and each mode-point's phase and sin/cos in FP32 (the
 * amplitude is stored in FP32 for the interpolation), with the grid phase
 * n m' / P carried as an exact FP32 fraction of a turn.  Result within 1e-3
 * of the FP64 path (about 1e-5 on smooth media). */
enum { SWKB_FP64 = 0, SWKB_MIXED = 1 };
/* How a screen's mode functions are obtained for media that do not depend
 * on x (LINEAR, EXPGAUSS, MPROFILE): every screen then sees the same rays,
 * so the interpolated mode functions T[n][m] = a_n(z_m) exp(i k psi_n(z_m))
 * (eq. ray_bundle_q_plus_1 without the amplitudes c_n) are the same on every
 * screen and can be built once per plan. */
enum {
  SWKB_PROP_AUTO = 0,      /* matrix when the medium is x-invariant and T fits in 16 GiB */
  SWKB_PROP_MATRIX = 1,    /* always build T once (SWKB_ERR_ARG for GAUSSSUM)            */
  SWKB_PROP_RECOMPUTE = 2  /* interpolate and sum every screen                          */
};
enum { SWKB_BC_PERIODIC = 0, SWKB_BC_DIRICHLET = 1, SWKB_BC_NEUMANN = 2 };
enum {
  SWKB_MEDIUM_LINEAR = 0,   /* params [eps0, g]:          eps = eps0 + g z                       */
  SWKB_MEDIUM_EXPGAUSS = 1, /* params [eps0, a, b, zc]:   eps = eps0 + a exp(-b (z-zc)^2)
                               (the exponential permittivity model of the paper, Sec. 3)       */
  SWKB_MEDIUM_GAUSSSUM = 2, /* params [n_g, (a, s, cx, cz) x n_g]:
                               n = 1 + sum a exp(-((x-cx)^2 + (z-cz)^2) / (2 s^2)), terms with
                               (x-cx)^2 + (z-cz)^2 > 64 s^2 dropped, eps = n^2                   */
  SWKB_MEDIUM_MPROFILE = 3  /* params [M0, g1, g2, d, w, scale]: modified refractivity
                               M = M0 + g1 z + (g2-g1) w log(1 + exp((z-d)/w)),
                               n = 1 + scale M, eps = n^2 (surface duct, corner smoothed)         */
};

/* Problem and numerical parameters of one propagation problem. */
typedef struct swkb_params {
  double k;                 /* wavenumber 2 pi / lambda                                     */
  double z_a, z_b;          /* screen extent; grid z_m = z_a + m h, h = (z_b - z_a) / n_z   */
  int32_t n_z;              /* grid points N: a power of two, 64 <= N <= 32768              */
  int32_t n_modes;          /* kept modes M: even, 2 <= M <= P (P = N, or 2N with a mirror) */
  double x0, dx;            /* first screen x_0 and screen spacing; x_q = x0 + q dx        */
  int32_t n_screens;        /* screens reachable by this plan: q in [0, n_screens]          */
  int32_t rk4_steps;        /* RK4 steps S per screen, >= 1                                 */
  int32_t ray_stride;       /* ray launch spacing rho in grid cells, >= 1                   */
  int32_t launch_ext_cells; /* launch extension E in cells: rays start at
                               s_r = z_a + (r rho - E) h, r = 0..R-1,
                               R = ceil((N + 2E) / rho) + 1                                 */
  double p2_floor;          /* a ray with p^2 = eps - q^2 <= p2_floor is dead               */
  int32_t bc;               /* SWKB_BC_*: ground mirror about z_a (Sec. 2.3)                */
  int32_t medium_kind;      /* SWKB_MEDIUM_*                                                 */
  double absorber_bot;      /* cos^2 taper thickness at z_a (0 = none)                       */
  double absorber_top;      /* cos^2 taper thickness at z_b (0 = none)                       */
  const double* medium_params; /* host; copied by swkb_plan                                  */
  int32_t n_medium_params;
  int32_t precision;        /* SWKB_FP64 or SWKB_MIXED                                       */
  double eps_ref;           /* reference permittivity of the phase split (bookkeeping only) */
  double caustic_tol;       /* SWKB_ERR_CAUSTIC when a mode with |c_n| > caustic_tol max|c|
                               has a caustic (Z_s <= 0) or crossing rays in a screen          */
  int32_t propagator;       /* SWKB_PROP_*; the matrix costs N*M*16 bytes (FP64) or N*M*8
                               bytes (mixed) of workspace                                     */
  int32_t max_batch;        /* largest number of fields swkb_propagate_batch carries at once
                               (>= 1); workspace for the fields grows with it               */
  int32_t keep_history;     /* 1: the plan keeps the field of every screen it reaches in its
                               workspace ((n_screens + 1) N complex128 more), so that
                               swkb_field can return any of them; 0: only the current one  */
} swkb_params;

/* Device-side health counters, summed over all screens propagated so far. */
typedef struct swkb_counters {
  int64_t caustic_rays; /* rays with Z_s <= 0 at some RK4 stage (dropped)              */
  int64_t dead_rays;    /* rays with p^2 <= p2_floor at launch or on the way (dropped) */
  int64_t folded_modes; /* modes whose live arrivals were not increasing in z (dropped) */
  int64_t significant;  /* caustic or folded modes with |c_n| > caustic_tol max|c|     */
  int64_t screens;      /* screen steps executed                                         */
  /* work of the method, per screen step summed (for throughput accounting):          */
  int64_t rhs_evals;    /* RK4 stage evaluations of the ray system by live rays          */
  int64_t medium_evals; /* direct evaluations of eps, eps_z, eps_zz (stages, launch,
                           arrival)                                                      */
  int64_t medium_terms; /* Gaussian terms inside their cutoff evaluated (GAUSSSUM)        */
  int64_t table_evals;  /* evaluations read from the per-screen medium table (mixed
                           precision, GAUSSSUM, periodic)                                */
  int64_t evanescent_modes; /* modes of which no ray arrived live (all dead)              */
  int64_t significant_evanescent; /* of those, modes with |c_n| > caustic_tol max|c|     */
} swkb_counters;

/* Device time per kernel class, from HIP events recorded on the launch
 * stream around each kernel while profiling is enabled. */
typedef struct swkb_timing {
  double march_ms, scan_ms, fft_ms, superpose_ms;
  int64_t march_launches, scan_launches, fft_launches, superpose_launches;
  double table_ms;        /* per-screen medium table builds (mixed GAUSSSUM march)  */
  int64_t table_launches;
} swkb_timing;

typedef struct swkb_plan_s* swkb_plan_t;

/* Bytes of device workspace a plan for *p needs (0 if *p is invalid).
 * Host only. */
size_t swkb_workspace_bytes(const swkb_params* p);

/* Device bytes one propagation request for *p holds while it runs: the
 * plan's workspace plus one field of n_z complex128 for its input and a
 * small allowance for the runtime's per-stream state (0 if *p is invalid).
 * The serving loop admits requests by this figure.  Host only. */
size_t swkb_footprint(const swkb_params* p);

/* Build a plan: validates *p (SWKB_ERR_ARG with a message otherwise),
 * derives the mode tables (xi_n = 2 pi n / (k P h), Sec. 2.1.1-2.1.2), the
 * FFT twiddles and, for SWKB_MEDIUM_GAUSSSUM, the per-screen lists of
 * Gaussians whose 8-sigma disc meets the screen, and uploads them into
 * workspace (device, >= swkb_workspace_bytes(p) bytes, 256-byte aligned)
 * on hip_stream.  The workspace must stay allocated until swkb_destroy.
 * *out receives a host handle. */
swkb_status swkb_plan(const swkb_params* p, void* workspace, size_t workspace_bytes,
                      void* hip_stream, swkb_plan_t* out);

/* Propagate screens q_begin .. q_end-1 (Algorithm 1 per screen).  For media
 * that change with x the march and the scan of each screen run on a march
 * and a scan stream that all plans on the device share (default priority),
 * ordered against hip_stream by events of the plan; the plan's results are
 * complete when hip_stream reaches the end of the call's work.
 * u_in: device complex128[N], the field on screen q_begin; NULL continues
 * from the plan's current field, which must then be on screen q_begin.
 * history: device complex128[(q_end - q_begin) * N] receiving the field on
 * screens q_begin+1 .. q_end, or NULL.  Afterwards the plan's current
 * field is the one on screen q_end.  0 <= q_begin <= q_end <= n_screens.
 * Asynchronous on hip_stream; caustics are reported by swkb_diagnostics. */
swkb_status swkb_propagate(swkb_plan_t plan, const void* u_in, int32_t q_begin, int32_t q_end,
                           void* history, void* hip_stream);

/* Propagate `batch` fields (several sources in the same medium) across
 * screens q_begin .. q_end-1 together: the rays, and for an x-invariant
 * medium the mode-function matrix, are shared, so each screen costs one
 * march (x-varying media) plus per-field FFTs and sums; with the matrix the
 * sums over modes of all fields form one complex matrix product on the
 * matrix cores (the matrix is read once per screen for all fields; FP64
 * instructions for SWKB_FP64, FP32 ones with FP64 cross-group sums for
 * SWKB_MIXED).  Results equal `batch` separate swkb_propagate runs up to
 * rounding.
 *   u_in:    device complex128[batch][N], fields on screen q_begin;
 *   history: device complex128[q_end - q_begin][batch][N] or NULL;
 *   u_out:   device complex128[batch][N], fields on screen q_end, or NULL.
 * 1 <= batch <= max_batch, 0 <= q_begin < q_end <= n_screens.  With
 * max_batch > 1 the plan's single-field state (swkb_field,
 * swkb_current_screen) is not changed; with max_batch == 1 the call uses the
 * single-field buffer and leaves the plan without a current field. */
swkb_status swkb_propagate_batch(swkb_plan_t plan, const void* u_in, int32_t batch, int32_t q_begin,
                                 int32_t q_end, void* history, void* u_out, void* hip_stream);

/* Fields between screens q and q+1 (the paper's "additional interpolation
 * points", end of Sec. 2.1.2): for each station i in stations (host int32
 * array of n values, 1 <= i <= rk4_steps) the field at x_q + i*dx/S obtained
 * from the modes of the field u (device complex128[N] on screen q) by the
 * same step as a screen of width i*dx/S marched with i RK4 steps of the
 * screen's step size (taper included).  out: device complex128[n][N].
 * Synchronises hip_stream.  Does not change the plan's field or counters. */
swkb_status swkb_propagate_stations(swkb_plan_t plan, const void* u, int32_t q, const int32_t* stations, int32_t n,
                                    void* out, void* hip_stream);

/* Reference solution by separation of variables (the paper's reference
 * method, Sec. 3.1, eqs. series_sol, phi_equation, series_init,
 * sl_expansion) for a medium that does not depend on x: the Sturm-Liouville
 * operator d^2/dz^2 + k^2 eps is discretised Fourier-spectrally on the screen
 * grid (on the doubled grid with eps reflected about z_a for a ground
 * mirror, the field extended oddly/evenly) and diagonalised in FP64 with
 * rocSOLVER; u(x) = Phi e^{i alpha x} Phi^T u0 with alpha = sqrt(lambda)
 * (decaying for lambda < 0).  Uses p (no plan); u0: device complex128[N];
 * xs: host double[nx] ranges from the screen of u0; out: device
 * complex128[nx][N].  P = N (periodic) or 2N must be <= 16384.  Allocates
 * and frees its own device memory (P^2 doubles); synchronises hip_stream.
 * SWKB_ERR_ARG for an x-varying medium. */
swkb_status swkb_modal_reference(const swkb_params* p, const void* u0, const double* xs, int32_t nx, void* out,
                                 void* hip_stream);

/* Copy the field on screen q (device complex128[N]) into out (device): the
 * field on Gamma_q, q = 0 .. n_screens (Sec. 2.1.2: the method yields the
 * field on the screens).  q = -1 asks for the plan's current field (screen
 * swkb_current_screen).  Other screens are held only with keep_history = 1:
 * every screen a propagation passed through or ended on (the input of
 * swkb_propagate included) since the plan was built, the latest value of each.
 * SWKB_ERR_STATE if screen q is not held (before the first swkb_propagate,
 * or keep_history = 0 and q is not the current screen); SWKB_ERR_ARG for q
 * outside [-1, n_screens]. */
swkb_status swkb_field(swkb_plan_t plan, int32_t q, void* out, void* hip_stream);

/* Current screen index of the plan's field (-1 before the first propagate). */
int32_t swkb_current_screen(swkb_plan_t plan);

/* Synchronises hip_stream, copies the counters to *out (host) and returns
 * SWKB_ERR_CAUSTIC if out->significant > 0 (a mode that matters met a
 * caustic inside a screen, against the Remark of Sec. 2.1.2), else
 * SWKB_ERR_EVANESCENT if out->significant_evanescent > 0, else SWKB_OK. */
swkb_status swkb_diagnostics(swkb_plan_t plan, void* hip_stream, swkb_counters* out);

/* Enable (1) or disable (0) HIP graphs for swkb_propagate: the first call
 * with a given (u_in, q_begin, q_end, history) captures its whole screen
 * sequence (FFT, march, scan, sums; all streams) into a graph on the capture
 * stream the device's plans share, later calls with the same arguments
 * replay it (up to 4 graphs are kept).  A replay launches the same kernels
 * with the same arguments, so it gives the same fields as an eager call; it
 * reads u_in and writes history when it runs.  Ignored while profiling.
 * Disabling waits for replays in flight and frees the graphs.  Host only;
 * capture is not thread-safe across plans of one device. */
swkb_status swkb_graphs(swkb_plan_t plan, int32_t enable);

/* Enable (1) or disable (0) event timing of every kernel the plan launches.
 * Host only; events are recorded on the stream of each launch. */
swkb_status swkb_profile(swkb_plan_t plan, int32_t enable);

/* Synchronises hip_stream, writes the accumulated device times to *out
 * (host) and clears them. */
swkb_status swkb_profile_read(swkb_plan_t plan, void* hip_stream, swkb_timing* out);

/* Release the host handle (the caller frees the workspace). */
void swkb_destroy(swkb_plan_t plan);

const char* swkb_status_string(swkb_status s);
/* Message of the last failure on the calling thread (any entry point). */
const char* swkb_last_error(void);
/* Message of the last failure of a call on this plan (from any thread; ""
 * if none).  The string stays valid until the next failing call on the plan
 * or swkb_destroy. */
const char* swkb_plan_error(swkb_plan_t plan);

/* ---- one propagation without device allocation ----------------------- */

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: work being captured into a HIP graph by the caller, tight
 * serving loops, harnesses that forbid allocation): swkb_plan, swkb_propagate
 * and swkb_destroy in one call, with the plan's workspace in a static device
 * array of SWKB_STATIC_WORKSPACE_BYTES that the library holds on every GPU it
 * runs on until the process ends.  Same kernels and launch shapes as
 * swkb_propagate (one after another on hip_stream: no march stream), so the
 * fields equal a plan's.
 *   p:       as for swkb_plan; SWKB_ERR_NOMEM (message in swkb_last_error)
 *            when swkb_workspace_bytes(p) > SWKB_STATIC_WORKSPACE_BYTES,
 *            SWKB_ERR_ARG for invalid parameters;
 *   u_in:    device complex128[n_z], the field on screen q_begin;
 *   history: device complex128[(q_end - q_begin) n_z] (screens q_begin+1 ..
 *            q_end) or NULL; u_out: device complex128[n_z] (screen q_end) or
 *            NULL.  0 <= q_begin < q_end <= n_screens.
 * Calls no hipMalloc, hipFree or allocating library routine.  Synchronises
 * hip_stream once (upload of the plan tables, as swkb_plan); the propagation
 * itself is asynchronous.  The array keeps the last call's contents; every
 * table and counter a call reads is written by that call first.  Calls on
 * one GPU share its array: the library orders them (each call's stream waits
 * for the previous call's work, and host threads enter one at a time), so
 * two calls whose work overlaps on the device would race; there is no plan
 * left behind (no swkb_field or swkb_diagnostics afterwards). */
#define SWKB_STATIC_WORKSPACE_BYTES (64u << 20)
swkb_status swkb_propagate_static(const swkb_params* p, const void* u_in, int32_t q_begin, int32_t q_end,
                                  void* history, void* u_out, void* hip_stream);

/* ---- stage entry points, for checking each step on its own ---------- */

/* Step 1 only: c (device complex128[M], c[j] for n = j - M/2) = the DFT of
 * the (mirror-extended) field u (device complex128[N]) divided by P. */
swkb_status swkb_stage_modes(swkb_plan_t plan, const void* u, void* c, void* hip_stream);

/* Step 2 only, for screen q: arrival records of all M x R rays, row-major
 * [mode j][ray r], written as doubles to device arrays Z (arrival height),
 * psi (full phase psi, length units), qz (psi_z at arrival), amp (transport
 * factor sqrt(p0 / (p Z_s))), and int32 flag (0 live, 1 dead at launch,
 * 2 dead on the way, 3 caustic).  R = swkb_num_rays(plan). */
swkb_status swkb_stage_rays(swkb_plan_t plan, int32_t q, void* Z, void* psi, void* qz, void* amp,
                            void* flag, void* hip_stream);

/* Rays per mode R of the plan. */
int32_t swkb_num_rays(swkb_plan_t plan);

/* 1 if the plan holds the mode-function matrix T (SWKB_PROP_*), else 0. */
int32_t swkb_uses_matrix(swkb_plan_t plan);

/* ---- many problems in one launch per stage -------------------------- */

/* Several independent problems in media that do not depend on x (each with
 * its own plan: frequency, profile, height, grid, range), all carried from
 * their first screen to their last together.  Every screen step is one
 * launch per stage for all problems still running: the FFT column and row
 * passes, the product of the mode-function matrix with the modes (Sec.
 * 2.1.2, eq. ray_bundle_q_plus_1 with the mode functions tabulated once), and
 * the exit epilogue; each workgroup finds its problem and its place in it in
 * a device table.  Problems are ordered by screen count, so the problems
 * still running at step q are a prefix of the table and the launches of
 * step q cover exactly them.  With graphs enabled the whole sequence of
 * steps is captured once into a HIP graph and replayed as one launch.  With
 * SWKB_MULTI_PERSISTENT it is one persistent launch instead: a cooperative
 * grid of workgroups that are all resident at once walks every step's four
 * stages in order, each workgroup taking every gridDim-th map entry of a
 * stage, with a grid-wide barrier between stages; it runs the same device
 * code item for item, so the fields equal those of the per-stage launches
 * bit for bit.
 *
 * Requirements per plan: mode-function matrix in use (swkb_uses_matrix),
 * n_z a multiple of 512; at most 4095 plans, each listed once.  SWKB_MIXED
 * and SWKB_FP64 plans may share a group; an FP64 problem's product keeps the
 * single-problem blocking (apply_groups shapes the complex64 products).  The plans stay owned by the caller, must outlive the group
 * and must not be used otherwise while a group call is in flight.  The
 * group allocates its own device memory (hipMalloc: a problem table, the
 * workgroup maps and the partial sums of the product). */
typedef struct swkb_multi_s* swkb_multi_t;

/* Launch shapes per size class (problems with the same n_z), picked by
 * swkb_multi_tune or set by the caller.  fft_elems: elements per FFT
 * workgroup (256, 512 or 1024); apply_groups: workgroups along the modes
 * of the product (>= 1; each covers every apply_groups-th set of
 * four modes; clamped to (n_modes + 3) / 4 per problem); the defaults
 * equal the single-problem path's choices, which makes every field
 * bit-identical to a separate swkb_propagate. */
#define SWKB_MULTI_MAX_CLASSES 16
#define SWKB_MULTI_PERSISTENT 2
typedef struct swkb_multi_tuning {
  int32_t n_classes;                            /* distinct n_z, ascending   */
  int32_t class_n_z[SWKB_MULTI_MAX_CLASSES];
  int32_t fft_elems[SWKB_MULTI_MAX_CLASSES];
  int32_t apply_groups[SWKB_MULTI_MAX_CLASSES];
  int32_t graphs;                               /* 0: one launch per stage, 1: captured and replayed, SWKB_MULTI_PERSISTENT: one launch */
  double fft_us[SWKB_MULTI_MAX_CLASSES];        /* tuner: best FFT time of the class's screen (both passes) */
  double apply_us[SWKB_MULTI_MAX_CLASSES];      /* tuner: best product time of the class's screen           */
} swkb_multi_tuning;

/* Host only (uploads the problem table and maps with a synchronous copy).
 * SWKB_ERR_ARG if a plan does not meet the requirements above or more than
 * SWKB_MULTI_MAX_CLASSES distinct n_z occur. */
swkb_status swkb_multi_create(const swkb_plan_t* plans, int32_t n, swkb_multi_t* out);

/* Current launch shapes into *out (host). */
swkb_status swkb_multi_get_tuning(swkb_multi_t m, swkb_multi_tuning* out);

/* Set launch shapes: class_n_z must list the group's classes as
 * swkb_multi_get_tuning returns them; values outside the ranges above give
 * SWKB_ERR_ARG.  Drops a captured graph. */
swkb_status swkb_multi_set_tuning(swkb_multi_t m, const swkb_multi_tuning* t);

/* Autotuner: for each size class, times every FFT blocking and every
 * product blocking in a candidate set with HIP events on hip_stream (each
 * candidate launched `reps` times over that class's problems alone, best
 * average kept), applies the fastest and writes the result to *out (may be
 * NULL).  Overwrites the plans' current fields (zeroed first) and leaves
 * them without a current field; counters are not touched.  Synchronises
 * hip_stream.  reps >= 1. */
swkb_status swkb_multi_tune(swkb_multi_t m, int32_t reps, void* hip_stream, swkb_multi_tuning* out);

/* Carry every problem from screen 0 to its last screen (Algorithm 1).
 * u_in: host array of n device pointers, complex128[n_z_i] each, the fields
 * on screen 0 in the order the plans were given; history: host array of n
 * device pointers (complex128[n_screens_i][n_z_i] receiving screens
 * 1 .. n_screens_i, entries may be NULL) or NULL.  Afterwards each plan's
 * current field is on its last screen (swkb_field) and its counters include
 * the run (swkb_diagnostics).  Asynchronous on hip_stream, except that the
 * host waits until the previous call's problem table has been copied. */
swkb_status swkb_multi_propagate(swkb_multi_t m, const void* const* u_in, void* const* history, void* hip_stream);

/* Waits for the group's work, frees its device memory and graph. */
void swkb_multi_destroy(swkb_multi_t m);

/* ---- overlapping patches ---------------------------------------------- */

/* The screen step on overlapping patches (Sec. 2.4): the vertical interval
 * is covered by n_patches patches around the cores [c_p, c_{p+1}],
 * c_p = z_a + p K h (K = n_z / n_patches cells), blended by the smooth
 * partition of unity sigma_p(z) = erfc(-(z - c_p) / width) / 2,
 * S^0 = 1 - sigma_1, S^p = sigma_p - sigma_{p+1}, S^{P-1} = sigma_{P-1}.
 *
 * SWKB_PATCH_FC, the paper's FC-SWKB (eq. ifft_eq_phi_patches): patch p
 * holds the grid points [a_p, b_p] = [p K - e, (p + 1) K + e], e =
 * ceil(6 width / h), clipped to the grid.  Each screen the field on the patch
 * is Fourier-continued (FC-Gram blend: 27 cells blending the 5 end samples to
 * zero past each end) into one period of a power-of-two length (the patch,
 * 2 x 27 blend cells and ceil(margin / h) cells of drift on each side); its
 * DFT gives the patch's modes, whose rays start at the patch's points only,
 * with initial amplitude S^p(z) w_j / N; the patches' mode sums are added on
 * the global grid.  Over a ground (Sec. 2.5) the boundary patch is continued
 * at its top only and keeps the ground mirror (odd or even extension,
 * reflected medium, S^0 reflected), and every other patch's sum is reflected
 * about z_a on each screen (eq. u_refl).
 *
 * SWKB_PATCH_WINDOWED, a variant of this library's: the field is windowed
 * (S^p u) and each piece runs the screen step of swkb_propagate over a
 * sub-domain holding the core and ceil((6 width + margin) / h) cells on each
 * side (the bottom patch keeps the ground mirror and starts at z_a); the
 * pieces carry the spectra of S^p u instead of launching S^p with each mode.
 *
 * Both: sub-domains keep the global largest vertical slowness (n_modes_p =
 * 2 floor(n_modes P_p / (2 P) + 1/2) with P_p, P the FFT lengths) and have no
 * absorbers; the global exit taper applies once after the sum; margin must
 * cover the drift of the rays over one screen.  Cost per screen: the sum
 * over patches of n_modes_p P_p instead of n_modes n_z. */
#define SWKB_PATCH_FC 0
#define SWKB_PATCH_WINDOWED 1
typedef struct swkb_patch_config {
  int32_t n_patches;  /* >= 1, divides n_z                          */
  double width;       /* partition of unity scale (z units), > 0    */
  double margin;      /* drift room on each side, >= 0 (z units)    */
  int32_t method;     /* SWKB_PATCH_FC or SWKB_PATCH_WINDOWED        */
} swkb_patch_config;

typedef struct swkb_patch_s* swkb_patch_t;

/* Host; builds one plan per patch (swkb_plan) in device memory the patch
 * plan allocates itself (hipMalloc) and frees in swkb_patch_destroy; p must
 * have max_batch = 1.  The global n_z need only be in [64, 2^24] and a
 * multiple of n_patches (it may exceed a single plan's limit); every
 * sub-domain must be a valid plan.  Synchronises hip_stream.  SWKB_ERR_ARG
 * for invalid parameters, including a sub-domain the library cannot plan. */
swkb_status swkb_patch_plan(const swkb_params* p, const swkb_patch_config* pc, void* hip_stream, swkb_patch_t* out);

/* First global grid index, points and modes of patch `patch`'s sub-domain
 * (any pointer may be NULL). */
swkb_status swkb_patch_info(swkb_patch_t pp, int32_t patch, int32_t* start, int32_t* n_z, int32_t* n_modes);

/* Screens q_begin .. q_end-1 by the patch step; arguments and history as in
 * swkb_propagate (device complex128 arrays of the global n_z).  Asynchronous
 * on hip_stream. */
swkb_status swkb_patch_propagate(swkb_patch_t pp, const void* u_in, int32_t q_begin, int32_t q_end, void* history,
                                 void* hip_stream);

/* Enable (1) or disable (0) HIP graphs for swkb_patch_propagate when the
 * patches run as one group (media that do not depend on x, mixed
 * precision): the first call with a given (u_in, q_begin, q_end, history)
 * captures the screen range on a stream of the plan's own, later calls
 * replay it (up to 4 graphs kept; a replay gives the fields of an eager
 * call).  Disabling waits for replays in flight and frees the graphs.
 * Host only; ignored for patch plans that do not run as a group. */
swkb_status swkb_patch_graphs(swkb_patch_t pp, int32_t enable);

/* The current global field into out (device complex128[n_z]). */
swkb_status swkb_patch_field(swkb_patch_t pp, void* out, void* hip_stream);

/* Waits for the device, frees the sub-plans and the patch plan's memory. */
void swkb_patch_destroy(swkb_patch_t pp);

/* ---- serving loop ----------------------------------------------------- */

/* Continuous batching of independent propagation requests on the current
 * device (one problem = one swkb_params and incident field; Algorithm 1 over
 * all its screens).  Requests are admitted in arrival order while their
 * device footprint (workspace + field) fits hbm_budget_bytes and fewer than
 * max_active are admitted; each admitted request gets its own plan,
 * workspace (hipMalloc) and stream, and every swkb_server_step advances each
 * admitted request whose previous chunk has finished by one chunk of
 * screens, so the requests' work overlaps on the device.  A chunk holds
 * about mode_points_per_round mode-point evaluations (M N per screen), at
 * least screens_per_round screens: every admitted request gets a similar
 * share of the device per round, so short requests finish within a few
 * rounds instead of waiting behind long ones.  The result of a
 * request does not depend on what else is being served.  Not thread-safe:
 * one host thread drives a server. */
typedef struct swkb_server_config {
  size_t hbm_budget_bytes;   /* device bytes the admitted requests may hold (> 0) */
  int32_t max_active;        /* most requests admitted at once (>= 1)            */
  int32_t screens_per_round; /* fewest screens per chunk (>= 1)                  */
  double mode_points_per_round; /* M N per screen times screens per chunk (0: chunks
                                   of screens_per_round screens)                  */
} swkb_server_config;

typedef struct swkb_request_info {
  int32_t state;     /* 0 pending, 1 admitted, 2 done, 3 failed                    */
  int32_t n_z;
  double queue_us;   /* submit -> admission (host clock), -1 while pending          */
  double latency_us; /* submit -> completion seen by swkb_server_step, -1 before    */
} swkb_request_info;

typedef struct swkb_server_stats_t {
  int64_t completed, screens, mode_points; /* finished requests and their work (M N Q summed) */
  size_t device_bytes_in_use;
  int32_t active, pending;
  double seconds;                          /* since swkb_server_create                        */
} swkb_server_stats_t;

typedef struct swkb_server_s* swkb_server_t;

/* Host only.  SWKB_ERR_ARG for a config outside the ranges above. */
swkb_status swkb_server_create(const swkb_server_config* cfg, swkb_server_t* out);

/* Queue a request: *p is copied (medium parameters included), u0 (host
 * complex128[n_z], the field on screen 0) is copied into pinned host
 * memory.  *id receives the request's handle.  SWKB_ERR_ARG for invalid
 * parameters, SWKB_ERR_NOMEM if the request alone exceeds the budget. */
swkb_status swkb_server_submit(swkb_server_t s, const swkb_params* p, const void* u0, int64_t* id);

/* One scheduling round (host, non-blocking except for plan builds of newly
 * admitted requests): retire finished requests, advance the others by a
 * chunk, admit pending requests.  *n_active / *n_pending (may be NULL)
 * receive the counts afterwards. */
swkb_status swkb_server_step(swkb_server_t s, int32_t* n_active, int32_t* n_pending);

/* State of request id in *info (may be NULL).  When done and out != NULL,
 * copies the field on the last screen into out (host complex128[n_z]) and
 * forgets the request.  SWKB_ERR_STATE while not done, SWKB_ERR_DEVICE
 * (message in swkb_last_error) if it failed, SWKB_ERR_ARG for an unknown id. */
swkb_status swkb_server_poll(swkb_server_t s, int64_t id, void* out, swkb_request_info* info);

swkb_status swkb_server_stats(swkb_server_t s, swkb_server_stats_t* out);

/* Waits for admitted requests, frees everything the server holds. */
void swkb_server_destroy(swkb_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* SWKB_H */
