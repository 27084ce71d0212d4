// Host side of the C ABI declared in include/swkb.h: argument validation,
// workspace layout, plan tables and the per-screen launch sequence.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "plan_guard.h"
#include "swkb_internal.h"

namespace swkb {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int waves_per_mode(const Geometry& g);

namespace {

bool is_pow2(long long x) { return x > 0 && (x & (x - 1)) == 0; }

int expected_params(const swkb_params* p) {
  switch (p->medium_kind) {
    case SWKB_MEDIUM_LINEAR: return 2;
    case SWKB_MEDIUM_EXPGAUSS: return 4;
    case SWKB_MEDIUM_MPROFILE: return 6;
    case SWKB_MEDIUM_GAUSSSUM:
      if (p->n_medium_params < 1 || !p->medium_params) return -1;
      return 1 + 4 * (int)p->medium_params[0];
    default: return -1;
  }
}

// Returns an empty string when *p is acceptable.
std::string validate(const swkb_params* p) {
  if (!p) return "params is NULL";
  if (!(p->k > 0.0) || !std::isfinite(p->k)) return "k must be positive and finite";
  if (!(p->z_b > p->z_a)) return "z_b must exceed z_a";
  if (!is_pow2(p->n_z) || p->n_z < 64 || p->n_z > 32768) return "n_z must be a power of two in [64, 32768]";
  const int P = p->bc == SWKB_BC_PERIODIC ? p->n_z : 2 * p->n_z;
  if (p->n_modes < 2 || (p->n_modes & 1) || p->n_modes > P) return "n_modes must be even and in [2, P]";
  if (!(p->dx > 0.0) || !std::isfinite(p->x0)) return "dx must be positive";
  if (p->n_screens < 1) return "n_screens must be >= 1";
  if (p->rk4_steps < 1 || p->rk4_steps > 4096) return "rk4_steps must be in [1, 4096]";
  if (p->ray_stride < 1 || p->ray_stride > p->n_z) return "ray_stride must be in [1, n_z]";
  if (p->launch_ext_cells < 0 || p->launch_ext_cells > 4 * p->n_z) return "launch_ext_cells must be in [0, 4 n_z]";
  if (!(p->p2_floor >= 0.0)) return "p2_floor must be >= 0";
  if (p->bc < 0 || p->bc > 2) return "bc must be SWKB_BC_PERIODIC, _DIRICHLET or _NEUMANN";
  if (p->precision != SWKB_FP64 && p->precision != SWKB_MIXED) return "precision must be SWKB_FP64 or SWKB_MIXED";
  const double L = p->z_b - p->z_a;
  if (!(p->absorber_bot >= 0.0 && p->absorber_top >= 0.0 && p->absorber_bot + p->absorber_top <= L))
    return "absorber thicknesses must be >= 0 and fit in [z_a, z_b]";
  if (!(p->caustic_tol >= 0.0)) return "caustic_tol must be >= 0";
  if (!(p->eps_ref > 0.0)) return "eps_ref must be positive";
  const int np = expected_params(p);
  if (np < 0) return "unknown medium_kind or missing parameters";
  if (p->n_medium_params != np || !p->medium_params) return "n_medium_params does not match medium_kind";
  for (int i = 0; i < np; ++i)
    if (!std::isfinite(p->medium_params[i])) return "medium_params must be finite";
  if (p->medium_kind == SWKB_MEDIUM_GAUSSSUM) {
    const int ng = (int)p->medium_params[0];
    if (ng < 0 || (double)ng != p->medium_params[0]) return "GAUSSSUM count must be a non-negative integer";
    for (int j = 0; j < ng; ++j)
      if (!(p->medium_params[2 + 4 * j] > 0.0)) return "GAUSSSUM widths must be positive";
  }
  if (p->medium_kind == SWKB_MEDIUM_MPROFILE && !(p->medium_params[4] > 0.0)) return "MPROFILE w must be > 0";
  if (p->propagator < SWKB_PROP_AUTO || p->propagator > SWKB_PROP_RECOMPUTE) return "propagator must be SWKB_PROP_*";
  if (p->propagator == SWKB_PROP_MATRIX && p->medium_kind == SWKB_MEDIUM_GAUSSSUM)
    return "SWKB_PROP_MATRIX needs a medium that does not depend on x";
  if (p->max_batch < 1 || p->max_batch > 4096) return "max_batch must be in [1, 4096]";
  if (p->keep_history != 0 && p->keep_history != 1) return "keep_history must be 0 or 1";
  return "";
}

// The mode-function matrix is used for x-invariant media unless the caller
// asks to recompute; AUTO also requires it to fit in 16 GiB.
size_t matrix_bytes(const swkb_params* p) {
  return (size_t)p->n_z * (size_t)p->n_modes * (p->precision == SWKB_FP64 ? sizeof(double2) : sizeof(float2));
}

bool use_matrix(const swkb_params* p) {
  if (p->medium_kind == SWKB_MEDIUM_GAUSSSUM || p->propagator == SWKB_PROP_RECOMPUTE) return false;
  if (p->propagator == SWKB_PROP_MATRIX) return true;
  return matrix_bytes(p) <= ((size_t)16 << 30);
}

Geometry geometry(const swkb_params* p) {
  Geometry g;
  g.N = p->n_z;
  g.M = p->n_modes;
  g.bc = p->bc;
  g.P = g.bc == SWKB_BC_PERIODIC ? g.N : 2 * g.N;
  g.rho = p->ray_stride;
  g.E = p->launch_ext_cells;
  g.R = (g.N + 2 * g.E + g.rho - 1) / g.rho + 1;
  g.T = g.N / kTile;
  g.S = p->rk4_steps;
  int lp = 0;
  while ((1 << lp) < g.P) ++lp;
  g.P1 = 1 << (lp / 2);
  g.P2 = g.P / g.P1;
  g.z_a = p->z_a;
  g.z_b = p->z_b;
  g.h = (p->z_b - p->z_a) / p->n_z;
  g.k = p->k;
  g.lam = 2.0 * M_PI / p->k;
  g.dx = p->dx;
  g.p2_floor = p->p2_floor;
  return g;
}

// Per-screen candidate Gaussians: bump j can reach the screen strip
// [x_q, x_q + dx] only if |x - cx_j| <= 8 s_j somewhere in it.
std::vector<int> gauss_lists(const swkb_params* p, std::vector<int>* off) {
  std::vector<int> list;
  off->assign(p->n_screens + 2, 0);
  if (p->medium_kind != SWKB_MEDIUM_GAUSSSUM) return list;
  const int ng = (int)p->medium_params[0];
  for (int q = 0; q <= p->n_screens; ++q) {
    (*off)[q] = (int)list.size();
    if (q == p->n_screens) break;
    const double xa = p->x0 + q * p->dx, xb = xa + p->dx;
    for (int j = 0; j < ng; ++j) {
      const double s = p->medium_params[2 + 4 * j], cx = p->medium_params[3 + 4 * j];
      const double slack = 1e-9 * (std::fabs(cx) + std::fabs(xb) + 1.0);
      const double near = cx < xa ? xa : (cx > xb ? xb : cx);
      if (std::fabs(near - cx) <= 8.0 * s + slack) list.push_back(j);
    }
  }
  (*off)[p->n_screens + 1] = (int)list.size();
  return list;
}

struct Layout {
  size_t xi, pbar, e1r, frac, frac_st, tw, mprm, glist, gstage, gterm, gczl, u, ub, Y, c, pan, menergy, cpol, part, tmat, hist,
      counters;
  // one ray-record slot (offsets from its start); nslots of them from slot0
  size_t mtab, D, Pp, G, A, cz, cidx, tstart, mflag, mcaus, mdead, mwork, wcount;
  size_t slot0, slot_bytes;
  int nslots;
  size_t total;
};

// The Gaussian-sum march without a mirror reads per-screen bump tables
// (precomputed per RK4 stage position and per wavefront reference height).
bool gauss_fast(const swkb_params* p, const std::vector<int>& off) {
  (void)off;
  return p->medium_kind == SWKB_MEDIUM_GAUSSSUM && p->bc == SWKB_BC_PERIODIC;
}

// Medium table of the mixed Gaussian-sum march: node spacing s_min / 40 over
// the launch span, widened on both sides by the launch extension plus the
// farthest a ray can travel in z across one screen (|q| / p with
// p^2 > p2_floor and eps <= 1 + max(0, sum of bump amplitudes)^2 terms).
// Returns n = 0 where the direct evaluation is used.
MedTab med_table(const swkb_params* p, const Geometry& g) {
  MedTab t{nullptr, 0, 0.0, 0.0};
  if (p->medium_kind != SWKB_MEDIUM_GAUSSSUM || p->bc != SWKB_BC_PERIODIC || p->precision != SWKB_MIXED) return t;
  const int ng = (int)p->medium_params[0];
  if (ng < 1) return t;
  double smin = p->medium_params[2], amax = 0.0;
  for (int j = 0; j < ng; ++j) {
    smin = std::min(smin, p->medium_params[2 + 4 * j]);
    amax += std::max(0.0, p->medium_params[1 + 4 * j]);
  }
  const double eps_max = (1.0 + amax) * (1.0 + amax);
  const double reach = p->dx * std::sqrt(eps_max / std::max(p->p2_floor, 1e-6));
  const double margin = g.E * g.h + std::min(reach, 0.5 * (g.z_b - g.z_a));
  t.dz = smin / 40.0;
  t.z_lo = g.z_a - margin;
  const double n = std::ceil(((g.z_b - g.z_a) + 2.0 * margin) / t.dz) + 2.0;
  if (n > (double)(1 << 22)) return MedTab{nullptr, 0, 0.0, 0.0};  // too fine: evaluate directly
  t.n = (int)n;
  return t;
}

Layout layout(const swkb_params* p, const Geometry& g, size_t nlist, bool gfast) {
  Layout L;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    size_t at = o;
    o += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const size_t MR = (size_t)g.M * g.R;
  const size_t ts = p->precision == SWKB_FP64 ? sizeof(double) : sizeof(float);
  L.xi = take(sizeof(double) * g.M);
  L.pbar = take(sizeof(double) * g.M);
  L.e1r = take(sizeof(double) * g.M);
  L.frac = take(sizeof(double) * g.M);
  L.frac_st = take(sizeof(double) * g.M * (size_t)g.S);
  L.tw = take(sizeof(double2) * g.P);
  L.mprm = take(sizeof(double) * p->n_medium_params);
  L.glist = take(sizeof(int) * (nlist ? nlist : 1));
  const size_t nl = gfast ? nlist : 0;
  L.gstage = take(2 * ts * nl * (size_t)(2 * g.S + 1));
  L.gterm = take(2 * ts * nl);
  L.gczl = take(ts * nl * (size_t)waves_per_mode(g));
  const size_t B = (size_t)p->max_batch;
  L.u = take(sizeof(double2) * g.N);
  L.ub = take(B > 1 ? sizeof(double2) * g.N * B : 0);
  L.Y = take(sizeof(double2) * g.P * B);
  L.c = take(sizeof(double2) * g.M * B);
  L.pan = take(B > 1 && use_matrix(p) ? batch_panel_bytes(g, (int)B) : 0);
  L.menergy = take(B > 1 && use_matrix(p) ? sizeof(double) * g.M : 0);
  L.cpol = take(p->precision == SWKB_MIXED ? sizeof(float2) * g.M : 0);
  size_t part_bytes = sizeof(double2) * (size_t)g.N * partial_groups(g) * B;
  if (B > 1 && use_matrix(p)) part_bytes = std::max(part_bytes, batch_part_bytes(g, p->precision, (int)B));
  L.part = take(part_bytes);
  L.tmat = take(use_matrix(p) ? matrix_bytes(p) : 0);
  L.hist = take(p->keep_history ? sizeof(double2) * (size_t)g.N * (size_t)(p->n_screens + 1) : 0);
  L.counters = take(sizeof(unsigned long long) * 32);
  // ray-record slots: two for media that change with x (march and sum overlap)
  L.slot0 = o;
  o = 0;
  L.mtab = take(sizeof(float4) * (size_t)med_table(p, g).n * (2 * g.S + 1));
  L.D = take(ts * MR);
  L.Pp = take(ts * MR);
  L.G = take(ts * MR);
  L.A = take(ts * MR);
  L.cz = take(sizeof(int) * MR);
  L.cidx = take(sizeof(int) * MR);
  L.tstart = take(sizeof(int) * (size_t)g.M * (g.T + 1));
  L.mflag = take(sizeof(int) * g.M);
  L.mcaus = take(sizeof(int) * g.M);
  L.mdead = take(sizeof(int) * g.M);
  L.mwork = take(sizeof(int) * 4 * (size_t)g.M);
  L.wcount = take(sizeof(int) * kWaveCounts * (size_t)g.M * waves_per_mode(g));
  L.slot_bytes = o;
  L.nslots = p->medium_kind == SWKB_MEDIUM_GAUSSSUM ? 2 : 1;
  L.total = L.slot0 + L.slot_bytes * L.nslots;
  return L;
}

swkb_status fail(swkb_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

swkb_status hip_fail(hipError_t e, const char* what) {
  return fail(SWKB_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace
}  // namespace swkb

using namespace swkb;

// Event timing: an event is recorded on the launch stream before and after
// each kernel (class 0 march, 1 scan, 2 fft, 3 superposition, 4 medium table).
enum { kProfMarch = 0, kProfScan = 1, kProfFft = 2, kProfSuper = 3, kProfTable = 4, kProfClasses = 5 };

static int prof_mark(swkb_plan_s* pl, hipStream_t st) {
  if (pl->ev_used == pl->ev_pool.size()) {
    hipEvent_t ev;
    if (hipEventCreate(&ev) != hipSuccess) return -1;
    pl->ev_pool.push_back(ev);
  }
  const int i = (int)pl->ev_used++;
  if (hipEventRecord(pl->ev_pool[i], st) != hipSuccess) return -1;
  return i;
}

template <typename F>
static hipError_t timed(swkb_plan_s* pl, int cls, hipStream_t st, F&& launch) {
  if (!pl->prof_on) return launch();
  const int a = prof_mark(pl, st);
  hipError_t e = launch();
  const int b = prof_mark(pl, st);
  if (a >= 0 && b >= 0) pl->marks.push_back({cls, a, b});
  return e;
}

// The launchers read the active slot's records through pl->rec, pl->wcount
// and pl->mtab (captured by value at each launch).
static void select_slot(swkb_plan_s* pl, int k) {
  const swkb_plan_s::Slot& sl = pl->slots[k];
  pl->rec = sl.rec;
  pl->wcount = sl.wcount;
  pl->mtab = sl.mtab;
  pl->march_valid_q = sl.q;
}

static void set_slot_q(swkb_plan_s* pl, int k, int q) {
  pl->slots[k].q = q;
  if (pl->rec.D == pl->slots[k].rec.D) pl->march_valid_q = q;
}

// March, scan and graph-capture streams shared by every plan on a device.
// A process gets few hardware queues, and streams that share a queue run in
// submission order (an event wait on one holds up the others), so streams of
// its own for every plan would serialise the pipelines of plans created
// later.  Created on first use, kept until the process ends.  Every plan
// orders its work on them with events of its own; each wait refers to an
// event recorded earlier in host order, so sharing cannot deadlock.
struct SharedStreams {
  hipStream_t ms = nullptr, ss = nullptr, cs = nullptr;
};
static std::mutex g_streams_mu;
static std::vector<SharedStreams> g_streams;  // by device

static hipError_t shared_streams(SharedStreams* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_streams_mu);
  if ((int)g_streams.size() <= dev) g_streams.resize(dev + 1);
  SharedStreams& s = g_streams[dev];
  if (!s.ms) {
    SharedStreams n;
    e = hipStreamCreateWithFlags(&n.ms, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&n.ss, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&n.cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (hipStream_t x : {n.ms, n.ss, n.cs})
        if (x) (void)hipStreamDestroy(x);
      return e;
    }
    s = n;
  }
  *out = s;
  return hipSuccess;
}

static void destroy_streams(swkb_plan_s* pl) {
  for (int k = 0; k < 2; ++k) {
    if (pl->ev_ready[k]) (void)hipEventDestroy(pl->ev_ready[k]);
    if (pl->ev_free[k]) (void)hipEventDestroy(pl->ev_free[k]);
    if (pl->ev_marched[k]) (void)hipEventDestroy(pl->ev_marched[k]);
  }
  pl->ms = pl->ss = nullptr;  // shared, not the plan's
  for (int k = 0; k < 2; ++k) pl->ev_ready[k] = pl->ev_free[k] = pl->ev_marched[k] = nullptr;
}

static int slot_of(const swkb_plan_s* pl, int q) { return pl->nslots == 2 ? (q & 1) : 0; }

// Table, march and scan of screen q into slot k on stream st.
static hipError_t march_chain(swkb_plan_s* pl, int q, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (pl->mtab.tab) e = timed(pl, kProfTable, st, [&] { return launch_medium_table(*pl, q, st); });
  if (e == hipSuccess) e = timed(pl, kProfMarch, st, [&] { return launch_march(*pl, q, st); });
  if (e == hipSuccess) e = timed(pl, kProfScan, st, [&] { return launch_scan(*pl, st); });
  return e;
}

// Rays of screen q in the active slot, marched on st if the slot lacks them.
static swkb_status ensure_rays(swkb_plan_s* pl, int q, hipStream_t st) {
  const int k = pl->x_invariant ? 0 : slot_of(pl, q);
  select_slot(pl, k);
  if (pl->x_invariant ? pl->slots[k].q == -2 : pl->slots[k].q == q) return SWKB_OK;
  const hipError_t e = march_chain(pl, q, st);
  if (e != hipSuccess) {
    set_slot_q(pl, k, -1);
    return hip_fail(e, "ray march launch");
  }
  set_slot_q(pl, k, pl->x_invariant ? -2 : q);
  return SWKB_OK;
}

namespace swkb {

// Launch amplitude factors of a patch's rays (device array [R], or NULL),
// set before the plan's first propagation.  A plan whose rays were marched
// when it was built (media that do not depend on x, mode-function matrix)
// marches them again with the factors and rebuilds its matrix; other plans
// with cached rays drop them.
swkb_status set_launch_window(swkb_plan_s* pl, const double* lw, hipStream_t st) {
  pl->lwin = lw;
  if (pl->use_matrix) {
    select_slot(pl, 0);
    hipError_t e = launch_march(*pl, 0, st);
    if (e == hipSuccess) e = launch_scan(*pl, st);
    if (e == hipSuccess) e = launch_build_matrix(*pl, st);
    if (e != hipSuccess) {
      set_slot_q(pl, 0, -1);
      return hip_fail(e, "launch window: ray march");
    }
    set_slot_q(pl, 0, -2);
  } else {
    for (int k = 0; k < pl->nslots; ++k) set_slot_q(pl, k, -1);
  }
  return SWKB_OK;
}

}  // namespace swkb

// Overlap march and sum on two streams: x-varying medium without profiling
// (per-kernel event times need the kernels one after another).
static bool overlap(const swkb_plan_s* pl) {
  return pl->nslots == 2 && pl->ms && !pl->use_matrix && !pl->x_invariant && !pl->prof_on;
}

// Screens [q_begin, q_end) of an x-varying medium with march and scan on
// streams of their own.  Slot k = q & 1 holds screen q's rays.  The
// caller's stream st builds the medium table of screen q (into slot k, once
// the sum of screen q - 2 has released it); the march stream marches screen
// q, the scan stream scans it, and st runs the FFT of screen q (which needs
// only the field) and, after the scan, its sum.  fft(q) and sum(q) launch
// those two parts.
template <typename F, typename G>
static swkb_status pipelined(swkb_plan_s* pl, int q_begin, int q_end, hipStream_t st, F&& fft, G&& sum) {
  hipError_t e = hipSuccess;
  // table of screen q into its slot on st, then the slot is open for the march
  auto prepare = [&](int q) {
    const int k = q & 1;
    select_slot(pl, k);
    hipError_t r = launch_medium_table(*pl, q, st);
    if (r == hipSuccess) r = hipEventRecord(pl->ev_free[k], st);
    return r;
  };
  for (int q = q_begin; q < q_end && q < q_begin + 2 && e == hipSuccess; ++q)
    if (pl->slots[q & 1].q != q) e = prepare(q);
  for (int q = q_begin; q < q_end && e == hipSuccess; ++q) {
    const int k = q & 1;
    select_slot(pl, k);
    const bool march = pl->slots[k].q != q;
    if (march) {
      e = hipStreamWaitEvent(pl->ms, pl->ev_free[k], 0);
      if (e == hipSuccess) e = launch_march(*pl, q, pl->ms);
      if (e == hipSuccess) e = hipEventRecord(pl->ev_marched[k], pl->ms);
      if (e == hipSuccess) e = hipStreamWaitEvent(pl->ss, pl->ev_marched[k], 0);
      if (e == hipSuccess) e = launch_scan(*pl, pl->ss);
      if (e == hipSuccess) e = hipEventRecord(pl->ev_ready[k], pl->ss);
      set_slot_q(pl, k, e == hipSuccess ? q : -1);
    }
    if (e == hipSuccess) e = fft(q);
    if (e == hipSuccess && march) e = hipStreamWaitEvent(st, pl->ev_ready[k], 0);
    if (e == hipSuccess) e = sum(q);
    if (e == hipSuccess && q + 2 < q_end) e = prepare(q + 2);
  }
  if (e != hipSuccess) return hip_fail(e, "screen launch");
  return SWKB_OK;
}

// Screens q_begin .. q_end-1 of one field on stream st (the body of
// swkb_propagate).
static swkb_status enqueue_screens(swkb_plan_s* pl, const void* u_in, int q_begin, int q_end, void* history,
                                   hipStream_t st) {
  const Geometry& g = pl->g;
  pl->sum_fields = 1;
  const double2* src = u_in ? static_cast<const double2*>(u_in) : pl->u;
  auto fft = [&](int) { return timed(pl, kProfFft, st, [&] { return launch_fft_modes(*pl, src, 1, st); }); };
  auto sum = [&](int q) {
    hipError_t e;
    double2* hist = history ? static_cast<double2*>(history) + (size_t)(q - q_begin) * g.N
                    : pl->hist_on   ? pl->H + (size_t)(q + 1) * g.N
                                    : nullptr;
    if (pl->use_matrix)
      e = timed(pl, kProfSuper, st, [&] { return launch_apply_matrix(*pl, pl->u, hist, 1, st); });
    else
      e = timed(pl, kProfSuper, st, [&] { return launch_superpose(*pl, pl->u, hist, 1, st); });
    src = pl->u;
    pl->cur_q = q + 1;
    return e;
  };
  if (overlap(pl)) return pipelined(pl, q_begin, q_end, st, fft, sum);
  for (int q = q_begin; q < q_end; ++q) {
    if (!pl->use_matrix) {
      swkb_status s = ensure_rays(pl, q, st);
      if (s != SWKB_OK) return s;
    }
    hipError_t e = fft(q);
    if (e == hipSuccess) e = sum(q);
    if (e != hipSuccess) return hip_fail(e, "screen launch");
  }
  return SWKB_OK;
}

static void destroy_graphs(swkb_plan_s* pl) {
  for (auto& ge : pl->graphs) {
    (void)hipGraphExecDestroy(ge.exec);
    (void)hipGraphDestroy(ge.graph);
  }
  pl->graphs.clear();
  if (pl->ev_g0) (void)hipEventDestroy(pl->ev_g0);
  if (pl->ev_g1) (void)hipEventDestroy(pl->ev_g1);
  pl->ev_g0 = pl->ev_g1 = nullptr;
  pl->cs = nullptr;  // shared, not the plan's
}

// The same screens through a HIP graph: captured on the plan's capture
// stream the first time a (u_in, q_begin, q_end, history, field buffer)
// combination is seen, replayed afterwards.  The captured sequence marches every screen
// itself (the ray slots are not reused across calls) and holds no memset;
// the caller's stream is joined to the capture stream by events.
static swkb_status propagate_graph(swkb_plan_s* pl, const void* u_in, int q_begin, int q_end, void* history,
                                   hipStream_t st) {
  swkb_plan_s::GraphEntry* hit = nullptr;
  for (auto& ge : pl->graphs)
    if (ge.u_in == u_in && ge.q0 == q_begin && ge.q1 == q_end && ge.hist == history && ge.u == pl->u &&
        ge.hist_on == pl->hist_on)
      hit = &ge;
  // Rays that do not change with x are marched outside the graph, once;
  // other calls (fields between screens) may have put other rays into the
  // slot since, so the check runs before every replay too.
  if (!pl->use_matrix && pl->x_invariant) {
    swkb_status s = ensure_rays(pl, q_begin, st);
    if (s != SWKB_OK) return s;
  }
  hipError_t e = hipSuccess;
  if (!hit) {
    if (pl->graphs.size() >= 4) {
      (void)hipGraphExecDestroy(pl->graphs.front().exec);
      (void)hipGraphDestroy(pl->graphs.front().graph);
      pl->graphs.erase(pl->graphs.begin());
    }
    // the capture starts after the caller's earlier work
    e = hipEventRecord(pl->ev_g0, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(pl->cs, pl->ev_g0, 0);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    if (pl->nslots == 2)
      for (int k = 0; k < 2; ++k) set_slot_q(pl, k, -1);
    e = hipStreamBeginCapture(pl->cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    const int keep_q = pl->cur_q;
    swkb_status s = enqueue_screens(pl, u_in, q_begin, q_end, history, pl->cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(pl->cs, &graph);
    if (s != SWKB_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      pl->cur_q = keep_q;
      for (int k = 0; k < pl->nslots; ++k) set_slot_q(pl, k, -1);
      return s != SWKB_OK ? s : hip_fail(e, "graph capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e, "graph instantiate");
    }
    pl->graphs.push_back({u_in, q_begin, q_end, history, pl->u, pl->hist_on, graph, exec});
    hit = &pl->graphs.back();
  } else {
    e = hipEventRecord(pl->ev_g0, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(pl->cs, pl->ev_g0, 0);
  }
  if (e == hipSuccess) e = hipGraphLaunch(hit->exec, pl->cs);
  if (e == hipSuccess) e = hipEventRecord(pl->ev_g1, pl->cs);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, pl->ev_g1, 0);
  if (e != hipSuccess) return hip_fail(e, "graph launch");
  // host state as after the eager sequence
  pl->cur_q = q_end;
  if (pl->nslots == 2) {
    for (int k = 0; k < 2; ++k) set_slot_q(pl, k, -1);
    for (int q = q_end - 2 > q_begin ? q_end - 2 : q_begin; q < q_end; ++q) set_slot_q(pl, q & 1, q);
    select_slot(pl, (q_end - 1) & 1);
  }
  return SWKB_OK;
}

// Body of swkb_propagate (the caller holds the plan).
swkb_status swkb::propagate_impl(swkb_plan_s* pl, const void* u_in, int q_begin, int q_end, void* history,
                                 hipStream_t st) {
  if (q_begin < 0 || q_end < q_begin || q_end > pl->p.n_screens)
    return fail(SWKB_ERR_ARG, "need 0 <= q_begin <= q_end <= n_screens");
  if (!u_in && pl->cur_q != q_begin)
    return fail(SWKB_ERR_STATE, "u_in is NULL but the plan's field is not on screen q_begin");
  if (q_end == q_begin) {
    if (u_in) {
      hipError_t e = hipMemcpyAsync(pl->u, u_in, sizeof(double2) * pl->g.N, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "field copy");
    }
    pl->cur_q = q_begin;
    return SWKB_OK;
  }
  if (pl->graphs_on && !pl->prof_on) return propagate_graph(pl, u_in, q_begin, q_end, history, st);
  return enqueue_screens(pl, u_in, q_begin, q_end, history, st);
}

// A public call on plan pl that enqueues on stream st (use_stream = false:
// host-only call).  SWKB_ERR_BUSY without running body while another thread
// is inside a call on the plan, or while the previous call's work on
// another stream has not finished; afterwards the end of the call's work is
// marked on st.  Failures are also kept as the plan's last error.
template <typename F>
static swkb_status plan_call(swkb_plan_s* pl, hipStream_t st, bool use_stream, F&& body) {
  PlanGuard guard(&pl->busy);
  if (!guard.held()) {
    set_error("plan is in use by another thread");
    return SWKB_ERR_BUSY;
  }
  if (use_stream && pl->ev_done && pl->has_last && st != pl->last_st &&
      hipEventQuery(pl->ev_done) == hipErrorNotReady) {
    set_error("the plan's previous call is still running on another stream");
    pl->err = g_err;
    return SWKB_ERR_BUSY;
  }
  const swkb_status s = body();
  if (s != SWKB_OK) pl->err = g_err;
  if (use_stream && pl->ev_done) {
    // a stream being captured by the caller gets no marker (its work runs at replay)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    pl->has_last = hipStreamIsCapturing(st, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone &&
                   hipEventRecord(pl->ev_done, st) == hipSuccess;
    pl->last_st = st;
  }
  return s;
}

extern "C" {

size_t swkb_workspace_bytes(const swkb_params* p) {
  if (!validate(p).empty()) return 0;
  const Geometry g = geometry(p);
  std::vector<int> off;
  const std::vector<int> list = gauss_lists(p, &off);
  return layout(p, g, list.size(), gauss_fast(p, off)).total;
}

swkb_status swkb_plan(const swkb_params* p, void* workspace, size_t workspace_bytes, void* hip_stream,
                      swkb_plan_t* out) {
  return plan_impl(p, workspace, workspace_bytes, (hipStream_t)hip_stream, true, out);
}

}  // extern "C"

// Body of swkb_plan.  own_streams = false: the plan creates no streams and no
// events (every kernel then runs on the caller's stream, one after another,
// and the single-stream check is off).
swkb_status swkb::plan_impl(const swkb_params* p, void* workspace, size_t workspace_bytes, hipStream_t st,
                            bool own_streams, swkb_plan_t* out) {
  if (!out) return fail(SWKB_ERR_ARG, "out is NULL");
  *out = nullptr;
  const std::string why = validate(p);
  if (!why.empty()) return fail(SWKB_ERR_ARG, why);
  if (!workspace) return fail(SWKB_ERR_ARG, "workspace is NULL");
  if (((uintptr_t)workspace & 255) != 0) return fail(SWKB_ERR_ARG, "workspace must be 256-byte aligned");
  swkb_plan_s* pl = new (std::nothrow) swkb_plan_s();
  if (!pl) return fail(SWKB_ERR_NOMEM, "host allocation failed");
  try {
    pl->p = *p;
    pl->mparams.assign(p->medium_params, p->medium_params + p->n_medium_params);
    pl->p.medium_params = pl->mparams.data();
    pl->g = geometry(p);
    pl->precision = p->precision;
    pl->x_invariant = p->medium_kind != SWKB_MEDIUM_GAUSSSUM;
    pl->march_valid_q = -1;
    pl->cur_q = -1;
    const Geometry& g = pl->g;
    const std::vector<int> list = gauss_lists(p, &pl->goff);
    pl->gfast = gauss_fast(p, pl->goff) ? 1 : 0;
    pl->tab_S = p->rk4_steps;
    const Layout L = layout(p, g, list.size(), pl->gfast != 0);
    if (workspace_bytes < L.total) {
      delete pl;
      return fail(SWKB_ERR_NOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    }
    char* ws = static_cast<char*>(workspace);
    pl->xi = reinterpret_cast<double*>(ws + L.xi);
    pl->pbar = reinterpret_cast<double*>(ws + L.pbar);
    pl->e1r = reinterpret_cast<double*>(ws + L.e1r);
    pl->frac = reinterpret_cast<double*>(ws + L.frac);
    pl->frac_st = reinterpret_cast<double*>(ws + L.frac_st);
    pl->tw = reinterpret_cast<double2*>(ws + L.tw);
    pl->mprm = reinterpret_cast<double*>(ws + L.mprm);
    pl->glist = reinterpret_cast<int*>(ws + L.glist);
    pl->gstage = ws + L.gstage;
    pl->gterm = ws + L.gterm;
    pl->gczl = ws + L.gczl;
    pl->u = reinterpret_cast<double2*>(ws + L.u);
    // buffers of zero size share their offset with the next one: leave them unset
    pl->ub = p->max_batch > 1 ? reinterpret_cast<double2*>(ws + L.ub) : nullptr;
    pl->pan = p->max_batch > 1 && use_matrix(p) ? static_cast<void*>(ws + L.pan) : nullptr;
    pl->menergy = p->max_batch > 1 && use_matrix(p) ? reinterpret_cast<double*>(ws + L.menergy) : nullptr;
    pl->cpol = p->precision == SWKB_MIXED ? reinterpret_cast<float2*>(ws + L.cpol) : nullptr;
    pl->max_batch = p->max_batch;
    pl->sum_fields = 1;
    pl->Y = reinterpret_cast<double2*>(ws + L.Y);
    pl->c = reinterpret_cast<double2*>(ws + L.c);
    pl->part = reinterpret_cast<double2*>(ws + L.part);
    pl->use_matrix = use_matrix(p) ? 1 : 0;
    pl->tmat = ws + L.tmat;
    pl->nslots = L.nslots;
    for (int k = 0; k < 2; ++k) {
      char* sb = ws + L.slot0 + L.slot_bytes * (k < L.nslots ? k : 0);
      swkb_plan_s::Slot& sl = pl->slots[k];
      sl.rec.D = sb + L.D;
      sl.rec.Pp = sb + L.Pp;
      sl.rec.G = sb + L.G;
      sl.rec.A = sb + L.A;
      sl.rec.cz = reinterpret_cast<int*>(sb + L.cz);
      sl.rec.cidx = reinterpret_cast<int*>(sb + L.cidx);
      sl.rec.tstart = reinterpret_cast<int*>(sb + L.tstart);
      sl.rec.mflag = reinterpret_cast<int*>(sb + L.mflag);
      sl.rec.mcaus = reinterpret_cast<int*>(sb + L.mcaus);
      sl.rec.mdead = reinterpret_cast<int*>(sb + L.mdead);
      sl.rec.mwork = reinterpret_cast<int*>(sb + L.mwork);
      sl.wcount = reinterpret_cast<int*>(sb + L.wcount);
      sl.mtab = med_table(p, g);
      if (sl.mtab.n > 0) {
        sl.mtab.tab = reinterpret_cast<const float4*>(sb + L.mtab);
      }
      sl.q = -1;
    }
    select_slot(pl, 0);
    pl->ms = nullptr;
    pl->cs = nullptr;
    pl->ev_g0 = pl->ev_g1 = nullptr;
    pl->graphs_on = 0;
    pl->ss = nullptr;
    for (int k = 0; k < 2; ++k) pl->ev_ready[k] = pl->ev_free[k] = pl->ev_marched[k] = nullptr;
    if (pl->nslots == 2 && own_streams) {
      SharedStreams ss;
      bool ok = shared_streams(&ss) == hipSuccess;
      pl->ms = ss.ms;
      pl->ss = ss.ss;
      for (int k = 0; k < 2 && ok; ++k)
        ok = hipEventCreateWithFlags(&pl->ev_ready[k], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&pl->ev_free[k], hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&pl->ev_marched[k], hipEventDisableTiming) == hipSuccess;
      if (!ok) {
        destroy_streams(pl);
        delete pl;
        return fail(SWKB_ERR_DEVICE, "swkb_plan: stream or event creation failed");
      }
    }
    pl->prof_on = 0;
    pl->ev_used = 0;
    pl->counters = reinterpret_cast<unsigned long long*>(ws + L.counters);
    pl->counters_scratch = pl->counters + 16;
    pl->H = p->keep_history ? reinterpret_cast<double2*>(ws + L.hist) : nullptr;
    pl->hvalid.assign(p->keep_history ? (size_t)p->n_screens + 1 : 0, 0);
    pl->hist_on = 0;
    pl->busy = 0;
    pl->last_st = nullptr;
    pl->has_last = 0;
    pl->ev_done = nullptr;
    if (own_streams && hipEventCreateWithFlags(&pl->ev_done, hipEventDisableTiming) != hipSuccess) {
      destroy_streams(pl);
      delete pl;
      return fail(SWKB_ERR_DEVICE, "swkb_plan: event creation failed");
    }

    // mode tables: xi_n = 2 pi n / (k P h); reference pbar and range phase
    std::vector<double> xi(g.M), pbar(g.M), e1r(g.M), frac(g.M);
    for (int j = 0; j < g.M; ++j) {
      const int n = j - g.M / 2;
      xi[j] = 2.0 * M_PI * n / (g.k * (double)g.P * g.h);
      const double pb2 = p->eps_ref - xi[j] * xi[j];
      if (pb2 >= p->p2_floor && pb2 > 0.0) {
        pbar[j] = std::sqrt(pb2);
        e1r[j] = p->eps_ref - 1.0;
      } else {
        const double f = p->p2_floor > 0.0 ? p->p2_floor : 1e-2;
        pbar[j] = std::sqrt(f);
        e1r[j] = (f + xi[j] * xi[j]) - 1.0;
      }
      const long double turns = (long double)pbar[j] * (long double)g.dx * (long double)g.k / (2.0L * M_PIl);
      frac[j] = (double)(turns - floorl(turns));
    }
    std::vector<double2> tw(g.P);
    for (int t = 0; t < g.P; ++t) {
      const long double a = 2.0L * M_PIl * (long double)t / (long double)g.P;
      tw[t] = make_double2((double)cosl(a), (double)-sinl(a));
    }
    hipError_t e = hipSuccess;
    auto put = [&](void* dst, const void* src, size_t n) {
      if (e == hipSuccess && n) e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, st);
    };
    put(pl->xi, xi.data(), sizeof(double) * g.M);
    put(pl->pbar, pbar.data(), sizeof(double) * g.M);
    put(pl->e1r, e1r.data(), sizeof(double) * g.M);
    put(pl->frac, frac.data(), sizeof(double) * g.M);
    put(pl->tw, tw.data(), sizeof(double2) * g.P);
    put(pl->mprm, pl->mparams.data(), sizeof(double) * p->n_medium_params);
    put(pl->glist, list.data(), sizeof(int) * list.size());
    // Gaussian-sum bump tables per screen and RK4 stage position
    std::vector<double> gst64, gtm64, gcz64;
    std::vector<float> gst32, gtm32, gcz32;
    if (pl->gfast) {
      const int ns = 2 * g.S + 1;
      const double* mp = pl->mparams.data();
      const double hx2 = 0.5 * p->dx / p->rk4_steps;
      const double log2e = 1.4426950408889634;
      for (int q = 0; q < p->n_screens; ++q) {
        const int o = pl->goff[q], nl = pl->goff[q + 1] - o;
        const double x_q = p->x0 + q * p->dx;
        for (int k = 0; k < ns; ++k) {
          const double x = x_q + k * hx2;
          for (int i = 0; i < nl; ++i) {
            const double* b = mp + 1 + 4 * list[o + i];
            const double ddx = x - b[2], s2 = b[1] * b[1];
            const double ax = b[0] * std::exp(-ddx * ddx / (2.0 * s2)), cut = 64.0 * s2 - ddx * ddx;
            if (p->precision == SWKB_FP64) { gst64.push_back(ax); gst64.push_back(cut); }
            else { gst32.push_back((float)ax); gst32.push_back((float)cut); }
          }
        }
        for (int i = 0; i < nl; ++i) {
          const double* b = mp + 1 + 4 * list[o + i];
          const double s2 = b[1] * b[1];
          if (p->precision == SWKB_FP64) { gtm64.push_back(-0.5 / s2); gtm64.push_back(1.0 / s2); }
          else { gtm32.push_back((float)(-0.5 * log2e / s2)); gtm32.push_back((float)(1.0 / s2)); }
        }
        const int wpm = waves_per_mode(g);
        for (int w = 0; w < wpm; ++w) {
          const double zw = g.z_a + (double)(w * 64 * g.rho - g.E) * g.h;
          for (int i = 0; i < nl; ++i) {
            const double czl = mp[1 + 4 * list[o + i] + 3] - zw;
            if (p->precision == SWKB_FP64) gcz64.push_back(czl);
            else gcz32.push_back((float)czl);
          }
        }
      }
      if (p->precision == SWKB_FP64) {
        put(pl->gstage, gst64.data(), sizeof(double) * gst64.size());
        put(pl->gterm, gtm64.data(), sizeof(double) * gtm64.size());
      } else {
        put(pl->gstage, gst32.data(), sizeof(float) * gst32.size());
        put(pl->gterm, gtm32.data(), sizeof(float) * gtm32.size());
      }
      if (p->precision == SWKB_FP64) put(pl->gczl, gcz64.data(), sizeof(double) * gcz64.size());
      else put(pl->gczl, gcz32.data(), sizeof(float) * gcz32.size());
    }
    if (e == hipSuccess) e = hipMemsetAsync(pl->counters, 0, sizeof(unsigned long long) * 32, st);
    if (e == hipSuccess && pl->use_matrix) {
      // x-invariant medium: march once and tabulate the mode functions
      e = launch_march(*pl, 0, st);
      if (e == hipSuccess) e = launch_scan(*pl, st);
      if (e == hipSuccess) e = launch_build_matrix(*pl, st);
      if (e == hipSuccess) set_slot_q(pl, 0, -2);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // host tables go out of scope
    if (e != hipSuccess) {
      destroy_streams(pl);
      (void)hipEventDestroy(pl->ev_done);
      delete pl;
      return hip_fail(e, "swkb_plan upload");
    }
  } catch (const std::exception& ex) {
    destroy_streams(pl);
    if (pl->ev_done) (void)hipEventDestroy(pl->ev_done);
    delete pl;
    return fail(SWKB_ERR_NOMEM, std::string("swkb_plan: ") + ex.what());
  }
  *out = pl;
  return SWKB_OK;
}

extern "C" {

swkb_status swkb_propagate(swkb_plan_t pl, const void* u_in, int32_t q_begin, int32_t q_end, void* history,
                           void* hip_stream) {
  if (!pl) return fail(SWKB_ERR_ARG, "plan is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  return plan_call(pl, st, true, [&]() -> swkb_status {
    pl->hist_on = pl->H != nullptr;
    const swkb_status s = propagate_impl(pl, u_in, q_begin, q_end, history, st);
    pl->hist_on = 0;
    if (s != SWKB_OK || !pl->H) return s;
    // kept history: the input screen, and the caller's history rows (the
    // kernels wrote the plan's rows directly when the caller gave none)
    const size_t row = sizeof(double2) * pl->g.N;
    hipError_t e = hipSuccess;
    if (u_in)
      e = hipMemcpyAsync(pl->H + (size_t)q_begin * pl->g.N, u_in, row, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && history && q_end > q_begin)
      e = hipMemcpyAsync(pl->H + (size_t)(q_begin + 1) * pl->g.N, history, row * (q_end - q_begin),
                         hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "kept history copy");
    for (int q = q_begin; q <= q_end; ++q) pl->hvalid[q] = 1;
    return SWKB_OK;
  });
}

swkb_status swkb_propagate_batch(swkb_plan_t pl, const void* u_in, int32_t batch, int32_t q_begin, int32_t q_end,
                                 void* history, void* u_out, void* hip_stream) {
  if (!pl || !u_in) return fail(SWKB_ERR_ARG, "plan or u_in is NULL");
  if (batch < 1 || batch > pl->max_batch) return fail(SWKB_ERR_ARG, "need 1 <= batch <= max_batch");
  if (q_begin < 0 || q_end <= q_begin || q_end > pl->p.n_screens)
    return fail(SWKB_ERR_ARG, "need 0 <= q_begin < q_end <= n_screens");
  hipStream_t st = (hipStream_t)hip_stream;
  return plan_call(pl, st, true, [&]() -> swkb_status {
    const Geometry& g = pl->g;
    pl->hist_on = 0;  // a batch never writes the plan's kept history
    if (batch == 1) {
      // one field: the single-field kernels, without touching the plan's field
      double2* keep = pl->u;
      const int keep_q = pl->cur_q;
      swkb_status s = SWKB_OK;
      if (!pl->ub) {
        // no separate batch buffer (max_batch == 1): the single-field state is consumed
        s = propagate_impl(pl, u_in, q_begin, q_end, history, st);
        if (s == SWKB_OK && u_out) {
          hipError_t e = hipMemcpyAsync(u_out, pl->u, sizeof(double2) * g.N, hipMemcpyDeviceToDevice, st);
          if (e != hipSuccess) s = hip_fail(e, "field copy");
        }
        pl->cur_q = -1;
        return s;
      }
      pl->u = pl->ub;
      s = propagate_impl(pl, u_in, q_begin, q_end, history, st);
      if (s == SWKB_OK && u_out) {
        hipError_t e = hipMemcpyAsync(u_out, pl->u, sizeof(double2) * g.N, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) s = hip_fail(e, "field copy");
      }
      pl->u = keep;
      pl->cur_q = keep_q;
      return s;
    }
    const double2* src = static_cast<const double2*>(u_in);
    pl->sum_fields = batch;
    auto fft = [&](int) { return timed(pl, kProfFft, st, [&] { return launch_fft_modes(*pl, src, batch, st); }); };
    auto sum = [&](int q) {
      hipError_t e;
      double2* hist = history ? static_cast<double2*>(history) + (size_t)(q - q_begin) * batch * g.N : nullptr;
      if (pl->use_matrix)
        e = timed(pl, kProfSuper, st, [&] { return launch_apply_matrix(*pl, pl->ub, hist, batch, st); });
      else
        e = timed(pl, kProfSuper, st, [&] { return launch_superpose(*pl, pl->ub, hist, batch, st); });
      src = pl->ub;
      return e;
    };
    if (overlap(pl)) {
      swkb_status s = pipelined(pl, q_begin, q_end, st, fft, sum);
      if (s != SWKB_OK) return s;
    } else {
      for (int q = q_begin; q < q_end; ++q) {
        if (!pl->use_matrix) {
          swkb_status s = ensure_rays(pl, q, st);
          if (s != SWKB_OK) return s;
        }
        hipError_t e = fft(q);
        if (e == hipSuccess) e = sum(q);
        if (e != hipSuccess) return hip_fail(e, "batched screen launch");
      }
    }
    if (u_out) {
      hipError_t e = hipMemcpyAsync(u_out, pl->ub, sizeof(double2) * g.N * batch, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "field copy");
    }
    return SWKB_OK;
  });
}

swkb_status swkb_propagate_stations(swkb_plan_t pl, const void* u, int32_t q, const int32_t* stations, int32_t n,
                                    void* out, void* hip_stream) {
  if (!pl || !u || !stations || !out || n < 1) return fail(SWKB_ERR_ARG, "NULL argument or n < 1");
  if (q < 0 || q >= pl->p.n_screens) return fail(SWKB_ERR_ARG, "q out of range");
  const Geometry& g = pl->g;
  for (int s = 0; s < n; ++s)
    if (stations[s] < 1 || stations[s] > g.S) return fail(SWKB_ERR_ARG, "stations must be in [1, rk4_steps]");
  hipStream_t st = (hipStream_t)hip_stream;
  return plan_call(pl, st, true, [&]() -> swkb_status {
  const double hx = pl->p.dx / pl->p.rk4_steps;
  const int k = pl->x_invariant ? 0 : slot_of(pl, q);  // slot the station rays go through
  select_slot(pl, k);
  try {
    // range phase frac(pbar * i hx / lambda) of every mode at every station
    std::vector<double> pbar(g.M), fr((size_t)n * g.M);
    hipError_t e = hipMemcpy(pbar.data(), pl->pbar, sizeof(double) * g.M, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "stations");
    for (int s = 0; s < n; ++s) {
      const double dxs = stations[s] * hx;
      for (int j = 0; j < g.M; ++j) {
        const long double turns = (long double)pbar[j] * (long double)dxs * (long double)g.k / (2.0L * M_PIl);
        fr[(size_t)s * g.M + j] = (double)(turns - floorl(turns));
      }
    }
    e = launch_fft_modes(*pl, static_cast<const double2*>(u), 1, st);
    for (int s0 = 0; s0 < n && e == hipSuccess; s0 += g.S) {
      const int cnt = n - s0 < g.S ? n - s0 : g.S;
      e = hipMemcpyAsync(pl->frac_st, fr.data() + (size_t)s0 * g.M, sizeof(double) * g.M * cnt,
                         hipMemcpyHostToDevice, st);
      for (int s = s0; s < s0 + cnt && e == hipSuccess; ++s) {
        swkb_plan_s tmp = *pl;  // same plan, a screen of width i hx marched with i steps
        tmp.sum_fields = 1;
        tmp.g.S = stations[s];
        tmp.g.dx = stations[s] * hx;
        tmp.frac = pl->frac_st + (size_t)(s - s0) * g.M;
        tmp.counters = pl->counters_scratch;
        tmp.use_matrix = 0;
        e = launch_medium_table(tmp, q, st);
        if (e == hipSuccess) e = launch_march(tmp, q, st);
        if (e == hipSuccess) e = launch_scan(tmp, st);
        if (e == hipSuccess)
          e = launch_superpose(tmp, static_cast<double2*>(out) + (size_t)s * g.N, nullptr, 1, st);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(st);  // host phase tables go out of scope
    }
    if (e != hipSuccess) return hip_fail(e, "stations");
    // the records now hold station rays: re-establish the plan's own march
    set_slot_q(pl, k, -1);
    if (pl->use_matrix) {
      e = launch_march(*pl, 0, st);
      if (e == hipSuccess) e = launch_scan(*pl, st);
      if (e != hipSuccess) return hip_fail(e, "stations");
      set_slot_q(pl, k, -2);
    }
  } catch (const std::exception& ex) {
    return fail(SWKB_ERR_NOMEM, std::string("stations: ") + ex.what());
  }
  return SWKB_OK;
  });
}

swkb_status swkb_field(swkb_plan_t pl, int32_t q, void* out, void* hip_stream) {
  if (!pl || !out) return fail(SWKB_ERR_ARG, "plan or out is NULL");
  if (q < -1 || q > pl->p.n_screens) return fail(SWKB_ERR_ARG, "q must be in [-1, n_screens]");
  hipStream_t st = (hipStream_t)hip_stream;
  return plan_call(pl, st, true, [&]() -> swkb_status {
    const double2* src = nullptr;
    if (q == -1 || q == pl->cur_q) {
      if (pl->cur_q < 0) return fail(SWKB_ERR_STATE, "no field yet: call swkb_propagate first");
      src = pl->u;
    } else if (pl->H && pl->hvalid[q]) {
      src = pl->H + (size_t)q * pl->g.N;
    } else {
      return fail(SWKB_ERR_STATE, pl->H ? "screen q has not been reached by a propagation of this plan"
                                        : "only the current screen is held (keep_history = 0)");
    }
    hipError_t e = hipMemcpyAsync(out, src, sizeof(double2) * pl->g.N, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "field copy");
    return SWKB_OK;
  });
}

int32_t swkb_current_screen(swkb_plan_t pl) { return pl ? pl->cur_q : -1; }

swkb_status swkb_diagnostics(swkb_plan_t pl, void* hip_stream, swkb_counters* out) {
  if (!pl || !out) return fail(SWKB_ERR_ARG, "plan or out is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  return plan_call(pl, st, true, [&]() -> swkb_status {
    unsigned long long h[11];
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(h, pl->counters, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "diagnostics");
    out->caustic_rays = (int64_t)h[0];
    out->dead_rays = (int64_t)h[1];
    out->folded_modes = (int64_t)h[2];
    out->significant = (int64_t)h[3];
    out->screens = (int64_t)h[4];
    out->rhs_evals = (int64_t)h[5];
    out->medium_evals = (int64_t)h[6];
    out->medium_terms = (int64_t)h[7];
    out->table_evals = (int64_t)h[8];
    out->evanescent_modes = (int64_t)h[9];
    out->significant_evanescent = (int64_t)h[10];
    if (out->significant > 0) return fail(SWKB_ERR_CAUSTIC, "a significant mode met a caustic inside a screen");
    if (out->significant_evanescent > 0)
      return fail(SWKB_ERR_EVANESCENT, "a significant mode had no live ray (evanescent)");
    return SWKB_OK;
  });
}

swkb_status swkb_graphs(swkb_plan_t pl, int32_t enable) {
  if (!pl) return fail(SWKB_ERR_ARG, "plan is NULL");
  return plan_call(pl, nullptr, false, [&]() -> swkb_status {
    if (enable && !pl->cs) {
      SharedStreams ss;
      hipError_t e = shared_streams(&ss);
      pl->cs = ss.cs;
      if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_g0, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_g1, hipEventDisableTiming);
      if (e != hipSuccess) {
        destroy_graphs(pl);
        return hip_fail(e, "graph stream");
      }
    }
    if (!enable) {
      // the plan's streams may still run a replay: wait before releasing the graphs
      if (pl->cs) (void)hipStreamSynchronize(pl->cs);
      destroy_graphs(pl);
    }
    pl->graphs_on = enable ? 1 : 0;
    return SWKB_OK;
  });
}

swkb_status swkb_profile(swkb_plan_t pl, int32_t enable) {
  if (!pl) return fail(SWKB_ERR_ARG, "plan is NULL");
  return plan_call(pl, nullptr, false, [&]() -> swkb_status {
    pl->prof_on = enable ? 1 : 0;
    return SWKB_OK;
  });
}

swkb_status swkb_profile_read(swkb_plan_t pl, void* hip_stream, swkb_timing* out) {
  if (!pl || !out) return fail(SWKB_ERR_ARG, "plan or out is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  return plan_call(pl, st, true, [&]() -> swkb_status {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "profile read");
    double ms[kProfClasses] = {0, 0, 0, 0, 0};
    int64_t n[kProfClasses] = {0, 0, 0, 0, 0};
    for (const auto& mk : pl->marks) {
      float t = 0.f;
      e = hipEventSynchronize(pl->ev_pool[mk.b]);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, pl->ev_pool[mk.a], pl->ev_pool[mk.b]);
      if (e != hipSuccess) return hip_fail(e, "profile read");
      ms[mk.cls] += t;
      n[mk.cls] += 1;
    }
    pl->marks.clear();
    pl->ev_used = 0;
    out->march_ms = ms[kProfMarch];
    out->scan_ms = ms[kProfScan];
    out->fft_ms = ms[kProfFft];
    out->superpose_ms = ms[kProfSuper];
    out->march_launches = n[kProfMarch];
    out->scan_launches = n[kProfScan];
    out->fft_launches = n[kProfFft];
    out->superpose_launches = n[kProfSuper];
    out->table_ms = ms[kProfTable];
    out->table_launches = n[kProfTable];
    return SWKB_OK;
  });
}

void swkb_destroy(swkb_plan_t pl) {
  if (!pl) return;
  for (hipEvent_t ev : pl->ev_pool) (void)hipEventDestroy(ev);
  if (pl->cs) (void)hipStreamSynchronize(pl->cs);
  destroy_graphs(pl);
  destroy_streams(pl);
  if (pl->ev_done) (void)hipEventDestroy(pl->ev_done);
  delete pl;
}

const char* swkb_status_string(swkb_status s) {
  switch (s) {
    case SWKB_OK: return "ok";
    case SWKB_ERR_ARG: return "invalid argument";
    case SWKB_ERR_NOMEM: return "workspace too small or out of memory";
    case SWKB_ERR_DEVICE: return "HIP runtime error";
    case SWKB_ERR_CAUSTIC: return "caustic inside a screen";
    case SWKB_ERR_STATE: return "call out of order";
    case SWKB_ERR_EVANESCENT: return "a significant mode was evanescent";
    case SWKB_ERR_BUSY: return "plan busy";
  }
  return "unknown status";
}

const char* swkb_last_error(void) { return g_err.c_str(); }

const char* swkb_plan_error(swkb_plan_t pl) { return pl ? pl->err.c_str() : ""; }

size_t swkb_footprint(const swkb_params* p) {
  const size_t ws = swkb_workspace_bytes(p);
  if (ws == 0) return 0;
  return ws + sizeof(double2) * (size_t)p->n_z + 4096;
}

swkb_status swkb_stage_modes(swkb_plan_t pl, const void* u, void* c, void* hip_stream) {
  if (!pl || !u || !c) return fail(SWKB_ERR_ARG, "NULL argument");
  hipStream_t st = (hipStream_t)hip_stream;
  return plan_call(pl, st, true, [&]() -> swkb_status {
    hipError_t e = launch_fft_modes(*pl, static_cast<const double2*>(u), 1, st);
    if (e == hipSuccess) e = hipMemcpyAsync(c, pl->c, sizeof(double2) * pl->g.M, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "stage modes");
    return SWKB_OK;
  });
}

swkb_status swkb_stage_rays(swkb_plan_t pl, int32_t q, void* Z, void* psi, void* qz, void* amp, void* flag,
                            void* hip_stream) {
  if (!pl || !Z || !psi || !qz || !amp || !flag) return fail(SWKB_ERR_ARG, "NULL argument");
  if (q < 0 || q >= pl->p.n_screens) return fail(SWKB_ERR_ARG, "q out of range");
  hipStream_t st = (hipStream_t)hip_stream;
  return plan_call(pl, st, true, [&]() -> swkb_status {
    swkb_status s = ensure_rays(pl, q, st);
    if (s != SWKB_OK) return s;
    hipError_t e = launch_export_rays(*pl, q, static_cast<double*>(Z), static_cast<double*>(psi),
                                      static_cast<double*>(qz), static_cast<double*>(amp), static_cast<int*>(flag),
                                      st);
    if (e != hipSuccess) return hip_fail(e, "stage rays");
    return SWKB_OK;
  });
}

int32_t swkb_num_rays(swkb_plan_t pl) { return pl ? pl->g.R : 0; }

int32_t swkb_uses_matrix(swkb_plan_t pl) { return pl ? pl->use_matrix : 0; }

}  // extern "C"
