// Many problems in media that do not depend on x, carried across their
// screens together (Algorithm 1 on each): every screen step is one launch
// per stage for all problems still running (FFT column pass, FFT row pass,
// mode-function matrix times modes, exit epilogue).  The problem table and
// one workgroup map per stage live in device memory; a map entry is
// problem << 20 | local workgroup.  Problems sit in the table by screen
// count, largest first, so the problems running at step q are a prefix of
// the table and a stage's launch at step q covers the first off[n(q)]
// entries of its map.  Launch shapes per size class come from the
// autotuner (swkb_multi_tune) or the caller; the defaults are those of the
// single-problem path, which keeps each field bit-identical to a separate
// swkb_propagate.
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "swkb_internal.h"

namespace {

using swkb::Geometry;
using swkb::MultiProblem;

constexpr int kMapShift = 20;
constexpr int kMaxProblems = 4095;  // problem index in the upper 12 bits of a map entry
enum { kCols = 0, kRows = 1, kApply = 2, kFin = 3, kKinds = 4 };

swkb_status fail(swkb_status s, const std::string& msg) {
  swkb::set_error(msg);
  return s;
}

swkb_status hip_fail(hipError_t e, const char* what) {
  swkb::set_error(std::string(what) + ": " + hipGetErrorString(e));
  return SWKB_ERR_DEVICE;
}

}  // namespace

struct swkb_multi_s {
  std::vector<swkb_plan_s*> plans;  // caller order
  std::vector<int> order;           // table slot -> caller index
  std::vector<int> cls;             // table slot -> size class
  std::vector<int> na;              // na[q]: problems still running at step q
  int qmax = 0;
  swkb_multi_tuning tun{};
  std::vector<MultiProblem> hp;     // problem table (slot order), without u_in / hist
  std::vector<int> off[kKinds];     // workgroup prefix sums over the table, [n + 1] each
  size_t lds_cols = 0, lds_rows = 0;
  // device memory
  MultiProblem* d_prob = nullptr;
  int4* d_counts = nullptr;         // [qmax]: map entries of the four stages at each step
  int* d_ctr = nullptr;             // [4 qmax]: the persistent launch's stage counters
  int persist_blocks = 0;           // grid of the last persistent launch
  unsigned* d_map = nullptr;
  size_t map_cap = 0;               // entries
  size_t map_base[kKinds] = {0, 0, 0, 0};
  double2* d_part = nullptr;
  size_t part_cap = 0;              // double2 elements
  MultiProblem* h_stage = nullptr;  // pinned staging of the problem table
  hipEvent_t ev_stage = nullptr;    // the last staging copy has been done
  hipEvent_t ev_done = nullptr;     // the last call's work has been done
  hipEvent_t t0 = nullptr, t1 = nullptr;
  // graph of the whole step sequence
  hipStream_t cs = nullptr;
  hipEvent_t g0 = nullptr, g1 = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

int class_of(const swkb_multi_s* m, int n_z) {
  for (int c = 0; c < m->tun.n_classes; ++c)
    if (m->tun.class_n_z[c] == n_z) return c;
  return -1;
}

int max_groups(const Geometry& g) { return (g.M + 3) / 4; }

// Workgroups of stage `kind` for a problem with the given shapes.
int stage_blocks(int kind, const MultiProblem& p) {
  switch (kind) {
    case kCols: return p.g.P2 / p.CA;
    case kRows: return p.g.P1 / p.RB;
    case kApply: return p.fp64 ? (p.g.T / p.sub) * p.groups : (p.g.N / 512) * p.groups;
    default: return swkb::finalize_blocks(p.g);
  }
}

void drop_graph(swkb_multi_s* m) {
  if (m->exec) (void)hipGraphExecDestroy(m->exec);
  if (m->graph) (void)hipGraphDestroy(m->graph);
  m->exec = nullptr;
  m->graph = nullptr;
}

// Device buffers of at least the given sizes (waits for the group's earlier
// work before freeing anything).
hipError_t reserve(swkb_multi_s* m, size_t map_entries, size_t part_elems) {
  hipError_t e = hipSuccess;
  if (map_entries > m->map_cap || part_elems > m->part_cap) {
    e = hipEventSynchronize(m->ev_done);
    if (e != hipSuccess) return e;
    drop_graph(m);
  }
  if (map_entries > m->map_cap) {
    if (m->d_map) (void)hipFree(m->d_map);
    m->d_map = nullptr;
    m->map_cap = 0;
    e = hipMalloc(reinterpret_cast<void**>(&m->d_map), sizeof(unsigned) * map_entries);
    if (e != hipSuccess) return e;
    m->map_cap = map_entries;
  }
  if (part_elems > m->part_cap) {
    if (m->d_part) (void)hipFree(m->d_part);
    m->d_part = nullptr;
    m->part_cap = 0;
    e = hipMalloc(reinterpret_cast<void**>(&m->d_part), sizeof(double2) * part_elems);
    if (e != hipSuccess) return e;
    m->part_cap = part_elems;
  }
  return hipSuccess;
}

// Problem table and workgroup maps from the current tuning (host), then
// uploaded with a synchronous copy.
hipError_t build_tables(swkb_multi_s* m) {
  const int n = (int)m->plans.size();
  size_t part_elems = 0;
  for (int k = 0; k < kKinds; ++k) m->off[k].assign(n + 1, 0);
  m->lds_cols = m->lds_rows = 0;
  for (int s = 0; s < n; ++s) {
    const swkb_plan_s* pl = m->plans[m->order[s]];
    const Geometry& g = pl->g;
    const int c = m->cls[s];
    const bool fp64 = pl->precision == SWKB_FP64;
    // FP64 problems keep the single-problem product blocking (the tuning
    // shapes the complex64 products)
    const int fe = m->tun.fft_elems[c];
    const int gr = fp64 ? swkb::apply_f64_groups(g) : std::min(m->tun.apply_groups[c], max_groups(g));
    MultiProblem& p = m->hp[s];
    p.g = g;
    p.ep = swkb::epi_of(*pl);
    p.rec = pl->rec;
    p.tw = pl->tw;
    p.Y = pl->Y;
    p.c = pl->c;
    p.fp64 = fp64 ? 1 : 0;
    p.sub = fp64 ? swkb::apply_f64_sub(g) : 0;
    p.tmat = fp64 ? nullptr : static_cast<const float4*>(pl->tmat);
    p.tmat64 = fp64 ? static_cast<const double2*>(pl->tmat) : nullptr;
    p.part = nullptr;  // set below
    p.u = pl->u;
    p.u_in = nullptr;
    p.hist = nullptr;
    p.counters = pl->counters;
    p.logP1 = swkb::ilog2(g.P1);
    p.logP2 = swkb::ilog2(g.P2);
    swkb::fft_blocking(g, fe, &p.CA, &p.RB);
    p.groups = gr;
    m->lds_cols = std::max(m->lds_cols, sizeof(double2) * (size_t)(p.CA * g.P1 + g.P1 / 2));
    m->lds_rows = std::max(m->lds_rows, sizeof(double2) * (size_t)(p.RB * g.P2 + g.P2 / 2));
    for (int k = 0; k < kKinds; ++k) m->off[k][s + 1] = m->off[k][s] + stage_blocks(k, p);
    part_elems += (size_t)gr * g.N;
  }
  size_t entries = 0;
  for (int k = 0; k < kKinds; ++k) {
    m->map_base[k] = entries;
    entries += (size_t)m->off[k][n];
  }
  hipError_t e = reserve(m, entries, part_elems);
  if (e != hipSuccess) return e;
  size_t po = 0;
  for (int s = 0; s < n; ++s) {
    m->hp[s].part = m->d_part + po;
    po += (size_t)m->hp[s].groups * m->hp[s].g.N;
  }
  std::vector<unsigned> map(entries);
  for (int k = 0; k < kKinds; ++k)
    for (int s = 0; s < n; ++s)
      for (int b = m->off[k][s]; b < m->off[k][s + 1]; ++b)
        map[m->map_base[k] + b] = ((unsigned)s << kMapShift) | (unsigned)(b - m->off[k][s]);
  e = hipMemcpy(m->d_map, map.data(), sizeof(unsigned) * entries, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_prob, m->hp.data(), sizeof(MultiProblem) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    std::vector<int4> cnt(m->qmax);
    for (int q = 0; q < m->qmax; ++q) {
      const int a = m->na[q];
      cnt[q] = make_int4(m->off[kCols][a], m->off[kRows][a], m->off[kApply][a], m->off[kFin][a]);
    }
    e = hipMemcpy(m->d_counts, cnt.data(), sizeof(int4) * m->qmax, hipMemcpyHostToDevice);
  }
  return e;
}

const unsigned* map_of(const swkb_multi_s* m, int kind) { return m->d_map + m->map_base[kind]; }

// The whole step sequence on stream st.
hipError_t enqueue_steps(swkb_multi_s* m, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int q = 0; q < m->qmax && e == hipSuccess; ++q) {
    const int n = m->na[q];
    e = swkb::launch_fft_multi(m->d_prob, map_of(m, kCols), m->off[kCols][n], map_of(m, kRows), m->off[kRows][n],
                               q == 0 ? 1 : 0, m->lds_cols, m->lds_rows, st);
    if (e == hipSuccess)
      e = swkb::launch_apply_multi(m->d_prob, map_of(m, kApply), m->off[kApply][n], map_of(m, kFin),
                                   m->off[kFin][n], q, st);
  }
  return e;
}

bool valid_elems(int v) { return v == 256 || v == 512 || v == 1024; }

void destroy_all(swkb_multi_s* m) {
  if (m->ev_done) (void)hipEventSynchronize(m->ev_done);
  drop_graph(m);
  if (m->d_prob) (void)hipFree(m->d_prob);
  if (m->d_counts) (void)hipFree(m->d_counts);
  if (m->d_ctr) (void)hipFree(m->d_ctr);
  if (m->d_map) (void)hipFree(m->d_map);
  if (m->d_part) (void)hipFree(m->d_part);
  if (m->h_stage) (void)hipHostFree(m->h_stage);
  for (hipEvent_t ev : {m->ev_stage, m->ev_done, m->t0, m->t1, m->g0, m->g1})
    if (ev) (void)hipEventDestroy(ev);
  if (m->cs) (void)hipStreamDestroy(m->cs);
  delete m;
}

// Average device milliseconds of one launch of `launch` over reps launches
// (after one untimed launch).
template <typename F>
hipError_t time_launches(swkb_multi_s* m, int reps, hipStream_t st, F&& launch, double* ms) {
  hipError_t e = launch();
  if (e == hipSuccess) e = hipEventRecord(m->t0, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  if (e == hipSuccess) e = hipEventRecord(m->t1, st);
  if (e == hipSuccess) e = hipEventSynchronize(m->t1);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, m->t0, m->t1);
  *ms = (double)t / reps;
  return e;
}

}  // namespace

extern "C" {

swkb_status swkb_multi_create(const swkb_plan_t* plans, int32_t n, swkb_multi_t* out) {
  if (!out) return fail(SWKB_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!plans || n < 1 || n > kMaxProblems) return fail(SWKB_ERR_ARG, "need 1 <= n <= 4095 plans");
  for (int i = 0; i < n; ++i) {
    const swkb_plan_s* pl = plans[i];
    if (!pl) return fail(SWKB_ERR_ARG, "plan " + std::to_string(i) + " is NULL");
    if (!pl->use_matrix || pl->g.N % 512 != 0)
      return fail(SWKB_ERR_ARG, "plan " + std::to_string(i) + " must use the mode-function matrix and n_z % 512 == 0");
    if (pl->H) return fail(SWKB_ERR_ARG, "plan " + std::to_string(i) + " keeps its history (keep_history = 1)");
    for (int j = 0; j < i; ++j)
      if (plans[j] == pl) return fail(SWKB_ERR_ARG, "plan listed twice");
    if ((size_t)(pl->g.N / 512) * (size_t)max_groups(pl->g) >= (1u << kMapShift))
      return fail(SWKB_ERR_ARG, "plan " + std::to_string(i) + " is too large for the workgroup map");
  }
  swkb_multi_s* m = new (std::nothrow) swkb_multi_s();
  if (!m) return fail(SWKB_ERR_NOMEM, "host allocation failed");
  try {
    m->plans.assign(plans, plans + n);
    // table order: screen count descending, caller order among equals
    m->order.resize(n);
    for (int i = 0; i < n; ++i) m->order[i] = i;
    std::stable_sort(m->order.begin(), m->order.end(), [&](int a, int b) {
      return m->plans[a]->p.n_screens > m->plans[b]->p.n_screens;
    });
    m->qmax = m->plans[m->order[0]]->p.n_screens;
    m->na.assign(m->qmax, 0);
    for (int q = 0; q < m->qmax; ++q) {
      int c = 0;
      while (c < n && m->plans[m->order[c]]->p.n_screens > q) ++c;
      m->na[q] = c;
    }
    // size classes and the single-problem path's shapes as defaults
    std::vector<int> sizes;
    for (int i = 0; i < n; ++i) sizes.push_back(m->plans[i]->g.N);
    std::sort(sizes.begin(), sizes.end());
    sizes.erase(std::unique(sizes.begin(), sizes.end()), sizes.end());
    if ((int)sizes.size() > SWKB_MULTI_MAX_CLASSES) {
      delete m;
      return fail(SWKB_ERR_ARG, "more than SWKB_MULTI_MAX_CLASSES distinct n_z");
    }
    m->tun.n_classes = (int)sizes.size();
    for (int c = 0; c < m->tun.n_classes; ++c) {
      m->tun.class_n_z[c] = sizes[c];
      m->tun.fft_elems[c] = swkb::kFftElems;
      m->tun.apply_groups[c] = 0;
    }
    m->cls.resize(n);
    for (int s = 0; s < n; ++s) {
      const swkb_plan_s* pl = m->plans[m->order[s]];
      const int c = class_of(m, pl->g.N);
      m->cls[s] = c;
      if (pl->precision == SWKB_FP64) continue;  // FP64 products keep their own blocking
      const int d = swkb::apply_multi_groups(pl->g);
      if (m->tun.apply_groups[c] == 0 || d > m->tun.apply_groups[c]) m->tun.apply_groups[c] = d;
    }
    for (int c = 0; c < m->tun.n_classes; ++c)
      if (m->tun.apply_groups[c] == 0) m->tun.apply_groups[c] = 1;  // a class of FP64 problems only
    // one n_z can come with different n_modes: the default is the largest
    // single-problem choice among them, clamped to (n_modes + 3) / 4 per
    // problem, which gives each problem its own single-problem choice
    m->tun.graphs = 0;
    m->hp.resize(n);
  } catch (const std::exception&) {
    delete m;
    return fail(SWKB_ERR_NOMEM, "host allocation failed");
  }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&m->d_prob), sizeof(MultiProblem) * n);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&m->d_counts), sizeof(int4) * m->qmax);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&m->d_ctr), sizeof(int) * 4 * m->qmax);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&m->h_stage), sizeof(MultiProblem) * n,
                                         hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_stage, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreate(&m->t0);
  if (e == hipSuccess) e = hipEventCreate(&m->t1);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->g0, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&m->g1, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->cs, hipStreamNonBlocking);
  // both events complete from the start
  if (e == hipSuccess) e = hipEventRecord(m->ev_stage, m->cs);
  if (e == hipSuccess) e = hipEventRecord(m->ev_done, m->cs);
  if (e == hipSuccess) e = build_tables(m);
  if (e != hipSuccess) {
    destroy_all(m);
    return hip_fail(e, "swkb_multi_create");
  }
  *out = m;
  return SWKB_OK;
}

swkb_status swkb_multi_get_tuning(swkb_multi_t m, swkb_multi_tuning* out) {
  if (!m || !out) return fail(SWKB_ERR_ARG, "NULL argument");
  *out = m->tun;
  return SWKB_OK;
}

swkb_status swkb_multi_set_tuning(swkb_multi_t m, const swkb_multi_tuning* t) {
  if (!m || !t) return fail(SWKB_ERR_ARG, "NULL argument");
  if (t->n_classes != m->tun.n_classes) return fail(SWKB_ERR_ARG, "n_classes does not match the group");
  for (int c = 0; c < t->n_classes; ++c) {
    if (t->class_n_z[c] != m->tun.class_n_z[c]) return fail(SWKB_ERR_ARG, "class_n_z does not match the group");
    if (!valid_elems(t->fft_elems[c])) return fail(SWKB_ERR_ARG, "fft_elems must be 256, 512 or 1024");
    if (t->apply_groups[c] < 1) return fail(SWKB_ERR_ARG, "apply_groups must be >= 1");
  }
  if (t->graphs < 0 || t->graphs > SWKB_MULTI_PERSISTENT)
    return fail(SWKB_ERR_ARG, "graphs must be 0, 1 or SWKB_MULTI_PERSISTENT");
  const hipError_t e0 = hipEventSynchronize(m->ev_done);
  if (e0 != hipSuccess) return hip_fail(e0, "swkb_multi_set_tuning");
  drop_graph(m);
  m->tun = *t;
  const hipError_t e = build_tables(m);
  if (e != hipSuccess) return hip_fail(e, "swkb_multi_set_tuning");
  return SWKB_OK;
}

swkb_status swkb_multi_tune(swkb_multi_t m, int32_t reps, void* hip_stream, swkb_multi_tuning* out) {
  if (!m || reps < 1) return fail(SWKB_ERR_ARG, "need a group and reps >= 1");
  hipStream_t st = (hipStream_t)hip_stream;
  const int n = (int)m->plans.size();
  hipError_t e = hipEventSynchronize(m->ev_done);
  if (e != hipSuccess) return hip_fail(e, "swkb_multi_tune");
  drop_graph(m);
  // candidate product blockings per class: the single-problem choice and
  // M/32 .. M/256 workgroups along the modes
  const int nc = m->tun.n_classes;
  std::vector<std::vector<int>> cand(nc);
  for (int s = 0; s < n; ++s) {
    const Geometry& g = m->plans[m->order[s]]->g;
    std::vector<int>& cv = cand[m->cls[s]];
    if (!cv.empty()) continue;
    cv.push_back(m->tun.apply_groups[m->cls[s]]);
    for (int d = 32; d <= 256; d *= 2)
      if (g.M / d >= 1 && std::find(cv.begin(), cv.end(), g.M / d) == cv.end()) cv.push_back(g.M / d);
  }
  // buffers for the largest candidates at once
  swkb_multi_tuning big = m->tun;
  for (int c = 0; c < nc; ++c) {
    big.fft_elems[c] = 256;
    big.apply_groups[c] = *std::max_element(cand[c].begin(), cand[c].end());
  }
  const swkb_multi_tuning keep = m->tun;
  m->tun = big;
  e = build_tables(m);
  // defined inputs: zero fields and modes
  for (int s = 0; s < n && e == hipSuccess; ++s) {
    swkb_plan_s* pl = m->plans[m->order[s]];
    e = hipMemsetAsync(pl->u, 0, sizeof(double2) * pl->g.N, st);
    if (e == hipSuccess) e = hipMemsetAsync(pl->c, 0, sizeof(double2) * pl->g.M, st);
    pl->cur_q = -1;
  }
  unsigned* d_sub = nullptr;
  size_t sub_cap = 0;
  swkb_multi_tuning best = keep;
  for (int c = 0; c < nc && e == hipSuccess; ++c) {
    std::vector<int> slots;
    for (int s = 0; s < n; ++s)
      if (m->cls[s] == c) slots.push_back(s);
    // the class's workgroups of one stage under the table's current shapes
    auto sub_map = [&](int kind, std::vector<unsigned>* mp) {
      mp->clear();
      for (int s : slots) {
        const MultiProblem& p = m->hp[s];
        const int nb = stage_blocks(kind, p);
        for (int b = 0; b < nb; ++b) mp->push_back(((unsigned)s << kMapShift) | (unsigned)b);
      }
    };
    auto upload = [&](const std::vector<unsigned>& a, const std::vector<unsigned>& b) {
      hipError_t r = hipSuccess;
      const size_t need = a.size() + b.size();
      if (need > sub_cap) {
        if (d_sub) (void)hipFree(d_sub);
        d_sub = nullptr;
        sub_cap = 0;
        r = hipMalloc(reinterpret_cast<void**>(&d_sub), sizeof(unsigned) * need);
        if (r != hipSuccess) return r;
        sub_cap = need;
      }
      r = hipStreamSynchronize(st);
      if (r == hipSuccess) r = hipMemcpy(d_sub, a.data(), sizeof(unsigned) * a.size(), hipMemcpyHostToDevice);
      if (r == hipSuccess && !b.empty())
        r = hipMemcpy(d_sub + a.size(), b.data(), sizeof(unsigned) * b.size(), hipMemcpyHostToDevice);
      if (r == hipSuccess) r = hipMemcpy(m->d_prob, m->hp.data(), sizeof(MultiProblem) * n, hipMemcpyHostToDevice);
      return r;
    };
    std::vector<unsigned> ma, mb;
    double best_fft = 1e30;
    for (int fe : {256, 512, 1024}) {
      if (e != hipSuccess) break;
      size_t lc = 0, lr = 0;
      for (int s : slots) {
        MultiProblem& p = m->hp[s];
        swkb::fft_blocking(p.g, fe, &p.CA, &p.RB);
        lc = std::max(lc, sizeof(double2) * (size_t)(p.CA * p.g.P1 + p.g.P1 / 2));
        lr = std::max(lr, sizeof(double2) * (size_t)(p.RB * p.g.P2 + p.g.P2 / 2));
      }
      sub_map(kCols, &ma);
      sub_map(kRows, &mb);
      e = upload(ma, mb);
      double ms = 0.0;
      const int na_ = (int)ma.size(), nb_ = (int)mb.size();
      if (e == hipSuccess)
        e = time_launches(m, reps, st, [&] {
          return swkb::launch_fft_multi(m->d_prob, d_sub, na_, d_sub + na_, nb_, 0, lc, lr, st);
        }, &ms);
      if (e == hipSuccess && ms * 1e3 < best_fft) {
        best_fft = ms * 1e3;
        best.fft_elems[c] = fe;
        best.fft_us[c] = ms * 1e3;
      }
    }
    double best_apply = 1e30;
    for (int gr : cand[c]) {
      if (e != hipSuccess) break;
      for (int s : slots)
        if (!m->hp[s].fp64) m->hp[s].groups = std::min(gr, max_groups(m->hp[s].g));
      sub_map(kApply, &ma);
      mb.clear();
      e = upload(ma, mb);
      double ms = 0.0;
      const int na_ = (int)ma.size();
      if (e == hipSuccess)
        e = time_launches(m, reps, st, [&] {
          return swkb::launch_apply_multi(m->d_prob, d_sub, na_, nullptr, 0, 0, st);
        }, &ms);
      if (e == hipSuccess && ms * 1e3 < best_apply) {
        best_apply = ms * 1e3;
        best.apply_groups[c] = gr;
        best.apply_us[c] = ms * 1e3;
      }
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (d_sub) (void)hipFree(d_sub);
  m->tun = e == hipSuccess ? best : keep;
  const hipError_t e2 = build_tables(m);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) return hip_fail(e, "swkb_multi_tune");
  if (out) *out = m->tun;
  return SWKB_OK;
}

swkb_status swkb_multi_propagate(swkb_multi_t m, const void* const* u_in, void* const* history, void* hip_stream) {
  if (!m || !u_in) return fail(SWKB_ERR_ARG, "NULL argument");
  const int n = (int)m->plans.size();
  for (int i = 0; i < n; ++i)
    if (!u_in[i]) return fail(SWKB_ERR_ARG, "u_in[" + std::to_string(i) + "] is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  // the staging buffer is free once the previous call's copy has been done
  hipError_t e = hipEventSynchronize(m->ev_stage);
  // and the table is rewritten only after the previous call's steps
  if (e == hipSuccess) e = hipStreamWaitEvent(st, m->ev_done, 0);
  if (e != hipSuccess) return hip_fail(e, "swkb_multi_propagate");
  for (int s = 0; s < n; ++s) {
    m->h_stage[s] = m->hp[s];
    m->h_stage[s].u_in = static_cast<const double2*>(u_in[m->order[s]]);
    m->h_stage[s].hist = history ? static_cast<double2*>(history[m->order[s]]) : nullptr;
  }
  e = hipMemcpyAsync(m->d_prob, m->h_stage, sizeof(MultiProblem) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(m->ev_stage, st);
  if (e != hipSuccess) return hip_fail(e, "swkb_multi_propagate: table upload");
  if (m->tun.graphs == SWKB_MULTI_PERSISTENT) {
    const size_t lds = std::max(std::max(m->lds_cols, m->lds_rows), swkb::apply_lds_bytes());
    e = swkb::launch_multi_persistent(m->d_prob, map_of(m, kCols), map_of(m, kRows), map_of(m, kApply),
                                      map_of(m, kFin), m->d_counts, m->d_ctr, m->qmax, lds, 0, st,
                                      &m->persist_blocks);
  } else if (m->tun.graphs) {
    if (!m->exec) {
      e = hipStreamBeginCapture(m->cs, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "swkb_multi_propagate: capture");
      const hipError_t ec = enqueue_steps(m, m->cs);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(m->cs, &graph);
      if (ec != hipSuccess || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(ec != hipSuccess ? ec : e, "swkb_multi_propagate: capture");
      }
      e = hipGraphInstantiate(&m->exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        m->exec = nullptr;
        return hip_fail(e, "swkb_multi_propagate: graph instantiate");
      }
      m->graph = graph;
    }
    e = hipEventRecord(m->g0, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(m->cs, m->g0, 0);
    if (e == hipSuccess) e = hipGraphLaunch(m->exec, m->cs);
    if (e == hipSuccess) e = hipEventRecord(m->g1, m->cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, m->g1, 0);
  } else {
    e = enqueue_steps(m, st);
  }
  if (e == hipSuccess) e = hipEventRecord(m->ev_done, st);
  if (e != hipSuccess) return hip_fail(e, "swkb_multi_propagate: launch");
  for (int i = 0; i < n; ++i) m->plans[i]->cur_q = m->plans[i]->p.n_screens;
  return SWKB_OK;
}

void swkb_multi_destroy(swkb_multi_t m) {
  if (!m) return;
  destroy_all(m);
}

}  // extern "C"

// For other parts of the library: every problem of the group reads its field
// from inputs[i] (caller order) on each step; synchronous upload.
hipError_t swkb::multi_set_inputs(swkb_multi_s* m, const double2* const* inputs) {
  hipError_t e = hipEventSynchronize(m->ev_done);
  if (e != hipSuccess) return e;
  drop_graph(m);
  const int n = (int)m->plans.size();
  for (int s = 0; s < n; ++s) m->hp[s].u_in = inputs[m->order[s]];
  return hipMemcpy(m->d_prob, m->hp.data(), sizeof(MultiProblem) * n, hipMemcpyHostToDevice);
}

// One screen step (screen q) of every problem from its input, on stream st.
hipError_t swkb::multi_step(swkb_multi_s* m, int q, hipStream_t st) {
  const int n = (int)m->plans.size();
  hipError_t e = launch_fft_multi(m->d_prob, map_of(m, kCols), m->off[kCols][n], map_of(m, kRows), m->off[kRows][n], 1,
                                  m->lds_cols, m->lds_rows, st);
  if (e == hipSuccess)
    e = launch_apply_multi(m->d_prob, map_of(m, kApply), m->off[kApply][n], map_of(m, kFin), m->off[kFin][n], q, st);
  // under stream capture the caller marks the end of the replay instead
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (e == hipSuccess) e = hipStreamIsCapturing(st, &cap);
  if (e == hipSuccess && cap == hipStreamCaptureStatusNone) e = hipEventRecord(m->ev_done, st);
  return e;
}

// Marks the group's work enqueued on st so far as the latest (for a replay).
hipError_t swkb::multi_mark(swkb_multi_s* m, hipStream_t st) { return hipEventRecord(m->ev_done, st); }
