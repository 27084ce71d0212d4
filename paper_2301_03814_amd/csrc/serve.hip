// Serving loop: continuous batching of independent propagation requests on
// one GPU.  Each request is one problem (its own medium, frequency, grid and
// range, Algorithm 1 over its screens) with its own plan, device workspace
// and stream; requests are admitted in arrival order as long as their
// device footprint fits the budget and a slot is free, and every scheduling
// round advances each admitted request by a chunk of screens on its stream,
// so the work of all admitted requests overlaps on the device.  Chunks hold
// about the same number of mode-point evaluations for every request (a
// processor-sharing quantum), and a request keeps at most one chunk in
// flight, so a newly admitted or short request gets GPU time within one
// round of the others and is not stuck behind long ones.  Results do not depend on the mix:
// every request runs the same deterministic kernels on its own data.
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "swkb_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

enum ReqState { kPending = 0, kActive = 1, kDone = 2, kFailed = 3 };

struct Request {
  int64_t id = 0;
  swkb_params p{};
  std::vector<double> mparams;
  double2* u0_host = nullptr;   // pinned complex128[N]: incident field, then the result
  size_t footprint = 0;         // device bytes while admitted
  int state = kPending;
  std::string error;
  void* ws = nullptr;           // plan workspace (device)
  double2* u_dev = nullptr;     // incident field (device)
  swkb_plan_t plan = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;      // end of the last enqueued chunk
  int q_next = 0;               // first screen not yet enqueued
  Clock::time_point t_submit, t_admit, t_done;
};

}  // namespace

struct swkb_server_s {
  swkb_server_config cfg;
  std::deque<Request*> pending;
  std::vector<Request*> active;
  std::map<int64_t, Request*> all;
  size_t used = 0;
  int64_t next_id = 1;
  int64_t screens = 0, mode_points = 0, completed = 0;
  Clock::time_point t0;
};

namespace {

size_t request_footprint(const swkb_params* p) { return swkb_footprint(p); }

void release(swkb_server_s* s, Request* r) {
  if (r->plan) swkb_destroy(r->plan);
  if (r->ev) (void)hipEventDestroy(r->ev);
  if (r->st) (void)hipStreamDestroy(r->st);
  if (r->ws) (void)hipFree(r->ws);
  if (r->u_dev) (void)hipFree(r->u_dev);
  r->plan = nullptr;
  r->ev = nullptr;
  r->st = nullptr;
  r->ws = nullptr;
  r->u_dev = nullptr;
  s->used -= r->footprint;  // zero unless admitted
  r->footprint = 0;
}

void fail_request(swkb_server_s* s, Request* r, const std::string& why) {
  r->error = why;
  release(s, r);
  r->state = kFailed;
  r->t_done = Clock::now();
}

// Allocate, plan and upload the incident field; false leaves r failed.
bool admit(swkb_server_s* s, Request* r) {
  r->footprint = request_footprint(&r->p);
  s->used += r->footprint;
  r->state = kActive;
  r->t_admit = Clock::now();
  const size_t wsb = swkb_workspace_bytes(&r->p);
  hipError_t e = hipStreamCreateWithFlags(&r->st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&r->ws, wsb);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&r->u_dev), sizeof(double2) * r->p.n_z);
  if (e != hipSuccess) {
    fail_request(s, r, std::string("device allocation: ") + hipGetErrorString(e));
    return false;
  }
  const swkb_status ps = swkb_plan(&r->p, r->ws, wsb, r->st, &r->plan);
  if (ps != SWKB_OK) {
    fail_request(s, r, std::string("plan: ") + swkb_last_error());
    return false;
  }
  e = hipMemcpyAsync(r->u_dev, r->u0_host, sizeof(double2) * r->p.n_z, hipMemcpyHostToDevice, r->st);
  if (e != hipSuccess) {
    fail_request(s, r, std::string("upload: ") + hipGetErrorString(e));
    return false;
  }
  r->q_next = 0;
  return true;
}

// Enqueue the next chunk of screens; the last chunk also copies the final
// field back into the pinned host buffer.
bool advance(swkb_server_s* s, Request* r) {
  const int Q = r->p.n_screens;
  int chunk = s->cfg.screens_per_round;
  if (s->cfg.mode_points_per_round > 0.0) {
    const double per_screen = (double)r->p.n_modes * (double)r->p.n_z;
    const double k = s->cfg.mode_points_per_round / per_screen;
    if (k > chunk) chunk = k < (double)Q ? (int)k : Q;
  }
  const int q1 = Q - r->q_next > chunk ? r->q_next + chunk : Q;
  const swkb_status ps = swkb_propagate(r->plan, r->q_next == 0 ? r->u_dev : nullptr, r->q_next, q1, nullptr, r->st);
  if (ps != SWKB_OK) {
    fail_request(s, r, std::string("propagate: ") + swkb_last_error());
    return false;
  }
  r->q_next = q1;
  hipError_t e = hipSuccess;
  if (q1 == Q) e = swkb_field(r->plan, -1, r->u_dev, r->st) == SWKB_OK ? hipSuccess : hipErrorUnknown;
  if (e == hipSuccess && q1 == Q)
    e = hipMemcpyAsync(r->u0_host, r->u_dev, sizeof(double2) * r->p.n_z, hipMemcpyDeviceToHost, r->st);
  if (e == hipSuccess) e = hipEventRecord(r->ev, r->st);
  if (e != hipSuccess) {
    fail_request(s, r, "chunk launch failed");
    return false;
  }
  return true;
}

}  // namespace

extern "C" {

swkb_status swkb_server_create(const swkb_server_config* cfg, swkb_server_t* out) {
  if (!out) return SWKB_ERR_ARG;
  *out = nullptr;
  if (!cfg || cfg->hbm_budget_bytes == 0 || cfg->max_active < 1 || cfg->screens_per_round < 1 ||
      !(cfg->mode_points_per_round >= 0.0)) {
    swkb::set_error(
        "server config needs hbm_budget_bytes > 0, max_active >= 1, screens_per_round >= 1, "
        "mode_points_per_round >= 0");
    return SWKB_ERR_ARG;
  }
  swkb_server_s* s = new (std::nothrow) swkb_server_s();
  if (!s) return SWKB_ERR_NOMEM;
  s->cfg = *cfg;
  s->t0 = Clock::now();
  *out = s;
  return SWKB_OK;
}

swkb_status swkb_server_submit(swkb_server_t s, const swkb_params* p, const void* u0, int64_t* id) {
  if (!s || !p || !u0 || !id) {
    swkb::set_error("NULL argument");
    return SWKB_ERR_ARG;
  }
  const size_t fp = request_footprint(p);
  if (fp == 0) return swkb_workspace_bytes(p) == 0 ? SWKB_ERR_ARG : SWKB_ERR_NOMEM;
  if (fp > s->cfg.hbm_budget_bytes) {
    swkb::set_error("request footprint " + std::to_string(fp) + " bytes exceeds the server's budget");
    return SWKB_ERR_NOMEM;
  }
  Request* r = new (std::nothrow) Request();
  if (!r) return SWKB_ERR_NOMEM;
  try {
    r->p = *p;
    r->mparams.assign(p->medium_params, p->medium_params + p->n_medium_params);
    r->p.medium_params = r->mparams.data();
  } catch (const std::exception&) {
    delete r;
    return SWKB_ERR_NOMEM;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&r->u0_host), sizeof(double2) * p->n_z, hipHostMallocDefault) !=
      hipSuccess) {
    delete r;
    swkb::set_error("pinned host allocation failed");
    return SWKB_ERR_NOMEM;
  }
  std::memcpy(r->u0_host, u0, sizeof(double2) * p->n_z);
  r->id = s->next_id++;
  r->t_submit = Clock::now();
  s->pending.push_back(r);
  s->all[r->id] = r;
  *id = r->id;
  return SWKB_OK;
}

swkb_status swkb_server_step(swkb_server_t s, int32_t* n_active, int32_t* n_pending) {
  if (!s) return SWKB_ERR_ARG;
  // retire requests whose last chunk has finished; advance the others
  std::vector<Request*> keep;
  for (Request* r : s->active) {
    if (r->state != kActive) continue;
    const hipError_t q = hipEventQuery(r->ev);
    if (q == hipErrorNotReady) {
      keep.push_back(r);
      continue;
    }
    if (q != hipSuccess) {
      fail_request(s, r, std::string("device error: ") + hipGetErrorString(q));
      continue;
    }
    if (r->q_next == r->p.n_screens) {
      s->screens += r->p.n_screens;
      s->mode_points += (int64_t)r->p.n_screens * r->p.n_modes * r->p.n_z;
      ++s->completed;
      release(s, r);
      r->state = kDone;
      r->t_done = Clock::now();
      continue;
    }
    if (advance(s, r)) keep.push_back(r);
  }
  s->active.swap(keep);
  // admission in arrival order, by device footprint
  while (!s->pending.empty() && (int)s->active.size() < s->cfg.max_active) {
    Request* r = s->pending.front();
    if (s->used + request_footprint(&r->p) > s->cfg.hbm_budget_bytes) break;
    s->pending.pop_front();
    if (admit(s, r) && advance(s, r)) s->active.push_back(r);
  }
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_pending) *n_pending = (int32_t)s->pending.size();
  return SWKB_OK;
}

swkb_status swkb_server_poll(swkb_server_t s, int64_t id, void* out, swkb_request_info* info) {
  if (!s) return SWKB_ERR_ARG;
  auto it = s->all.find(id);
  if (it == s->all.end()) {
    swkb::set_error("unknown request id");
    return SWKB_ERR_ARG;
  }
  Request* r = it->second;
  if (info) {
    info->state = r->state;
    auto us = [](Clock::time_point a, Clock::time_point b) {
      return std::chrono::duration<double, std::micro>(b - a).count();
    };
    info->queue_us = r->state == kPending ? -1.0 : us(r->t_submit, r->t_admit);
    info->latency_us = (r->state == kDone || r->state == kFailed) ? us(r->t_submit, r->t_done) : -1.0;
    info->n_z = r->p.n_z;
  }
  if (r->state == kFailed) {
    swkb::set_error(r->error);
    return SWKB_ERR_DEVICE;
  }
  if (r->state != kDone) return SWKB_ERR_STATE;
  if (out) {
    std::memcpy(out, r->u0_host, sizeof(double2) * r->p.n_z);
    (void)hipHostFree(r->u0_host);
    s->all.erase(it);
    delete r;
  }
  return SWKB_OK;
}

swkb_status swkb_server_stats(swkb_server_t s, swkb_server_stats_t* out) {
  if (!s || !out) return SWKB_ERR_ARG;
  out->completed = s->completed;
  out->screens = s->screens;
  out->mode_points = s->mode_points;
  out->device_bytes_in_use = s->used;
  out->active = (int32_t)s->active.size();
  out->pending = (int32_t)s->pending.size();
  out->seconds = std::chrono::duration<double>(Clock::now() - s->t0).count();
  return SWKB_OK;
}

void swkb_server_destroy(swkb_server_t s) {
  if (!s) return;
  for (Request* r : s->active) (void)hipStreamSynchronize(r->st);
  for (auto& kv : s->all) {
    Request* r = kv.second;
    release(s, r);
    if (r->u0_host) (void)hipHostFree(r->u0_host);
    delete r;
  }
  delete s;
}

}  // extern "C"
