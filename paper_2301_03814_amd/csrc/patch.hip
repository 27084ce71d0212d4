// Overlapping-patch screened WKB (Sec. 2.4, FC-SWKB): the vertical interval
// is covered by P patches around the cores [c_p, c_{p+1}], c_p = z_a + p K h
// (K = N / P cells), blended by the smooth partition of unity
//   sigma_p(z) = erfc(-(z - c_p) / w) / 2,
//   S^0 = 1 - sigma_1,  S^p = sigma_p - sigma_{p+1},  S^{P-1} = sigma_{P-1},
// which sums to one and falls below 1e-17 more than 6 w outside each core.
//
// Fourier continuation (the paper's method, SWKB_PATCH_FC): patch p holds
// the grid points [a_p, b_p] = [p K - e_w, (p + 1) K + e_w] (e_w =
// ceil(6 w / h), clipped to the grid).  Each screen, the field on the patch
// is continued past both ends by the FC-Gram blend (fc_gram.h: 27 values
// blending the last 5 samples to zero) into one period of a power-of-two
// length, the patch in its middle (eq. ifft_eq_phi_patches); that period is
// the input of an ordinary periodic plan whose rays are launched only at the
// patch's points with initial amplitude S^p(z) w_j / N (the plan's launch
// window, applied after every march).  The patches' sums over their modes
// are added on the global grid.  Over a ground (Sec. 2.5) the boundary
// patch is continued only at its top and keeps the ground mirror of the
// ordinary step (odd or even extension, medium reflected, launch amplitude
// S^0 reflected), so it is never reflected afterwards; every other patch's
// sum is reflected about z_a on each screen (eq. u_refl).
//
// Windowed pieces (SWKB_PATCH_WINDOWED, a variant of this library's): the
// field is windowed, u_p = S^p u, and each piece runs the ordinary step on a
// sub-domain holding the core plus e = ceil((6 w + margin) / h) cells on
// each side, with the ground mirror on the bottom patch; the pieces carry the
// spectrum of S^p u instead of launching S^p with each mode.
//
// Both: each sub-domain keeps the global largest vertical slowness (M_p =
// 2 floor(M P_p / (2 P_g) + 1/2), P_p and P_g the FFT lengths), has no
// absorbers of its own and has room for ceil(margin / h) cells of drift; the
// global exit taper applies once after the sum; for media that do not depend
// on x in mixed precision all patches' steps run as one multi-problem group
// (one launch per stage).  The per-screen cost is the sum of the
// sub-domains' M_p n_p instead of M N.
#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "fc_gram.h"
#include "swkb_internal.h"

namespace {

struct PatchView {
  int start, n;        // global index of the sub-domain's first point, its points
  const double2* f;    // the sub-plan's field after its screen step
  const double* S;     // window at the sub-domain's points (windowed pieces)
  double2* v;          // the sub-plan's input
  int a, b;            // the patch's points [a, b] (Fourier continuation)
  int cont_below;      // 1: continued below a as well (0: the boundary patch over a ground)
  int reflect;         // 1: the sum is reflected about z_a (eq. u_refl)
};

__constant__ double c_blend[swkb::kFcCont][swkb::kFcMatch] = SWKB_FC_BLEND_INIT;

swkb_status fail(swkb_status s, const std::string& msg) {
  swkb::set_error(msg);
  return s;
}

swkb_status hip_fail(hipError_t e, const char* what) {
  swkb::set_error(std::string(what) + ": " + hipGetErrorString(e));
  return SWKB_ERR_DEVICE;
}

// Windowed pieces of every patch (patch blockIdx.y): v[i] = S[i] u[start + i]
// inside the global grid, 0 outside.
__global__ void patch_window_all_kernel(const double2* __restrict__ u, int N, const PatchView* __restrict__ views) {
  const PatchView& pv = views[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pv.n) return;
  const int m = pv.start + i;
  double2 r = make_double2(0.0, 0.0);
  if (m >= 0 && m < N) {
    const double2 x = u[m];
    r = make_double2(pv.S[i] * x.x, pv.S[i] * x.y);
  }
  pv.v[i] = r;
}

// The sub-plans' inputs of every patch (patch blockIdx.y): the field on
// [a, b] and its Fourier continuation, c + 1 cells past b the blend row c of
// the last kFcMatch samples, c + 1 cells below a (cont_below) row c of the
// first kFcMatch samples taken downwards, zero elsewhere in the period.
__global__ void patch_fc_all_kernel(const double2* __restrict__ u, const PatchView* __restrict__ views) {
  const PatchView& pv = views[blockIdx.y];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pv.n) return;
  const int g = pv.start + i;
  double re = 0.0, im = 0.0;
  if (g >= pv.a && g <= pv.b) {
    const double2 x = u[g];
    re = x.x;
    im = x.y;
  } else if (g > pv.b && g <= pv.b + swkb::kFcCont) {
    const int c = g - pv.b - 1;
    for (int k = 0; k < swkb::kFcMatch; ++k) {
      const double2 x = u[pv.b - swkb::kFcMatch + 1 + k];
      re += c_blend[c][k] * x.x;
      im += c_blend[c][k] * x.y;
    }
  } else if (pv.cont_below && g < pv.a && g >= pv.a - swkb::kFcCont) {
    const int c = pv.a - g - 1;
    for (int k = 0; k < swkb::kFcMatch; ++k) {
      const double2 x = u[pv.a + swkb::kFcMatch - 1 - k];
      re += c_blend[c][k] * x.x;
      im += c_blend[c][k] * x.y;
    }
  }
  pv.v[i] = make_double2(re, im);
}

// u'[m] = W[m] sum_p (f_p[m - start_p] + sgn f_p[-m - start_p] if reflected)
// (patches in order), and the history row.
__global__ void patch_add_kernel(const PatchView* __restrict__ views, int P, int N, const double* __restrict__ W,
                                 double sgn, double2* __restrict__ out, double2* __restrict__ hist) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  double re = 0.0, im = 0.0;
  for (int p = 0; p < P; ++p) {
    const PatchView& pv = views[p];
    const int i = m - pv.start;
    if (i >= 0 && i < pv.n) {
      const double2 x = pv.f[i];
      re += x.x;
      im += x.y;
    }
    if (pv.reflect) {
      const int j = -m - pv.start;
      if (j >= 0 && j < pv.n) {
        const double2 x = pv.f[j];
        re += sgn * x.x;
        im += sgn * x.y;
      }
    }
  }
  const double2 r = make_double2(W[m] * re, W[m] * im);
  out[m] = r;
  if (hist) hist[m] = r;
}

int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p *= 2;
  return p;
}

}  // namespace

struct swkb_patch_s {
  swkb_params p;
  std::vector<double> mparams;
  int P = 0, N = 0;
  int method = SWKB_PATCH_FC;
  double width = 0.0, margin = 0.0, h = 0.0;
  double sgn = 0.0;  // reflection of the non-boundary patches' sums: -1 Dirichlet, +1 Neumann, 0 none
  struct Sub {
    int start = 0, n = 0;
    int a = 0, b = 0;      // the patch's points (Fourier continuation)
    swkb_params sp{};
    void* ws = nullptr;
    swkb_plan_t plan = nullptr;
    double2* v = nullptr;  // the sub-plan's input [n]
    double* S = nullptr;   // windowed pieces: window at the sub-domain's points [n] (0 outside the grid)
    double* lw = nullptr;  // Fourier continuation: launch amplitude factor per ray of the sub-plan [R]
  };
  std::vector<Sub> subs;
  double2* u = nullptr;    // current field [N]
  double* W = nullptr;     // global exit taper [N]
  PatchView* views = nullptr;
  int max_n = 0;
  // media that do not depend on x, mixed precision: the sub-plans' steps as
  // one multi-problem group (one launch per stage for all patches)
  swkb_multi_t grp = nullptr;
  int cur_q = -1;
  // screen ranges of the grouped path captured into HIP graphs
  struct Graph {
    const void* u_in;
    int q0, q1;
    void* hist;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<Graph> graphs;
  int graphs_on = 0;
  hipStream_t cs = nullptr;
  hipEvent_t g0 = nullptr, g1 = nullptr;
};

namespace {

void drop_graphs(swkb_patch_s* pp) {
  for (auto& g : pp->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  pp->graphs.clear();
}

void destroy_patch(swkb_patch_s* pp) {
  drop_graphs(pp);
  if (pp->g0) (void)hipEventDestroy(pp->g0);
  if (pp->g1) (void)hipEventDestroy(pp->g1);
  if (pp->cs) (void)hipStreamDestroy(pp->cs);
  if (pp->grp) swkb_multi_destroy(pp->grp);
  for (auto& s : pp->subs) {
    if (s.plan) swkb_destroy(s.plan);
    if (s.ws) (void)hipFree(s.ws);
    if (s.v) (void)hipFree(s.v);
    if (s.S) (void)hipFree(s.S);
    if (s.lw) (void)hipFree(s.lw);
  }
  if (pp->u) (void)hipFree(pp->u);
  if (pp->W) (void)hipFree(pp->W);
  if (pp->views) (void)hipFree(pp->views);
  delete pp;
}

// Partition of unity S^p at height z.
double window(const swkb_patch_s* pp, int p, double z) {
  if (pp->P == 1) return 1.0;
  const int K = pp->N / pp->P;
  auto sigma = [&](int q) { return 0.5 * std::erfc(-(z - (pp->p.z_a + (double)(q * K) * pp->h)) / pp->width); };
  if (p == 0) return 1.0 - sigma(1);
  if (p == pp->P - 1) return sigma(pp->P - 1);
  return sigma(p) - sigma(p + 1);
}

// Exit taper of the global problem (cos^2 over each absorber layer).
double exit_taper(const swkb_params& p, double z) {
  double w = 1.0;
  if (p.absorber_bot > 0.0 && z < p.z_a + p.absorber_bot) {
    const double c = std::cos(0.5 * M_PI * ((p.z_a + p.absorber_bot - z) / p.absorber_bot));
    w *= c * c;
  }
  if (p.absorber_top > 0.0 && z > p.z_b - p.absorber_top) {
    const double c = std::cos(0.5 * M_PI * ((z - (p.z_b - p.absorber_top)) / p.absorber_top));
    w *= c * c;
  }
  return w;
}

// Screens q_begin .. q_end-1 on stream st (the body of swkb_patch_propagate).
swkb_status enqueue_screens(swkb_patch_s* pp, const void* u_in, int q_begin, int q_end, void* history,
                            hipStream_t st) {
  hipError_t e = hipSuccess;
  if (u_in) e = hipMemcpyAsync(pp->u, u_in, sizeof(double2) * pp->N, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "swkb_patch_propagate: field copy");
  for (int q = q_begin; q < q_end; ++q) {
    // every patch's input: its Fourier-continued period, or its windowed piece
    if (pp->method == SWKB_PATCH_FC)
      hipLaunchKernelGGL(patch_fc_all_kernel, dim3((pp->max_n + 255) / 256, pp->P), dim3(256), 0, st, pp->u,
                         pp->views);
    else
      hipLaunchKernelGGL(patch_window_all_kernel, dim3((pp->max_n + 255) / 256, pp->P), dim3(256), 0, st, pp->u,
                         pp->N, pp->views);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "swkb_patch_propagate: patch inputs");
    if (pp->grp) {
      e = swkb::multi_step(pp->grp, q, st);
      if (e != hipSuccess) return hip_fail(e, "swkb_patch_propagate: grouped step");
    } else {
      for (auto& s : pp->subs) {
        const swkb_status ps = swkb::propagate_impl(s.plan, s.v, q, q + 1, nullptr, st);
        if (ps != SWKB_OK) return ps;
      }
    }
    double2* hist = history ? static_cast<double2*>(history) + (size_t)(q - q_begin) * pp->N : nullptr;
    hipLaunchKernelGGL(patch_add_kernel, dim3((pp->N + 255) / 256), dim3(256), 0, st, pp->views, pp->P, pp->N, pp->W,
                       pp->sgn, pp->u, hist);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "swkb_patch_propagate: overlap-add");
  }
  return SWKB_OK;
}

}  // namespace

extern "C" {

swkb_status swkb_patch_plan(const swkb_params* p, const swkb_patch_config* pc, void* hip_stream,
                            swkb_patch_t* out) {
  if (!out) return fail(SWKB_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!p || !pc) return fail(SWKB_ERR_ARG, "NULL argument");
  // the global grid is only windowed and summed; every sub-domain is
  // validated as a plan of its own below (so n_z may exceed a single plan's)
  if (p->n_z < 64 || p->n_z > (1 << 24)) return fail(SWKB_ERR_ARG, "n_z must be in [64, 2^24]");
  if (pc->n_patches < 1 || p->n_z % pc->n_patches != 0)
    return fail(SWKB_ERR_ARG, "n_patches must be >= 1 and divide n_z");
  {
    const long P_g = p->bc == SWKB_BC_PERIODIC ? p->n_z : 2L * p->n_z;
    if (p->n_modes < 2 || (p->n_modes & 1) || p->n_modes > P_g) return fail(SWKB_ERR_ARG, "n_modes must be even and in [2, P]");
    if (!(p->z_b > p->z_a) || !(p->k > 0.0) || !std::isfinite(p->k)) return fail(SWKB_ERR_ARG, "need z_b > z_a and k > 0");
    if (!(p->absorber_bot >= 0.0 && p->absorber_top >= 0.0 && p->absorber_bot + p->absorber_top <= p->z_b - p->z_a))
      return fail(SWKB_ERR_ARG, "absorber thicknesses must be >= 0 and fit in [z_a, z_b]");
    if (p->bc < 0 || p->bc > 2 || !p->medium_params || p->n_medium_params < 1)
      return fail(SWKB_ERR_ARG, "invalid bc or medium parameters");
  }
  if (!(pc->width > 0.0) || !(pc->margin >= 0.0) || !std::isfinite(pc->width) || !std::isfinite(pc->margin))
    return fail(SWKB_ERR_ARG, "width must be > 0 and margin >= 0");
  if (p->max_batch != 1) return fail(SWKB_ERR_ARG, "patch plans carry one field (max_batch = 1)");
  if (pc->method != SWKB_PATCH_FC && pc->method != SWKB_PATCH_WINDOWED)
    return fail(SWKB_ERR_ARG, "method must be SWKB_PATCH_FC or SWKB_PATCH_WINDOWED");
  hipStream_t st = (hipStream_t)hip_stream;
  swkb_patch_s* pp = new (std::nothrow) swkb_patch_s();
  if (!pp) return fail(SWKB_ERR_NOMEM, "host allocation failed");
  try {
    pp->p = *p;
    pp->mparams.assign(p->medium_params, p->medium_params + p->n_medium_params);
    pp->p.medium_params = pp->mparams.data();
    pp->P = pc->n_patches;
    pp->N = p->n_z;
    pp->method = pc->method;
    pp->width = pc->width;
    pp->margin = pc->margin;
    pp->h = (p->z_b - p->z_a) / p->n_z;
    const bool ground = p->bc != SWKB_BC_PERIODIC;
    pp->sgn = pc->method == SWKB_PATCH_FC && ground ? (p->bc == SWKB_BC_DIRICHLET ? -1.0 : 1.0) : 0.0;
    const int K = pp->N / pp->P;
    const int e = (int)std::ceil((6.0 * pc->width + pc->margin) / pp->h);
    const int e_w = (int)std::ceil(6.0 * pc->width / pp->h);
    const int e_m = (int)std::ceil(pc->margin / pp->h);
    const int P_g = ground ? 2 * pp->N : pp->N;
    pp->subs.resize(pp->P);
    for (int q = 0; q < pp->P; ++q) {
      auto& s = pp->subs[q];
      s.sp = pp->p;
      s.sp.launch_ext_cells = 0;
      if (pc->method == SWKB_PATCH_FC) {
        // the patch's points; its period holds 27 blend cells and the drift
        // margin on both sides, the patch in the middle
        s.a = std::max(0, q * K - e_w);
        s.b = std::min(pp->N - 1, (q + 1) * K + e_w);
        const int n = s.b - s.a + 1;
        if (n < 2 * swkb::kFcMatch) {
          delete pp;
          return fail(SWKB_ERR_ARG, "a patch holds fewer than two matching stencils (10 points)");
        }
        if (q == 0 && ground) {
          s.n = pow2_at_least(s.b + 1 + swkb::kFcCont + e_m);
          s.start = 0;
          s.sp.launch_ext_cells = e_m;  // rays of the mirror half that reach z_a
        } else {
          s.n = pow2_at_least(n + 2 * swkb::kFcCont + 2 * e_m);
          s.start = s.a - (s.n - n) / 2;
          s.sp.bc = SWKB_BC_PERIODIC;
        }
      } else if (q == 0 && ground) {
        s.n = pow2_at_least(K + e);
        s.start = 0;
      } else {
        const int need = K + 2 * e;
        s.n = pow2_at_least(need);
        s.start = q * K - e - (s.n - need) / 2;
        s.sp.bc = SWKB_BC_PERIODIC;
      }
      if (pc->method == SWKB_PATCH_WINDOWED) s.sp.launch_ext_cells = p->launch_ext_cells;
      const int P_p = s.sp.bc == SWKB_BC_PERIODIC ? s.n : 2 * s.n;
      s.sp.n_z = s.n;
      s.sp.n_modes = std::max(2, 2 * (int)std::floor((double)p->n_modes * P_p / (2.0 * P_g) + 0.5));
      s.sp.z_a = p->z_a + (double)s.start * pp->h;
      s.sp.z_b = p->z_a + (double)(s.start + s.n) * pp->h;
      s.sp.absorber_bot = 0.0;
      s.sp.absorber_top = 0.0;
      s.sp.keep_history = 0;
    }
  } catch (const std::exception&) {
    delete pp;
    return fail(SWKB_ERR_NOMEM, "host allocation failed");
  }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&pp->u), sizeof(double2) * pp->N);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pp->W), sizeof(double) * pp->N);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&pp->views), sizeof(PatchView) * pp->P);
  if (e != hipSuccess) {
    destroy_patch(pp);
    return hip_fail(e, "swkb_patch_plan");
  }
  std::vector<PatchView> views(pp->P);
  for (int q = 0; q < pp->P; ++q) {
    auto& s = pp->subs[q];
    const size_t wb = swkb_workspace_bytes(&s.sp);
    if (wb == 0) {
      destroy_patch(pp);
      return fail(SWKB_ERR_ARG, "sub-domain " + std::to_string(q) + " has invalid parameters (n_z " +
                                    std::to_string(pp->subs[q].n) + ", n_modes " +
                                    std::to_string(pp->subs[q].sp.n_modes) + ")");
    }
    e = hipMalloc(&s.ws, wb);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s.v), sizeof(double2) * s.n);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s.S), sizeof(double) * s.n);
    if (e != hipSuccess) {
      destroy_patch(pp);
      return hip_fail(e, "swkb_patch_plan: sub-domain allocation");
    }
    const swkb_status ps = swkb_plan(&s.sp, s.ws, wb, st, &s.plan);
    if (ps != SWKB_OK) {
      const std::string why = std::string("sub-domain ") + std::to_string(q) + ": " + swkb_last_error();
      destroy_patch(pp);
      return fail(ps, why);
    }
    std::vector<double> S(s.n, 0.0);
    for (int i = 0; i < s.n; ++i) {
      const int m = s.start + i;
      if (m >= 0 && m < pp->N) S[i] = window(pp, q, p->z_a + (double)m * pp->h);
    }
    e = hipMemcpy(s.S, S.data(), sizeof(double) * s.n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      destroy_patch(pp);
      return hip_fail(e, "swkb_patch_plan: window upload");
    }
    const bool ground_patch = q == 0 && p->bc != SWKB_BC_PERIODIC;
    if (pp->method == SWKB_PATCH_FC) {
      // launch amplitude S^p(s_r) of the sub-plan's rays (reflected about z_a
      // on the mirror half of the boundary patch); 0 outside [a, b]
      const int R = s.plan->g.R;
      std::vector<double> lw(R, 0.0);
      for (int r = 0; r < R; ++r) {
        int gi = s.start + r * s.sp.ray_stride - s.sp.launch_ext_cells;
        if (ground_patch && gi < 0) gi = -gi;
        if (gi >= s.a && gi <= s.b) lw[r] = window(pp, q, p->z_a + (double)gi * pp->h);
      }
      e = hipMalloc(reinterpret_cast<void**>(&s.lw), sizeof(double) * R);
      if (e == hipSuccess) e = hipMemcpy(s.lw, lw.data(), sizeof(double) * R, hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        destroy_patch(pp);
        return hip_fail(e, "swkb_patch_plan: launch window upload");
      }
      const swkb_status ws = swkb::set_launch_window(s.plan, s.lw, st);
      if (ws != SWKB_OK) {
        destroy_patch(pp);
        return ws;
      }
    }
    views[q] = PatchView{s.start, s.n, s.plan->u, s.S, s.v, s.a, s.b, ground_patch ? 0 : 1,
                         pp->method == SWKB_PATCH_FC && p->bc != SWKB_BC_PERIODIC && !ground_patch ? 1 : 0};
    pp->max_n = std::max(pp->max_n, s.n);
  }
  std::vector<double> W(pp->N);
  for (int m = 0; m < pp->N; ++m) W[m] = exit_taper(pp->p, p->z_a + (double)m * pp->h);
  e = hipMemcpy(pp->W, W.data(), sizeof(double) * pp->N, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(pp->views, views.data(), sizeof(PatchView) * pp->P, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    destroy_patch(pp);
    return hip_fail(e, "swkb_patch_plan: upload");
  }
  // sub-plans that a multi-problem group can carry: one group, autotuned
  bool grouped = true;
  for (auto& s : pp->subs)
    grouped = grouped && s.plan->use_matrix && s.plan->precision == SWKB_MIXED && s.n % 512 == 0;
  if (grouped) {
    std::vector<swkb_plan_t> plans;
    std::vector<const double2*> inputs;
    for (auto& s : pp->subs) {
      plans.push_back(s.plan);
      inputs.push_back(s.v);
    }
    swkb_status gs = swkb_multi_create(plans.data(), pp->P, &pp->grp);
    if (gs == SWKB_OK) gs = swkb_multi_tune(pp->grp, 3, st, nullptr);
    if (gs == SWKB_OK) {
      e = swkb::multi_set_inputs(pp->grp, inputs.data());
      if (e != hipSuccess) gs = hip_fail(e, "swkb_patch_plan: group inputs");
    }
    if (gs != SWKB_OK) {
      destroy_patch(pp);
      return gs;
    }
  }
  *out = pp;
  return SWKB_OK;
}

swkb_status swkb_patch_info(swkb_patch_t pp, int32_t patch, int32_t* start, int32_t* n_z, int32_t* n_modes) {
  if (!pp || patch < 0 || patch >= pp->P) return fail(SWKB_ERR_ARG, "no such patch");
  const auto& s = pp->subs[patch];
  if (start) *start = s.start;
  if (n_z) *n_z = s.n;
  if (n_modes) *n_modes = s.sp.n_modes;
  return SWKB_OK;
}

swkb_status swkb_patch_propagate(swkb_patch_t pp, const void* u_in, int32_t q_begin, int32_t q_end, void* history,
                                 void* hip_stream) {
  if (!pp) return fail(SWKB_ERR_ARG, "patch plan is NULL");
  if (q_begin < 0 || q_end < q_begin || q_end > pp->p.n_screens)
    return fail(SWKB_ERR_ARG, "need 0 <= q_begin <= q_end <= n_screens");
  if (!u_in && pp->cur_q != q_begin)
    return fail(SWKB_ERR_STATE, "u_in is NULL but the plan's field is not on screen q_begin");
  hipStream_t st = (hipStream_t)hip_stream;
  if (!(pp->graphs_on && pp->grp && q_end > q_begin)) {
    const swkb_status s = enqueue_screens(pp, u_in, q_begin, q_end, history, st);
    if (s == SWKB_OK) pp->cur_q = q_end;
    return s;
  }
  swkb_patch_s::Graph* hit = nullptr;
  for (auto& g : pp->graphs)
    if (g.u_in == u_in && g.q0 == q_begin && g.q1 == q_end && g.hist == history) hit = &g;
  hipError_t e = hipEventRecord(pp->g0, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(pp->cs, pp->g0, 0);
  if (e != hipSuccess) return hip_fail(e, "swkb_patch_propagate: graph");
  if (!hit) {
    if (pp->graphs.size() >= 4) {
      (void)hipGraphExecDestroy(pp->graphs.front().exec);
      (void)hipGraphDestroy(pp->graphs.front().graph);
      pp->graphs.erase(pp->graphs.begin());
    }
    e = hipStreamBeginCapture(pp->cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "swkb_patch_propagate: capture");
    const swkb_status s = enqueue_screens(pp, u_in, q_begin, q_end, history, pp->cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(pp->cs, &graph);
    if (s != SWKB_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return s != SWKB_OK ? s : hip_fail(e, "swkb_patch_propagate: capture");
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return hip_fail(e, "swkb_patch_propagate: graph instantiate");
    }
    pp->graphs.push_back({u_in, q_begin, q_end, history, graph, exec});
    hit = &pp->graphs.back();
  }
  e = hipGraphLaunch(hit->exec, pp->cs);
  if (e == hipSuccess) e = swkb::multi_mark(pp->grp, pp->cs);
  if (e == hipSuccess) e = hipEventRecord(pp->g1, pp->cs);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, pp->g1, 0);
  if (e != hipSuccess) return hip_fail(e, "swkb_patch_propagate: graph launch");
  pp->cur_q = q_end;
  return SWKB_OK;
}

swkb_status swkb_patch_graphs(swkb_patch_t pp, int32_t enable) {
  if (!pp) return fail(SWKB_ERR_ARG, "patch plan is NULL");
  if (enable && !pp->cs) {
    hipError_t e = hipStreamCreateWithFlags(&pp->cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pp->g0, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&pp->g1, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "swkb_patch_graphs");
  }
  if (!enable && pp->cs) {
    const hipError_t e = hipStreamSynchronize(pp->cs);
    if (e != hipSuccess) return hip_fail(e, "swkb_patch_graphs");
    drop_graphs(pp);
  }
  pp->graphs_on = enable ? 1 : 0;
  return SWKB_OK;
}

swkb_status swkb_patch_field(swkb_patch_t pp, void* out, void* hip_stream) {
  if (!pp || !out) return fail(SWKB_ERR_ARG, "NULL argument");
  if (pp->cur_q < 0) return fail(SWKB_ERR_STATE, "no field yet");
  const hipError_t e =
      hipMemcpyAsync(out, pp->u, sizeof(double2) * pp->N, hipMemcpyDeviceToDevice, (hipStream_t)hip_stream);
  return e == hipSuccess ? SWKB_OK : hip_fail(e, "swkb_patch_field");
}

void swkb_patch_destroy(swkb_patch_t pp) {
  if (!pp) return;
  (void)hipDeviceSynchronize();  // replays and sub-plan work in flight
  destroy_patch(pp);
}

}  // extern "C"
