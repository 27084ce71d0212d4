// Internal declarations shared by the HIP translation units of libswkb.
// Not part of the C ABI (include/swkb.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "swkb.h"

namespace swkb {

// Points per superposition tile (one wavefront lane per grid point).
constexpr int kTile = 64;

// Device view of the medium for one screen.
struct DevMedium {
  int kind;            // SWKB_MEDIUM_*
  int mirror;          // nonzero: eps reflected about z_a (ground mirror)
  double z_a;
  const double* prm;   // raw parameter array (device)
  const int* list;     // GAUSSSUM: candidate Gaussians of this screen (device)
  int nlist;
};

// Per-mode constants (device arrays of length M).
struct DevModes {
  const double* xi;    // vertical slowness xi_n = 2 pi n / (k P h)
  const double* pbar;  // reference horizontal slowness of the phase split
  const double* e1r;   // pbar^2 + xi^2 - 1 (reference eps - 1 of the mode)
  const double* frac;  // frac(pbar dx / lambda): range phase in turns, mod 1
};

// Arrival records, row-major [mode][ray].  T = double (FP64) or float (mixed).
struct DevRecords {
  void* D;        // arrival height minus launch height, T
  void* Pp;       // phase deviation delta psi, T
  void* G;        // q - xi at arrival, T
  void* A;        // transport factor a (> 0 live); -flag otherwise, T
  int* cz;        // first grid index m in [0, N] with z_m >= the ray's own arrival (live rays; march)
  int* cidx;      // first grid index m in [0, N] with z_m >= key_r, N + 1 if none, key_r = running
                  // maximum of live arrival heights (ray r owns the points [cidx_r, cidx_{r+1}))
  int* tstart;    // [mode][tile 0..T]: largest r with key_r <= z of the tile's first point
  int* mflag;     // per mode: bit0 folded, bit1 has caustic rays, bit2 no live ray (all dead)
  int* mcaus;     // per mode: caustic rays this march
  int* mdead;     // per mode: dead rays this march
  int* mwork;     // per mode: RK4 evaluations, direct medium evaluations, medium terms, table reads (4 ints)
};

// Per-wavefront march counts: caustic, dead, RK4 evaluations, direct medium
// evaluations, medium terms, table reads.
constexpr int kWaveCounts = 6;

// Per-screen medium table of the mixed Gaussian-sum march (tab == NULL: none).
struct MedTab {
  const float4* tab;  // cubic coefficients of eps - 1 per interval: c0..c3 [(2S+1)][n - 1]
  int n;              // z-nodes
  double z_lo, dz;    // node i at z_lo + i dz
};

struct Geometry {
  int N, M, P, R, T, S, rho, E, bc, P1, P2;
  double z_a, z_b, h, k, lam, dx, p2_floor;
};

// Exit epilogue of a plan: absorber layers, the caustic significance
// threshold, and the offset of the grid index from the phase origin.
struct Epi {
  double absorber_bot, absorber_top;
  double caustic_tol;
  int mprime_off;  // m' = m + mprime_off
};

// Elements per FFT workgroup on the single-problem path.
constexpr int kFftElems = 512;

// One problem of a multi-problem launch (entry of a device table): the
// plan's buffers and the blocking the launch uses for it.
struct MultiProblem {
  Geometry g;
  Epi ep;
  DevRecords rec;
  const double2* tw;
  double2* Y;
  double2* c;
  const float4* tmat;    // complex64 mode-function matrix [M][N] (mixed precision)
  const double2* tmat64; // complex128 mode-function matrix [M][N] (FP64)
  int fp64, sub;         // FP64 problem; its product's 64-point tiles per workgroup
  double2* part;         // [groups][N] partial sums of the product
  double2* u;            // the problem's field
  const double2* u_in;   // field on the problem's first screen
  double2* hist;         // [n_screens][N] or NULL
  unsigned long long* counters;
  int logP1, logP2, CA, RB, groups;
};

// Energy of mode j summed over the batch in field order (the loads of eight
// fields are issued before their terms are added).
__device__ inline double batch_energy(const double2* __restrict__ c, int M, int j, int batch) {
  double e = 0.0;
  int bb = 0;
  for (; bb + 8 <= batch; bb += 8) {
    double2 cv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) cv[u] = c[(size_t)(bb + u) * M + j];
#pragma unroll
    for (int u = 0; u < 8; ++u) e += cv[u].x * cv[u].x + cv[u].y * cv[u].y;
  }
  for (; bb < batch; ++bb) {
    const double2 cv = c[(size_t)bb * M + j];
    e += cv.x * cv.x + cv.y * cv.y;
  }
  return e;
}

}  // namespace swkb

struct swkb_plan_s {
  swkb_params p;
  std::vector<double> mparams;
  swkb::Geometry g;
  int precision;
  int x_invariant;
  int march_valid_q;   // screen whose rays the active slot holds (-1 none; -2 any, x-invariant)
  int cur_q;
  // device pointers inside the caller's workspace
  double *xi, *pbar, *e1r, *frac;
  double2* tw;         // e^{-2 pi i t / P}, t in [0, P)
  double* mprm;
  int* glist;          // concatenated per-screen Gaussian lists
  std::vector<int> goff;  // host offsets into glist per screen (n_screens + 1)
  int gfast;           // Gaussian-sum march from per-screen bump tables
  int tab_S;           // RK4 steps the bump tables were built for (stage stride 2*tab_S+1)
  void* gstage;        // per screen [(2S+1)][nl] (a e^{-dx^2/2s^2}, 64 s^2 - dx^2) pairs of T
  void* gterm;         // per screen [nl] (-1/(2 s^2) [x log2 e in FP32], 1/s^2) pairs of T
  void* gczl;          // per screen [waves_per_mode][nl] bump heights minus each wavefront's z_w, T
  swkb::MedTab mtab;   // mixed Gaussian-sum path: the current screen's medium table
  double2 *u, *ub;               // single field [N]; batch fields [B][N] (max_batch > 1)
  double2 *Y, *c;                // FFT scratch [B][P], modes [B][M]
  double2* part;                 // superposition partials [B][mode groups][N]
  void* pan;                     // batched product's B operands per mode (matrix plans, max_batch > 1)
  double* menergy;               // batched product: each mode's energy summed over the batch [M] (same plans)
  const double* lwin = nullptr;  // launch amplitude factor per ray [R] (a patch's S^p; 0: ray not launched), or
                                 // NULL; device memory of the caller's, applied after every march
  float2* cpol;                  // one field's modes in polar form [M]: |c|, frac(arg c / (2 pi))
                                 // (FP32 interval sum; mixed-precision plans only)
  int max_batch;
  int sum_fields;                // fields summed per screen by the running propagation (march shape)
  int use_matrix;                // mode functions tabulated once (x-invariant medium)
  void* tmat;                    // T[mode][point], complex T (double2 or float2)
  swkb::DevRecords rec;
  int* wcount;                   // per-wavefront march counts [M][waves][kWaveCounts]
  unsigned long long* counters;  // caustic, dead, folded, significant, screens, rhs, med, terms, table reads
  unsigned long long* counters_scratch;  // diagnostics of station evaluations (discarded)
  double* frac_st;               // per-station range phases [rk4_steps][M]
  // Ray records of two screens (x-varying media): the march of screen q + 1
  // fills one slot on stream `ms` while screen q is summed from the other on
  // the caller's stream; the scan of each march runs on stream `ss`, so the
  // march stream goes on to the next screen.  rec, wcount and mtab above are
  // the active slot.  ev_free[k]: slot k's table is built and its last sum
  // done (march may start); ev_marched[k]: its march is done (scan may
  // start); ev_ready[k]: its scan is done (sum may start).
  struct Slot {
    swkb::DevRecords rec;
    int* wcount;
    swkb::MedTab mtab;
    int q;  // screen whose rays the slot holds (-1 none, -2 x-invariant)
  };
  Slot slots[2];
  int nslots;
  hipStream_t ms;                // march stream (default priority, shared by the device's plans), or NULL
  hipStream_t ss;                // scan stream (likewise), or NULL
  hipEvent_t ev_ready[2], ev_free[2], ev_marched[2];
  // screen ranges captured into HIP graphs (swkb_graphs)
  struct GraphEntry {
    const void* u_in;
    int q0, q1;
    void* hist;
    double2* u;   // field buffer the graph writes (the plan's own, or the batch buffer)
    int hist_on;  // the graph also writes the plan's kept history
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  int graphs_on;
  hipStream_t cs;                // capture and replay stream (shared by the device's plans), or NULL
  hipEvent_t ev_g0, ev_g1;
  // fields on every screen reached (keep_history = 1): [n_screens + 1][N] in
  // the workspace, and which of them hold a value; hist_on: the running
  // propagation writes them (not for batches)
  double2* H;
  std::vector<char> hvalid;
  int hist_on;
  // single user: busy is taken by the thread inside a call (PlanGuard);
  // ev_done is recorded on last_st at the end of every call
  int busy;
  hipEvent_t ev_done;
  hipStream_t last_st;
  int has_last;
  std::string err;  // last failure of a call on this plan
  // event timing
  int prof_on;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used;
  struct Mark { int cls, a, b; };
  std::vector<Mark> marks;
};

namespace swkb {

void set_error(const std::string& msg);
// Body of swkb_plan; own_streams = false creates no streams and no events.
swkb_status plan_impl(const swkb_params* p, void* workspace, size_t workspace_bytes, hipStream_t st,
                      bool own_streams, swkb_plan_t* out);
// Screens q_begin .. q_end-1 of one field, without the single-user check of
// the public entry point (for callers inside the library that hold the plan).
swkb_status propagate_impl(swkb_plan_s* pl, const void* u_in, int q_begin, int q_end, void* history,
                           hipStream_t st);

// Launchers (return hipSuccess or the launch error).
hipError_t launch_fft_modes(const swkb_plan_s& pl, const double2* u, int batch, hipStream_t st);
// Builds screen q's medium table where the plan marches through one (mixed
// precision, Gaussian sum, periodic); no-op otherwise.  Call before
// launch_march for the same screen.
hipError_t launch_medium_table(const swkb_plan_s& pl, int q, hipStream_t st);
hipError_t launch_march(const swkb_plan_s& pl, int q, hipStream_t st);
// Launch amplitude factors per ray (overlapping patches); api.hip.
swkb_status set_launch_window(swkb_plan_s* pl, const double* lw, hipStream_t st);
hipError_t launch_scan(const swkb_plan_s& pl, hipStream_t st);
// out [batch][N]; hist [batch][N] for this screen (or NULL).
hipError_t launch_superpose(const swkb_plan_s& pl, double2* out, double2* hist, int batch, hipStream_t st);
int superpose_groups(const Geometry& g);
// Largest number of mode groups any superposition writes partial sums for.
int partial_groups(const Geometry& g);
hipError_t launch_build_matrix(const swkb_plan_s& pl, hipStream_t st);
// U[b][m] = sum_j C[b][j] T[j][m] for batch > 1: mode-group partial sums into
// pl.part ([batch][groups][N], complex64 or complex128), groups written to
// *groups (matrix cores, batch.hip).
hipError_t launch_batch_product(const swkb_plan_s& pl, int batch, hipStream_t st, int* groups);
int batch_groups(const Geometry& g, int precision, int B);
size_t batch_part_bytes(const Geometry& g, int precision, int Bmax);
size_t batch_panel_bytes(const Geometry& g, int B);
hipError_t launch_apply_matrix(const swkb_plan_s& pl, double2* out, double2* hist, int batch, hipStream_t st);
// Multi-problem launches (tables and workgroup maps in device memory; map
// entries are problem << 20 | local workgroup).
void fft_blocking(const Geometry& g, int elems, int* CA, int* RB);
int ilog2(int x);
Epi epi_of(const swkb_plan_s& pl);
int finalize_blocks(const Geometry& g);
int apply_multi_groups(const Geometry& g);
hipError_t launch_fft_multi(const MultiProblem* mp, const unsigned* map_cols, int n_cols, const unsigned* map_rows,
                            int n_rows, int first, size_t lds_cols, size_t lds_rows, hipStream_t st);
// Every screen step of a multi-problem group in one cooperative launch
// (superpose.hip); n[q] = map entries of the four stages at step q.
hipError_t launch_multi_persistent(const MultiProblem* mp, const unsigned* map_cols, const unsigned* map_rows,
                                   const unsigned* map_apply, const unsigned* map_fin, const int4* n, int* ctr,
                                   int qmax, size_t lds, int max_blocks, hipStream_t st, int* blocks_out);
size_t apply_lds_bytes();
int apply_f64_sub(const Geometry& g);
int apply_f64_groups(const Geometry& g);
hipError_t launch_apply_multi(const MultiProblem* mp, const unsigned* map_apply, int n_apply,
                              const unsigned* map_fin, int n_fin, int step, hipStream_t st);
// Inside the library: a multi-problem group whose problems read their fields
// from fixed inputs, one screen step at a time (multi.hip).
hipError_t multi_set_inputs(swkb_multi_s* m, const double2* const* inputs);
hipError_t multi_step(swkb_multi_s* m, int q, hipStream_t st);
hipError_t multi_mark(swkb_multi_s* m, hipStream_t st);
hipError_t launch_export_rays(const swkb_plan_s& pl, int q, double* Z, double* psi, double* qz,
                              double* amp, int* flag, hipStream_t st);

}  // namespace swkb
