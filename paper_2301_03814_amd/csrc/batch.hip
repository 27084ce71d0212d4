// Several sources through the mode-function matrix of a medium that does not
// depend on x: for B fields on one screen the sums over modes
//   U[b][m] = sum_j c[b][j] T[j][m]        (eq. ray_bundle_q_plus_1, T tabulated once)
// are one complex matrix product of the streamed matrix T (N points x M
// modes) with the B fields' mode amplitudes, computed on the matrix cores.
//
// Written as a real product: with T = Tr + i Ti and c = cr + i ci,
//   Re U = sum_j (Tr cr - Ti ci),  Im U = sum_j (Ti cr + Tr ci),
// the reduction index is (mode j, component of T) and the output columns are
// (field b, component of U): column 2 b takes cr from the Re T row and -ci
// from the Im T row, column 2 b + 1 takes ci and cr.  A small kernel lays
// these B operands out once per screen in the matrix instruction's lane
// order (the "panel"); the A operand is read straight from T's interleaved
// complex rows, each lane loading one whole complex entry.
//
// complex64 T (mixed precision): v_mfma_f32_32x32x2f32, 32 points x
//   (16 fields x Re/Im) per instruction; lanes i and i + 32 load point i of
//   modes 2p and 2p + 1, so one instruction reduces over Re T of the pair
//   and a second one over Im T (K = 2 = the two modes).
// complex128 T (FP64): v_mfma_f64_16x16x4f64, 16 points x (8 fields x
//   Re/Im); lane i + 16 k loads point i of mode 4q + k, one instruction per
//   component (K = 4 = the four modes).
// Lane layouts (checked on the MI355X with integer products): A[i][k] from
// lane i + 32k (resp. 16k), B[k][n] from lane n + 32k (16k); the f32 result
// D[row][col] is register r of lane l with col = l % 32, row = 8 (r/4) +
// 4 (l/32) + r % 4; the f64 result has col = l % 16, row = 4 r + l / 16.
//
// The modes are split into interleaved groups (one workgroup per point block
// and mode group) so that the chip fills; each group's partial sums (FP32 or
// FP64) are added in a fixed order in FP64 by the epilogue, as in the
// one-field product.  The panel (M x 256 bytes per column tile) stays in the
// cache: the product reads T once from HBM and nothing else.
#include "swkb_internal.h"

namespace swkb {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kBWaves = 8;     // wavefronts per workgroup
constexpr int kChunkF32 = 4;   // mode pairs per operand chunk (FP32)
constexpr int kChunkF64 = 2;   // mode quads per operand chunk (FP64)
constexpr int kMaxTiles = 4;   // column tiles per pass (FP32: 64 fields, FP64: 32 fields)

// B operand for column n = 2 b + cp (field b, component cp of U) and row
// k = component cc of T:  cr if cc == cp, else ci (cc = Re) or -ci (cc = Im).
__device__ inline double panel_value(const double2 cv, int cc, int cp) {
  return cc == cp ? cv.x : (cc == 0 ? cv.y : -cv.y);
}

// The panel kernels' last ceil(M / 256) workgroups (when energy is given):
// each mode's energy summed over the B fields, for the epilogue's
// diagnostics, which then read M values instead of B M coefficients in one
// workgroup.  Workgroup e takes modes 256 e + thread.
__device__ inline void mode_energies(const double2* __restrict__ c, int M, int B, unsigned e,
                                     double* __restrict__ energy) {
  const int j = (int)(e * blockDim.x + threadIdx.x);
  if (j < M) energy[j] = batch_energy(c, M, j, B);
}

// FP32 panel [mode pair p][cc][tile][lane]: lane l = n + 32 k holds row k =
// mode 2 p + k (component cc of T), column n; tile t covers fields 16 t ..
// 16 t + 15.
__global__ void panel_f32_kernel(const double2* __restrict__ c, int M, int B, int tiles, float* __restrict__ pan,
                                 unsigned pblocks, double* __restrict__ energy) {
  if (blockIdx.x >= pblocks) {
    mode_energies(c, M, B, blockIdx.x - pblocks, energy);
    return;
  }
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)M * tiles * 64) return;
  const int l = (int)(i & 63), t = (int)((i >> 6) % tiles);
  const size_t pc = i / ((size_t)tiles * 64);
  const int cc = (int)(pc & 1), j = (int)(pc >> 1) * 2 + (l >> 5);
  const int n = l & 31, b = 16 * t + (n >> 1);
  pan[i] = b < B ? (float)panel_value(c[(size_t)b * M + j], cc, n & 1) : 0.0f;
}

// FP64 panel [mode quad q][cc][tile][lane]: lane l = n + 16 k holds row k =
// mode 4 q + k (zero past the last mode), column n; tile t covers fields
// 8 t .. 8 t + 7.
__global__ void panel_f64_kernel(const double2* __restrict__ c, int M, int B, int tiles, double* __restrict__ pan,
                                 unsigned pblocks, double* __restrict__ energy) {
  if (blockIdx.x >= pblocks) {
    mode_energies(c, M, B, blockIdx.x - pblocks, energy);
    return;
  }
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int quads = (M + 3) / 4;
  if (i >= (size_t)quads * 2 * tiles * 64) return;
  const int l = (int)(i & 63), t = (int)((i >> 6) % tiles);
  const size_t qc = i / ((size_t)tiles * 64);
  const int cc = (int)(qc & 1), j = (int)(qc >> 1) * 4 + (l >> 4);
  const int n = l & 15, b = 8 * t + (n >> 1);
  pan[i] = b < B && j < M ? panel_value(c[(size_t)b * M + j], cc, n & 1) : 0.0;
}

typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef double doublex2 __attribute__((ext_vector_type(2)));

// complex64 T [M][N] times the FP32 panel; part [B][G][N] complex64.
// Wavefront w of workgroup (bx, gi, pass) takes NR row tiles of 32 points
// from 32 NR (8 bx + w), the mode pairs of group gi and column tiles
// NT pass .. NT pass + NT - 1.  Lane i + 32 k loads the whole complex entry
// of point i for mode 2 p + k (one coalesced 8-byte load per lane); its Re
// part feeds one instruction (reduction rows: Re T of modes 2 p, 2 p + 1),
// its Im part a second one, against the panel rows of that component.  Per
// chunk of CH mode pairs a wavefront requests every operand first (T
// non-temporal, streamed once per screen; the panel, shared by the whole
// screen, from the cache) and multiplies after; the panel values of a mode
// serve NR row tiles.  Points past N repeat the last point (in bounds, not
// stored).
template <int NR, int NT, int CH>
__global__ void __launch_bounds__(64 * kBWaves) batch_f32_kernel(int N, int B, int pend, int tiles,
                                                                 const floatx2* __restrict__ T,
                                                                 const float* __restrict__ pan,
                                                                 float2* __restrict__ part, int G) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = (blockIdx.x * kBWaves + w) * 32 * NR;
  if (m0 >= N) return;  // uniform per wavefront
  const int gi = blockIdx.y, t0 = blockIdx.z * NT;
  const int np = (pend - gi + G - 1) / G;  // mode pairs gi, gi + G, gi + 2 G, ... of this group
  floatx16 acc[NR][NT];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[r][t][q] = 0.0f;
  const floatx2* __restrict__ ta[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) ta[r] = T + (size_t)(lane >> 5) * N + min(m0 + 32 * r + (lane & 31), N - 1);
  for (int i0 = 0; i0 < np; i0 += CH) {
    const int cnt = min(CH, np - i0);
    floatx2 a[CH][NR];
    float bv[CH][2][NT];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int p = gi + (i0 + min(u, cnt - 1)) * G;
#pragma unroll
      for (int r = 0; r < NR; ++r) a[u][r] = __builtin_nontemporal_load(ta[r] + (size_t)p * 2 * N);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          bv[u][cc][t] = t0 + t < tiles ? pan[(((size_t)p * 2 + cc) * tiles + t0 + t) * 64 + lane] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (u < cnt)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            acc[r][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u][r].x, bv[u][0][t], acc[r][t], 0, 0, 0);
            acc[r][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u][r].y, bv[u][1][t], acc[r][t], 0, 0, 0);
          }
  }
  const int col = lane & 31, cp = col & 1;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = 16 * (t0 + t) + (col >> 1);
    if (b >= B) continue;
    float* dst = reinterpret_cast<float*>(part + ((size_t)b * G + gi) * N) + cp;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int m = m0 + 32 * r + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        if (m < N) dst[2 * m] = acc[r][t][q];
      }
  }
}

// complex128 T [M][N] times the FP64 panel; part [B][G][N] complex128.
// Wavefront w takes NR row tiles of 16 points from 16 NR (8 bx + w); lane
// i + 16 k loads the complex entry of point i for mode 4 q + k (16 bytes,
// row clamped to the last mode, whose panel rows are zero); Re and Im feed
// one instruction each (reduction rows: that component of 4 modes).
template <int NR, int NT, int CH>
__global__ void __launch_bounds__(64 * kBWaves) batch_f64_kernel(int N, int M, int B, int qend, int tiles,
                                                                 const doublex2* __restrict__ T,
                                                                 const double* __restrict__ pan,
                                                                 double2* __restrict__ part, int G) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = (blockIdx.x * kBWaves + w) * 16 * NR;
  if (m0 >= N) return;  // uniform per wavefront
  const int gi = blockIdx.y, t0 = blockIdx.z * NT;
  const int nq = (qend - gi + G - 1) / G;  // mode quads gi, gi + G, gi + 2 G, ... of this group
  doublex4 acc[NR][NT];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[r][t][q] = 0.0;
  const int k = lane >> 4;
  int pt[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) pt[r] = min(m0 + 16 * r + (lane & 15), N - 1);
  for (int i0 = 0; i0 < nq; i0 += CH) {
    const int cnt = min(CH, nq - i0);
    doublex2 a[CH][NR];
    double bv[CH][2][NT];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int q = gi + (i0 + min(u, cnt - 1)) * G;
      const size_t row = (size_t)min(4 * q + k, M - 1) * N;
#pragma unroll
      for (int r = 0; r < NR; ++r) a[u][r] = __builtin_nontemporal_load(T + row + pt[r]);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          bv[u][cc][t] = t0 + t < tiles ? pan[(((size_t)q * 2 + cc) * tiles + t0 + t) * 64 + lane] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (u < cnt)
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            acc[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][r].x, bv[u][0][t], acc[r][t], 0, 0, 0);
            acc[r][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][r].y, bv[u][1][t], acc[r][t], 0, 0, 0);
          }
  }
  const int col = lane & 15, cp = col & 1;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = 8 * (t0 + t) + (col >> 1);
    if (b >= B) continue;
    double* dst = reinterpret_cast<double*>(part + ((size_t)b * G + gi) * N) + cp;
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + 16 * r + 4 * q + (lane >> 4);
        if (m < N) dst[2 * m] = acc[r][t][q];
      }
  }
}

int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Column tiles of the panel and per pass.
int panel_tiles(int precision, int B) { return ceil_div(B, precision == SWKB_FP64 ? 8 : 16); }
int pass_tiles(int tiles) { return tiles < kMaxTiles ? tiles : kMaxTiles; }

// Row tiles per wavefront for NT column tiles per pass (accumulators: 16
// FP32 or 8 FP64 registers per row and column tile, at most 64).
int row_tiles(int precision, int nt) {
  if (precision == SWKB_FP64) return nt == 1 ? 4 : 2;
  return nt <= 2 ? 2 : 1;
}

// Wavefronts a product aims for: on the MI355X (256 compute units) the FP32
// product ran fastest with one workgroup of 8 wavefronts per compute unit
// (N = 16384, M = 4096, 16 fields: 118 us against 160 us with two and 214 us
// with an uneven 1.25), the FP64 product with two.
int target_waves(int precision) { return precision == SWKB_FP64 ? 4096 : 2048; }

// Points per wavefront, modes per operand chunk.
int wave_points(int precision, int nt) { return (precision == SWKB_FP64 ? 16 : 32) * row_tiles(precision, nt); }
int chunk_modes(int precision) { return precision == SWKB_FP64 ? 4 * kChunkF64 : 2 * kChunkF32; }

}  // namespace

// Mode groups of a batched product: about target_waves wavefronts over the
// chip and at least one operand chunk per group.  Group gi takes the mode
// pairs (FP32) or quads (FP64) gi, gi + G, gi + 2 G, ...: at any moment the
// groups stream neighbouring rows of T.
int batch_groups(const Geometry& g, int precision, int B) {
  const int tiles = panel_tiles(precision, B);
  const int nt = pass_tiles(tiles);
  const int waves = ceil_div(g.N, wave_points(precision, nt)) * ceil_div(tiles, nt);
  int G = ceil_div(target_waves(precision), waves);
  const int gmax = ceil_div(g.M, chunk_modes(precision));
  if (G > gmax) G = gmax;
  return G < 1 ? 1 : G;
}

// Largest partial-sum buffer a product of 2 .. Bmax fields writes ([B][G][N]).
size_t batch_part_bytes(const Geometry& g, int precision, int Bmax) {
  size_t most = 0;
  for (int b = 2; b <= Bmax; ++b) {
    const size_t s = (size_t)b * batch_groups(g, precision, b) * g.N;
    most = s > most ? s : most;
  }
  return most * (precision == SWKB_FP64 ? sizeof(double2) : sizeof(float2));
}

size_t batch_panel_bytes(const Geometry& g, int B) {
  // FP64: ceil(M/4) quads x 2 components x ceil(B/8) tiles x 64 doubles; the
  // FP32 panel (M/2 pairs x 2 x ceil(B/16) x 64 floats) is never larger
  return (size_t)ceil_div(g.M, 4) * 2 * panel_tiles(SWKB_FP64, B) * 64 * sizeof(double);
}

static unsigned energy_blocks(const swkb_plan_s& pl) {
  return pl.menergy ? (unsigned)ceil_div(pl.g.M, 256) : 0u;
}

hipError_t launch_batch_product(const swkb_plan_s& pl, int batch, hipStream_t st, int* groups_out) {
  const Geometry& g = pl.g;
  const int prec = pl.precision;
  const int tiles = panel_tiles(prec, batch);
  const int nt = pass_tiles(tiles);
  const int passes = ceil_div(tiles, nt);
  const int G = batch_groups(g, prec, batch);
  *groups_out = G;
  const dim3 grid(ceil_div(ceil_div(g.N, wave_points(prec, nt)), kBWaves), G, passes), blk(64 * kBWaves);
  if (prec == SWKB_FP64) {
    const int quads = ceil_div(g.M, 4);
    const size_t n = (size_t)quads * 2 * tiles * 64;
    const unsigned pb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(panel_f64_kernel, dim3(pb + energy_blocks(pl)), dim3(256), 0, st, pl.c, g.M, batch, tiles,
                       static_cast<double*>(pl.pan), pb, pl.menergy);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const doublex2* T = static_cast<const doublex2*>(pl.tmat);
    const double* P = static_cast<const double*>(pl.pan);
    double2* part = pl.part;
    switch (nt) {
      case 1: hipLaunchKernelGGL((batch_f64_kernel<4, 1, kChunkF64>), grid, blk, 0, st, g.N, g.M, batch, quads, tiles, T, P, part, G); break;
      case 2: hipLaunchKernelGGL((batch_f64_kernel<2, 2, kChunkF64>), grid, blk, 0, st, g.N, g.M, batch, quads, tiles, T, P, part, G); break;
      case 3: hipLaunchKernelGGL((batch_f64_kernel<2, 3, kChunkF64>), grid, blk, 0, st, g.N, g.M, batch, quads, tiles, T, P, part, G); break;
      default: hipLaunchKernelGGL((batch_f64_kernel<2, 4, kChunkF64>), grid, blk, 0, st, g.N, g.M, batch, quads, tiles, T, P, part, G); break;
    }
    return hipGetLastError();
  }
  const int pairs = g.M / 2;
  const size_t n = (size_t)g.M * tiles * 64;
  const unsigned pb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(panel_f32_kernel, dim3(pb + energy_blocks(pl)), dim3(256), 0, st, pl.c, g.M, batch, tiles,
                     static_cast<float*>(pl.pan), pb, pl.menergy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const floatx2* T = static_cast<const floatx2*>(pl.tmat);
  const float* P = static_cast<const float*>(pl.pan);
  float2* part = reinterpret_cast<float2*>(pl.part);
  switch (nt) {
    case 1: hipLaunchKernelGGL((batch_f32_kernel<2, 1, kChunkF32>), grid, blk, 0, st, g.N, batch, pairs, tiles, T, P, part, G); break;
    case 2: hipLaunchKernelGGL((batch_f32_kernel<2, 2, kChunkF32>), grid, blk, 0, st, g.N, batch, pairs, tiles, T, P, part, G); break;
    case 3: hipLaunchKernelGGL((batch_f32_kernel<1, 3, kChunkF32>), grid, blk, 0, st, g.N, batch, pairs, tiles, T, P, part, G); break;
    default: hipLaunchKernelGGL((batch_f32_kernel<1, 4, kChunkF32>), grid, blk, 0, st, g.N, batch, pairs, tiles, T, P, part, G); break;
  }
  return hipGetLastError();
}

}  // namespace swkb
