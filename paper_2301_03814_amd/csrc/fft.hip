// Step 1 of a screen: vertical DFT of the screen field and selection of the
// kept modes (Sec. 2.1.1, eqs. fft_eq / ifft_eq; the 1/P of the inverse
// transform is folded into the mode amplitudes).
//
// Four-step FFT of length P = P1 * P2 (input index i = P2 m1 + m2, output
// index n = n1 + P1 n2):
//   fft_cols: for each column m2, a length-P1 FFT over m1 in LDS, then the
//             twiddle e^{-2 pi i n1 m2 / P}; writes Y[n1][m2];
//   fft_rows: for each row n1, a length-P2 FFT over m2 in LDS; writes only
//             the M kept bins n in [-M/2, M/2), scaled by 1/P.
// Both sub-FFTs are in-place radix-2 (bit-reversed load) in LDS, several
// short sequences per workgroup so that global loads and stores move
// contiguous runs.  The ground-mirror extension of the field (Sec. 2.3) is
// applied on the fly in fft_cols' loads.
#include "fft_body.h"
#include "swkb_internal.h"

namespace swkb {
namespace {

using fftb::fft_cols_body;
using fftb::fft_rows_body;

__global__ void __launch_bounds__(256) fft_cols(const double2* __restrict__ u, double2* __restrict__ Y,
                                                const double2* __restrict__ tw, int N, int bc, int P, int P1,
                                                int P2, int logP1, int CA) {
  extern __shared__ double2 L[];
  fft_cols_body(u + (size_t)blockIdx.y * N, Y + (size_t)blockIdx.y * P, tw, N, bc, P, P1, P2, logP1, CA,
                blockIdx.x, L);
}

__global__ void __launch_bounds__(256) fft_rows(const double2* __restrict__ Y, double2* __restrict__ c,
                                                const double2* __restrict__ tw, int P, int P1, int P2,
                                                int logP2, int RB, int M, float2* __restrict__ cp) {
  extern __shared__ double2 L[];
  fft_rows_body(Y + (size_t)blockIdx.y * P, c + (size_t)blockIdx.y * M, tw, P, P1, P2, logP2, RB, M, blockIdx.x,
                L, cp);
}

// The two passes for many problems in one launch each: workgroup b runs
// local workgroup map[b] & 0xfffff of problem map[b] >> 20.  A screen's
// input is u_in on the problem's first step, its field u afterwards.
__global__ void __launch_bounds__(256) fft_cols_multi(const MultiProblem* __restrict__ mp,
                                                      const unsigned* __restrict__ map, int first) {
  extern __shared__ double2 L[];
  const unsigned e = map[blockIdx.x];
  const MultiProblem& p = mp[e >> 20];
  fft_cols_body(first ? p.u_in : p.u, p.Y, p.tw, p.g.N, p.g.bc, p.g.P, p.g.P1, p.g.P2, p.logP1, p.CA, e & 0xfffff,
                L);
}

__global__ void __launch_bounds__(256) fft_rows_multi(const MultiProblem* __restrict__ mp,
                                                      const unsigned* __restrict__ map) {
  extern __shared__ double2 L[];
  const unsigned e = map[blockIdx.x];
  const MultiProblem& p = mp[e >> 20];
  fft_rows_body(p.Y, p.c, p.tw, p.g.P, p.g.P1, p.g.P2, p.logP2, p.RB, p.g.M, e & 0xfffff, L);
}

}  // namespace

int ilog2(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

void fft_blocking(const Geometry& g, int elems, int* CA, int* RB) {
  int ca = elems / g.P1;
  if (ca < 1) ca = 1;
  if (ca > g.P2) ca = g.P2;
  int rb = elems / g.P2;
  if (rb < 1) rb = 1;
  if (rb > g.P1) rb = g.P1;
  *CA = ca;
  *RB = rb;
}

hipError_t launch_fft_modes(const swkb_plan_s& pl, const double2* u, int batch, hipStream_t st) {
  const Geometry& g = pl.g;
  // about 512 elements per workgroup: one butterfly per thread and stage, and
  // P / 512 workgroups working on the latency-bound stages in parallel
  int CA, RB;
  fft_blocking(g, kFftElems, &CA, &RB);
  hipLaunchKernelGGL(fft_cols, dim3(g.P2 / CA, batch), dim3(256), sizeof(double2) * (CA * g.P1 + g.P1 / 2), st, u,
                     pl.Y, pl.tw,
                     g.N, g.bc, g.P, g.P1, g.P2, ilog2(g.P1), CA);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fft_rows, dim3(g.P1 / RB, batch), dim3(256), sizeof(double2) * (RB * g.P2 + g.P2 / 2), st,
                     pl.Y, pl.c, pl.tw,
                     g.P, g.P1, g.P2, ilog2(g.P2), RB, g.M, batch == 1 ? pl.cpol : nullptr);
  return hipGetLastError();
}

hipError_t launch_fft_multi(const MultiProblem* mp, const unsigned* map_cols, int n_cols, const unsigned* map_rows,
                            int n_rows, int first, size_t lds_cols, size_t lds_rows, hipStream_t st) {
  hipLaunchKernelGGL(fft_cols_multi, dim3(n_cols), dim3(256), lds_cols, st, mp, map_cols, first);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fft_rows_multi, dim3(n_rows), dim3(256), lds_rows, st, mp, map_rows);
  return hipGetLastError();
}

}  // namespace swkb
