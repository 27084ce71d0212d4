// Device bodies of the screen FFT (Sec. 2.1.1, eqs. fft_eq / ifft_eq): the
// column and row passes of the four-step transform described in fft.hip,
// shared by its kernels and by the multi-problem persistent kernel.
#pragma once

#include "swkb_internal.h"

namespace swkb {
namespace fftb {

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline int bitrev(int x, int bits) { return (int)(__brev((unsigned)x) >> (32 - bits)); }

// Element i in [0, P) of the periodic vector whose DFT gives the modes.
// Mirror: v[N+m] = u[m]; v[N-m] = -/+ u[m] (Dirichlet / Neumann);
// v[0] = 0; v[N] = 0 for Dirichlet.
__device__ inline double2 extended(const double2* __restrict__ u, int i, int N, int bc) {
  if (bc == SWKB_BC_PERIODIC) return u[i];
  if (i > N) return u[i - N];
  if (i == N) return bc == SWKB_BC_DIRICHLET ? make_double2(0.0, 0.0) : u[0];
  if (i == 0) return make_double2(0.0, 0.0);
  double2 x = u[N - i];
  return bc == SWKB_BC_DIRICHLET ? make_double2(-x.x, -x.y) : x;
}

// nb sequences of length len (power of two) stored at L[b * len + i] in
// bit-reversed order; in-place radix-2 decimation in time.  The twiddle of
// butterfly k at half-size hs is e^{-2 pi i k / (2 hs)} = wl[k * len / (2 hs)],
// wl[k] = e^{-2 pi i k / len} (k < len / 2) staged in LDS.  Two consecutive
// stages (half-sizes hs and 2 hs) run together from registers: a thread
// takes the four elements base + {0, 1, 2, 3} hs that the two stages' four
// butterflies connect, so each pair of stages costs one LDS round trip and
// one barrier; the butterflies and their twiddles are those of the radix-2
// stages (a last stage runs alone when the number of stages is odd).
__device__ inline void lds_fft(double2* L, int nb, int len, const double2* wl) {
  int hs = 1;
  for (; 4 * hs <= len; hs <<= 2) {
    const int quarter = len >> 2;
    const int ta = len / (2 * hs), tb = ta >> 1;  // twiddle strides of the two stages
    for (int q = threadIdx.x; q < nb * quarter; q += blockDim.x) {
      const int seq = q / quarter, r = q - seq * quarter;
      const int grp = r / hs, kk = r - grp * hs;
      const int i0 = seq * len + grp * 4 * hs + kk;
      const double2 wa = wl[kk * ta], wb0 = wl[kk * tb], wb1 = wl[(kk + hs) * tb];
      const double2 x0 = L[i0], x1 = cmul(L[i0 + hs], wa);
      const double2 x2 = L[i0 + 2 * hs], x3 = cmul(L[i0 + 3 * hs], wa);
      // half-size hs: (i0, i0 + hs) and (i0 + 2 hs, i0 + 3 hs)
      const double2 a0 = make_double2(x0.x + x1.x, x0.y + x1.y), a1 = make_double2(x0.x - x1.x, x0.y - x1.y);
      const double2 a2 = make_double2(x2.x + x3.x, x2.y + x3.y), a3 = make_double2(x2.x - x3.x, x2.y - x3.y);
      // half-size 2 hs: (i0, i0 + 2 hs) at k = kk, (i0 + hs, i0 + 3 hs) at k = kk + hs
      const double2 b2 = cmul(a2, wb0), b3 = cmul(a3, wb1);
      L[i0] = make_double2(a0.x + b2.x, a0.y + b2.y);
      L[i0 + 2 * hs] = make_double2(a0.x - b2.x, a0.y - b2.y);
      L[i0 + hs] = make_double2(a1.x + b3.x, a1.y + b3.y);
      L[i0 + 3 * hs] = make_double2(a1.x - b3.x, a1.y - b3.y);
    }
    __syncthreads();
  }
  if (hs < len) {  // one radix-2 stage left (hs = len / 2)
    const int half = len >> 1;
    const int tstride = len / (2 * hs);
    for (int b = threadIdx.x; b < nb * half; b += blockDim.x) {
      const int seq = b / half, bb = b - seq * half;
      const int grp = bb / hs, kk = bb - grp * hs;
      const int i0 = seq * len + grp * 2 * hs + kk, i1 = i0 + hs;
      const double2 w = wl[kk * tstride];
      const double2 x0 = L[i0];
      const double2 x1 = cmul(L[i1], w);
      L[i0] = make_double2(x0.x + x1.x, x0.y + x1.y);
      L[i1] = make_double2(x0.x - x1.x, x0.y - x1.y);
    }
    __syncthreads();
  }
}

// Column pass of one field: workgroup bx of P2 / CA.  L holds CA sequences of
// length P1, then P1 / 2 twiddles.
__device__ inline void fft_cols_body(const double2* __restrict__ u, double2* __restrict__ Y,
                                     const double2* __restrict__ tw, int N, int bc, int P, int P1, int P2,
                                     int logP1, int CA, int bx, double2* L) {
  double2* wl = L + CA * P1;
  const int c0 = bx * CA;
  for (int k = threadIdx.x; k < P1 / 2; k += blockDim.x) wl[k] = tw[k * (P / P1)];
  for (int idx = threadIdx.x; idx < CA * P1; idx += blockDim.x) {
    const int cc = idx % CA, m1 = idx / CA;
    L[cc * P1 + bitrev(m1, logP1)] = extended(u, P2 * m1 + c0 + cc, N, bc);
  }
  __syncthreads();
  lds_fft(L, CA, P1, wl);
  for (int idx = threadIdx.x; idx < CA * P1; idx += blockDim.x) {
    const int cc = idx % CA, n1 = idx / CA, m2 = c0 + cc;
    Y[n1 * P2 + m2] = cmul(L[cc * P1 + n1], tw[n1 * m2]);  // n1 m2 < P
  }
}

// Row pass of one field: workgroup bx of P1 / RB; writes the M kept bins.
// With cp set (one field), each kept bin is also written in polar form for
// the FP32 interval sum: modulus, and argument in turns in [0, 1), both
// rounded once from FP64.
__device__ inline void fft_rows_body(const double2* __restrict__ Y, double2* __restrict__ c,
                                     const double2* __restrict__ tw, int P, int P1, int P2, int logP2, int RB,
                                     int M, int bx, double2* L, float2* __restrict__ cp = nullptr) {
  double2* wl = L + RB * P2;
  const int r0 = bx * RB;
  for (int k = threadIdx.x; k < P2 / 2; k += blockDim.x) wl[k] = tw[k * (P / P2)];
  for (int idx = threadIdx.x; idx < RB * P2; idx += blockDim.x) {
    const int rr = idx / P2, m2 = idx - rr * P2;
    L[rr * P2 + bitrev(m2, logP2)] = Y[(r0 + rr) * P2 + m2];
  }
  __syncthreads();
  lds_fft(L, RB, P2, wl);
  const double inv = 1.0 / (double)P;  // exact: P is a power of two
  const int halfM = M >> 1;
  for (int idx = threadIdx.x; idx < RB * P2; idx += blockDim.x) {
    const int rr = idx / P2, n2 = idx - rr * P2;
    const int n = (r0 + rr) + P1 * n2;
    int j = -1;
    if (n < halfM) j = n + halfM;
    else if (n >= P - halfM) j = n - P + halfM;
    if (j >= 0) {
      const double2 x = L[rr * P2 + n2];
      const double cr = x.x * inv, ci = x.y * inv;
      c[j] = make_double2(cr, ci);
      if (cp) {
        double t = atan2(ci, cr) * (0.5 / M_PI);
        t -= floor(t);
        cp[j] = make_float2((float)sqrt(cr * cr + ci * ci), (float)t);
      }
    }
  }
}

}  // namespace fftb
}  // namespace swkb
