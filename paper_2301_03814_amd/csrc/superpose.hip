// Steps 3 and 4 of a screen, fused: interpolation of each mode's ray
// arrivals onto the grid of screen x_{q+1} (Sec. 2.1.2) and the sum over
// modes (eq. ray_bundle_q_plus_1), followed by the exit epilogue (cos^2
// taper at open ends) and the writes of the new screen field.
//
// Layout: one workgroup per tile of 64 consecutive grid points (lane =
// point), `ms` wavefronts per workgroup splitting the modes round-robin;
// the per-wavefront partial sums are reduced in LDS in a fixed order, so the
// result does not depend on scheduling.  No [mode][point] intermediate is
// ever written to memory.
//
// Per (mode, point): the bracket is the largest ray r with key_r <= z_m,
// searched inside the tile's window [tstart[t], tstart[t+1]]; it
// contributes when rays r and r+1 are both live.  dpsi: cubic Hermite with
// end slopes q - xi (dpsi_z at fixed x); amplitude: 4-point Lagrange over
// r-1..r+2 when all four are live, else linear.  The phase in turns is
//   (n m' mod P)/P + frac(pbar dx / lambda) + dpsi / lambda,
// the first term exact in integers.
#include <type_traits>

#include "swkb_internal.h"

namespace swkb {
namespace {

struct Epi {
  double absorber_bot, absorber_top;
  double caustic_tol;
  int mprime_off;  // m' = m + mprime_off (grid index from the phase origin)
};

__device__ inline double taper(const Geometry& g, const Epi& e, double z) {
  double w = 1.0;
  if (e.absorber_bot > 0.0 && z < g.z_a + e.absorber_bot) {
    const double c = cospi(0.5 * ((g.z_a + e.absorber_bot - z) / e.absorber_bot));
    w *= c * c;
  }
  if (e.absorber_top > 0.0 && z > g.z_b - e.absorber_top) {
    const double c = cospi(0.5 * ((z - (g.z_b - e.absorber_top)) / e.absorber_top));
    w *= c * c;
  }
  return w;
}

template <typename T>
__global__ void __launch_bounds__(1024) superpose_kernel(Geometry g, DevModes modes, DevRecords rec,
                                                         const double2* __restrict__ c, double2* __restrict__ out,
                                                         double2* __restrict__ hist,
                                                         unsigned long long* __restrict__ counters, Epi ep, int ms) {
  extern __shared__ double2 red[];  // ms * 64
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int t = blockIdx.x;
  const int m = t * kTile + lane;
  const double zm = g.z_a + (double)m * g.h;
  const long long mp = (long long)m + ep.mprime_off;
  const double inv_lam = 1.0 / g.lam;
  const T* __restrict__ D = static_cast<const T*>(rec.D);
  const T* __restrict__ Pp = static_cast<const T*>(rec.Pp);
  const T* __restrict__ G = static_cast<const T*>(rec.G);
  const T* __restrict__ A = static_cast<const T*>(rec.A);

  double re = 0.0, im = 0.0;  // FP64 path accumulators
  float ref = 0.f, imf = 0.f; // mixed path accumulators (per wavefront)
  for (int j = w; j < g.M; j += ms) {
    if (rec.mflag[j] & 1) continue;  // folded mode
    const int* ts = rec.tstart + (size_t)j * (g.T + 1);
    int lo = ts[t], hi = ts[t + 1];
    const size_t base = (size_t)j * g.R;
    const double* __restrict__ key = rec.key + base;
    while (hi > lo) {
      const int mid = (lo + hi + 1) >> 1;
      if (key[mid] <= zm) lo = mid;
      else hi = mid - 1;
    }
    const int r = lo;
    if (r < 0 || r >= g.R - 1) continue;
    const T a0 = A[base + r], a1 = A[base + r + 1];
    if (!(a0 > T(0) && a1 > T(0))) continue;
    const bool cubic = r >= 1 && r + 2 < g.R && A[base + r - 1] > T(0) && A[base + r + 2] > T(0);
    const long long n = (long long)j - (g.M >> 1);
    long long nm = (n * mp) % g.P;
    if (nm < 0) nm += g.P;
    if constexpr (std::is_same<T, double>::value) {
      const double sr = g.z_a + (double)(r * g.rho - g.E) * g.h;
      const double Z0 = sr + D[base + r];
      const double Z1 = (g.z_a + (double)((r + 1) * g.rho - g.E) * g.h) + D[base + r + 1];
      const double H = Z1 - Z0;
      const double tt = (zm - Z0) / H;
      const double t2 = tt * tt, t3 = t2 * tt;
      const double dps = (2 * t3 - 3 * t2 + 1) * Pp[base + r] + (t3 - 2 * t2 + tt) * H * G[base + r] +
                         (-2 * t3 + 3 * t2) * Pp[base + r + 1] + (t3 - t2) * H * G[base + r + 1];
      double a;
      if (cubic) {
        const double x0 = (g.z_a + (double)((r - 1) * g.rho - g.E) * g.h) + D[base + r - 1];
        const double x3 = (g.z_a + (double)((r + 2) * g.rho - g.E) * g.h) + D[base + r + 2];
        const double x1 = Z0, x2 = Z1;
        const double l0 = (zm - x1) * (zm - x2) * (zm - x3) / ((x0 - x1) * (x0 - x2) * (x0 - x3));
        const double l1 = (zm - x0) * (zm - x2) * (zm - x3) / ((x1 - x0) * (x1 - x2) * (x1 - x3));
        const double l2 = (zm - x0) * (zm - x1) * (zm - x3) / ((x2 - x0) * (x2 - x1) * (x2 - x3));
        const double l3 = (zm - x0) * (zm - x1) * (zm - x2) / ((x3 - x0) * (x3 - x1) * (x3 - x2));
        a = l0 * A[base + r - 1] + l1 * a0 + l2 * a1 + l3 * A[base + r + 2];
      } else {
        a = (1.0 - tt) * a0 + tt * a1;
      }
      double turns = (double)nm / (double)g.P + modes.frac[j] + dps * inv_lam;
      turns -= floor(turns);
      double sn, cs;
      sincospi(2.0 * turns, &sn, &cs);
      const double2 cj = c[j];
      const double er = a * cs, ei = a * sn;
      re += cj.x * er - cj.y * ei;
      im += cj.x * ei + cj.y * er;
    } else {
      // heights relative to Z_r: (m - r rho + E) h - D_r, small numbers in FP32
      const float hf = (float)g.h;
      const float rh = (float)g.rho * hf;
      const float d0 = D[base + r], d1 = D[base + r + 1];
      const float zr = (float)(m - r * g.rho + g.E) * hf - d0;  // z_m - Z_r
      const float H = rh + (d1 - d0);
      const float tt = zr / H;
      const float t2 = tt * tt, t3 = t2 * tt;
      const float dps = (2.f * t3 - 3.f * t2 + 1.f) * Pp[base + r] + (t3 - 2.f * t2 + tt) * H * G[base + r] +
                        (-2.f * t3 + 3.f * t2) * Pp[base + r + 1] + (t3 - t2) * H * G[base + r + 1];
      float a;
      if (cubic) {
        const float x0 = -rh + (D[base + r - 1] - d0);
        const float x1 = 0.f, x2 = H;
        const float x3 = 2.f * rh + (D[base + r + 2] - d0);
        const float l0 = (zr - x1) * (zr - x2) * (zr - x3) / ((x0 - x1) * (x0 - x2) * (x0 - x3));
        const float l1 = (zr - x0) * (zr - x2) * (zr - x3) / ((x1 - x0) * (x1 - x2) * (x1 - x3));
        const float l2 = (zr - x0) * (zr - x1) * (zr - x3) / ((x2 - x0) * (x2 - x1) * (x2 - x3));
        const float l3 = (zr - x0) * (zr - x1) * (zr - x2) / ((x3 - x0) * (x3 - x1) * (x3 - x2));
        a = l0 * (float)A[base + r - 1] + l1 * (float)a0 + l2 * (float)a1 + l3 * (float)A[base + r + 2];
      } else {
        a = (1.f - tt) * (float)a0 + tt * (float)a1;
      }
      float turns = (float)nm / (float)g.P + (float)modes.frac[j] + dps * (float)inv_lam;
      turns -= floorf(turns);
      const float sn = __builtin_amdgcn_sinf(turns);  // argument in revolutions
      const float cs = __builtin_amdgcn_cosf(turns);
      const double2 cjd = c[j];
      const float cr = (float)cjd.x, ci = (float)cjd.y;
      const float er = a * cs, ei = a * sn;
      ref += cr * er - ci * ei;
      imf += cr * ei + ci * er;
    }
  }
  if constexpr (!std::is_same<T, double>::value) {
    re = ref;
    im = imf;
  }
  red[w * 64 + lane] = make_double2(re, im);
  __syncthreads();
  if (w == 0) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < ms; ++k) {
      const double2 v = red[k * 64 + lane];
      sr += v.x;
      si += v.y;
    }
    const double wz = taper(g, ep, zm);
    const double2 val = make_double2(wz * sr, wz * si);
    out[m] = val;
    if (hist) hist[m] = val;
  }
  // screen diagnostics, once per screen (block 0): ray counts of the march,
  // folded modes, and caustic/folded modes whose weight exceeds the tolerance
  if (t == 0) {
    __shared__ unsigned long long cnt[7];
    double* sm = reinterpret_cast<double*>(red);
    __syncthreads();
    double cmax = 0.0;
    for (int j = threadIdx.x; j < g.M; j += blockDim.x) cmax = fmax(cmax, hypot(c[j].x, c[j].y));
    sm[threadIdx.x] = cmax;
    if (threadIdx.x < 7) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
      __syncthreads();
    }
    cmax = sm[0];
    unsigned long long v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int j = threadIdx.x; j < g.M; j += blockDim.x) {
      const int f = rec.mflag[j];
      v[0] += rec.mcaus[j];
      v[1] += rec.mdead[j];
      v[2] += f & 1;
      if (f && hypot(c[j].x, c[j].y) > ep.caustic_tol * cmax) ++v[3];
      v[4] += (unsigned)rec.mwork[3 * j];
      v[5] += (unsigned)rec.mwork[3 * j + 1];
      v[6] += (unsigned)rec.mwork[3 * j + 2];
    }
    for (int k = 0; k < 7; ++k)
      if (v[k]) atomicAdd(&cnt[k], v[k]);
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int k = 0; k < 4; ++k) atomicAdd(&counters[k], cnt[k]);
      atomicAdd(&counters[4], 1ull);
      for (int k = 4; k < 7; ++k) atomicAdd(&counters[k + 1], cnt[k]);
    }
  }
}

}  // namespace

// Wavefronts per workgroup (a power of two): enough workgroups x
// wavefronts to fill 256 CUs several times over.
int superpose_waves(const Geometry& g) {
  int ms = 2048 / g.T;
  if (ms < 1) ms = 1;
  if (ms > 16) ms = 16;
  while (ms > g.M) ms >>= 1;
  return ms;
}

hipError_t launch_superpose(const swkb_plan_s& pl, double2* out, double2* hist, hipStream_t st) {
  const Geometry& g = pl.g;
  Epi ep;
  ep.absorber_bot = pl.p.absorber_bot;
  ep.absorber_top = pl.p.absorber_top;
  ep.caustic_tol = pl.p.caustic_tol;
  ep.mprime_off = g.bc == SWKB_BC_PERIODIC ? 0 : g.N;
  const int ms = superpose_waves(g);
  DevModes md{pl.xi, pl.pbar, pl.e1r, pl.frac};
  const size_t shmem = sizeof(double2) * 64 * (ms < 16 ? 16 : ms);
  if (pl.precision == SWKB_FP64)
    hipLaunchKernelGGL(superpose_kernel<double>, dim3(g.T), dim3(64 * ms), shmem, st, g, md, pl.rec, pl.c, out,
                       hist, pl.counters, ep, ms);
  else
    hipLaunchKernelGGL(superpose_kernel<float>, dim3(g.T), dim3(64 * ms), shmem, st, g, md, pl.rec, pl.c, out,
                       hist, pl.counters, ep, ms);
  return hipGetLastError();
}

}  // namespace swkb
