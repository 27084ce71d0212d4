// Steps 3 and 4 of a screen, fused: interpolation of each mode's ray
// arrivals onto the grid of screen x_{q+1} (Sec. 2.1.2) and the sum over
// modes (eq. ray_bundle_q_plus_1), followed by the exit epilogue (cos^2
// taper at open ends) and the writes of the new screen field.
//
// Per (mode, point): the bracket is the largest ray r whose key (running
// maximum of live arrival heights) is <= z_m; it contributes when rays r and
// r+1 are both live.  dpsi: cubic Hermite with end slopes q - xi (dpsi_z at
// fixed x); amplitude: 4-point Lagrange over r-1..r+2 when all four are
// live, else linear.  The phase in turns is
//   (n m' mod P)/P + frac(pbar dx / lambda) + dpsi / lambda,
// the first term exact in integers.  No [mode][point] intermediate is
// written to memory (except the mode-function matrix of an x-invariant
// medium, built once per plan).
#include <type_traits>

#include <hip/hip_cooperative_groups.h>

#include "fft_body.h"
#include "swkb_internal.h"

// wavefront reductions of the device library (cross-lane DPP steps)
extern "C" __device__ unsigned long long __ockl_wfred_add_u64(unsigned long long);
extern "C" __device__ double __ockl_wfred_max_f64(double);

namespace swkb {
namespace {

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
__device__ inline T wave_shfl(T v, int src) { return __shfl(v, src, 64); }

constexpr int kWaves = 4;  // wavefronts per workgroup
// Bytes of a wavefront's one-field accumulator row: 9 per point (a padding
// point every 8), at most 7 tiles of 64 points, rounded up to a power of two.
constexpr unsigned kPolarTiles = 7;
constexpr unsigned kPolarStride = 4096;
static_assert(9 * 64 * kPolarTiles <= kPolarStride, "one-field accumulator row");
constexpr int kSub = 4;    // 64-point tiles per super-tile of the matrix product

template <typename T>
__device__ inline T rcp_t(T x);
template <>
__device__ inline double rcp_t<double>(double x) { return 1.0 / x; }
template <>
__device__ inline float rcp_t<float>(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename T>
__device__ inline T fma_t(T a, T b, T c) { return fma(a, b, c); }
template <>
__device__ inline float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }

template <typename T>
struct CplxOf;
template <>
struct CplxOf<double> { using type = double2; };
template <>
struct CplxOf<float> { using type = float2; };

// Interval (r, r+1) of one pass in power form around Z_r: zr = Z_r minus
// the super-tile's first grid height, dpsi(tau) = c0 + c1 tau + c2 tau^2 +
// c3 tau^3 (cubic Hermite, slopes q - xi), a(tau) = q0 + ... + q3 tau^3
// (Lagrange over r-1..r+2, or linear); the interval owns the super-tile's
// points [mlo, mhi) (empty unless rays r and r+1 are live).
template <typename T>
struct IvRec {
  T zr, c0, c1, c2, c3, q0, q1, q2, q3;
  int mlo, mhi;
};

// Lane l of a pass holds ray rl = a0 - 1 + l (values dl, al, pl, gl, first
// point cl); the neighbours come through shuffles, so lanes 1..61 can own
// intervals [a0, a1].  Every lane evaluates the same straight-line
// formulas and a lane without a live interval gets an empty point range; a
// value of a ray outside [0, R) enters only terms that are then not selected
// (the ownership and cubic tests check the indices), so such lanes may hold
// any ray's data.
template <typename T>
__device__ inline IvRec<T> build_interval(const Geometry& g, int rl, int a0, int a1, int m0, int npts, double zs0,
                                          T dl, T al, T pl, T gl, int cl) {
  const int lane = threadIdx.x & 63;
  const T dm1 = wave_shfl(dl, lane - 1), dp1 = wave_shfl(dl, lane + 1), dp2 = wave_shfl(dl, lane + 2);
  const T am1 = wave_shfl(al, lane - 1), ap1 = wave_shfl(al, lane + 1), ap2 = wave_shfl(al, lane + 2);
  const T pp1 = wave_shfl(pl, lane + 1), gp1 = wave_shfl(gl, lane + 1);
  const int cp1 = __shfl(cl, lane + 1, 64);
  IvRec<T> r;
  T H, xm, x3;
  if constexpr (std::is_same<T, double>::value) {
    const double Zl = (g.z_a + (double)(rl * g.rho - g.E) * g.h) + dl;
    const double Zn = (g.z_a + (double)((rl + 1) * g.rho - g.E) * g.h) + dp1;
    r.zr = Zl - zs0;
    H = Zn - Zl;
    xm = ((g.z_a + (double)((rl - 1) * g.rho - g.E) * g.h) + dm1) - Zl;
    x3 = ((g.z_a + (double)((rl + 2) * g.rho - g.E) * g.h) + dp2) - Zl;
  } else {
    const float hf = (float)g.h;
    const float rh = (float)g.rho * hf;
    r.zr = (float)(rl * g.rho - g.E - m0) * hf + dl;
    H = rh + (dp1 - dl);
    xm = -rh + (dm1 - dl);
    x3 = T(2) * rh + (dp2 - dl);
  }
  const bool own = rl >= a0 && rl <= a1 && al > T(0) && ap1 > T(0) && H > T(0);
  const T iH = rcp_t<T>(H);
  const T dlt = (pp1 - pl) * iH;
  r.c0 = pl;
  r.c1 = gl;
  r.c2 = (T(3) * dlt - T(2) * gl - gp1) * iH;
  r.c3 = (gl + gp1 - T(2) * dlt) * iH * iH;
  const bool cubic = rl >= 1 && rl + 2 < g.R && am1 > T(0) && ap2 > T(0);
  const T f01 = (ap1 - al) * iH;
  // Newton form on nodes 0, H, xm (ray r-1), x3 (ray r+2), then powers of tau
  const T f12 = (am1 - ap1) * rcp_t<T>(xm - H);
  const T f23 = (ap2 - am1) * rcp_t<T>(x3 - xm);
  const T f012 = (f12 - f01) * rcp_t<T>(xm);
  const T f123 = (f23 - f12) * rcp_t<T>(x3 - H);
  const T f0123 = (f123 - f012) * rcp_t<T>(x3);
  r.q0 = al;
  r.q1 = cubic ? f01 - H * f012 + H * xm * f0123 : f01;
  r.q2 = cubic ? f012 - (H + xm) * f0123 : T(0);
  r.q3 = cubic ? f0123 : T(0);
  r.mlo = own ? (cl - m0 > 0 ? cl - m0 : 0) : 0;
  r.mhi = own ? (cp1 - m0 < npts ? cp1 - m0 : npts) : 0;
  return r;
}

// Phase factor e^{2 pi i turns} at grid index m' (nm = n m' mod P) of mode
// n with range phase fj and phase deviation dps.
template <typename T>
__device__ inline void phase_of(int nm, const Geometry& g, T fj, double fjd, T dps, double inv_lam, T& sn, T& cs) {
  if constexpr (std::is_same<T, double>::value) {
    double turns = (double)nm / (double)g.P + fjd + dps * inv_lam;
    turns -= floor(turns);
    sincospi(2.0 * turns, &sn, &cs);
  } else {
    // fractional part in one instruction (x - floor(x), kept below 1)
    const float turns = __builtin_amdgcn_fractf((float)nm * (1.0f / (float)g.P) + fj + dps * (float)inv_lam);
    sn = __builtin_amdgcn_sinf(turns);  // argument in revolutions
    cs = __builtin_amdgcn_cosf(turns);
  }
}

// Sum over modes for one screen, organised by interval owner.  For a mode,
// grid point m belongs to the interval of the largest ray r with
// key_r <= z_m, i.e. to the points [ci_r, ci_{r+1}) where ci_r is the first
// grid index at or above key_r (computed by the scan).  So every point has
// exactly one interval per mode and the intervals of one mode cover
// disjoint point ranges: the lane that owns interval (r, r+1) builds its
// record in registers and adds its contribution to each of its points in
// the wavefront's LDS accumulator, with no search and no write conflict.
//
// Grid (super-tiles, mode groups, field chunks); block = kWaves wavefronts.
// Wavefront w of group gi takes modes j = gi * kWaves + w + k * (groups *
// kWaves).  Per mode it walks the super-tile's intervals [tstart of its
// first tile, tstart of the next super-tile], 61 per pass (the lane holds
// ray a0 - 1 + lane; interval lanes 1..61 read rays r - 1 .. r + 2 through
// shuffles).  At the end the kWaves accumulators are summed in a fixed order
// into part[b][gi][m]; the contributions to one accumulator entry arrive in
// program order, so the result does not depend on scheduling.
//
// LDS accumulator row of a wavefront: point m at m + m / 8 (intervals are
// about rho points long, so the lanes of one step fall into different banks).
// TABLE = true: write the mode functions T[j][m] = a e^{2 pi i turns} of an
// x-invariant medium instead (entries without an owning interval must be
// zero beforehand); c, part and the accumulators are not used.
//
// One FP32 field (POLAR): the mode's coefficient comes in polar form, its
// argument joins the phase constant and its modulus the amplitude
// polynomial, so a point adds |c| a (cos, sin) with two FMAs.
template <typename T, int NB, bool TABLE>
__global__ void __launch_bounds__(64 * kWaves) superpose_iv_kernel(Geometry g, DevModes modes, DevRecords rec,
                                                                   const double2* __restrict__ c,
                                                                   const float2* __restrict__ cpol,
                                                                   double2* __restrict__ part,
                                                                   typename CplxOf<T>::type* __restrict__ tab, Epi ep,
                                                                   int sub, int batch) {
  constexpr bool POLAR = std::is_same<T, float>::value && NB == 1 && !TABLE;
  extern __shared__ double2 lds_raw[];
  // one-field accumulators: kWaves rows of kPolarStride bytes at a fixed
  // LDS offset (so that a row address is one and-or of the point counter)
  __shared__ __align__(16) char polar_acc[POLAR ? kWaves * kPolarStride : 16];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int gi = blockIdx.y;
  const int jstep = (int)gridDim.y * kWaves;
  const int b0 = (int)blockIdx.z * NB;
  const int nb = batch - b0 < NB ? batch - b0 : NB;
  const int t0 = (int)blockIdx.x * sub;                 // first 64-point tile of the super-tile
  const int t1 = t0 + sub < g.T ? t0 + sub : g.T;       // (the last super-tile may be shorter)
  const int npts = (t1 - t0) * 64;
  const int m0 = t0 * 64;                                // its first grid point
  const int row = sub * 64 + sub * 8;
  using C2 = typename CplxOf<T>::type;
  // POLAR: wavefront w's row starts at byte w * kPolarStride of polar_acc
  const unsigned wstride = POLAR ? kPolarStride : 0u;
  C2* acc = POLAR ? reinterpret_cast<C2*>(polar_acc + (size_t)w * wstride)
                  : reinterpret_cast<C2*>(lds_raw) + (size_t)w * NB * row;  // [NB][row] (re, im)
  if constexpr (!TABLE)
    for (int i = lane; i < NB * row; i += 64) {
      acc[i].x = T(0);
      acc[i].y = T(0);
    }
  const double inv_lam = 1.0 / g.lam;
  const T* __restrict__ D = static_cast<const T*>(rec.D);
  const T* __restrict__ Pp = static_cast<const T*>(rec.Pp);
  const T* __restrict__ G = static_cast<const T*>(rec.G);
  const T* __restrict__ A = static_cast<const T*>(rec.A);
  const int pmask = g.P - 1;  // P is a power of two
  const int mp0 = m0 + ep.mprime_off;
  const double zs0 = g.z_a + (double)m0 * g.h;
  for (int j = gi * kWaves + w; j < g.M; j += jstep) {
    if (rec.mflag[j] & 1) continue;  // folded mode
    const int* ts = rec.tstart + (size_t)j * (g.T + 1);
    const int lo = ts[t0], hi = ts[t1];
    // intervals (r, r + 1) for r in [ia, ib]
    const int ia = lo > 0 ? lo : 0;
    const int ib = hi < g.R - 2 ? hi : g.R - 2;
    if (ia > ib) continue;
    const size_t base = (size_t)j * g.R;
    const int n = j - (g.M >> 1);
    const int nm0 = (n * mp0) & pmask;
    T cjr[NB], cji[NB];
    float cmod = 0.0f, carg = 0.0f;  // POLAR: |c|, arg c in turns plus the range phase
    const T fj = (T)modes.frac[j];
    const double fjd = modes.frac[j];
    if constexpr (POLAR) {
      const float2 pc = cpol[j];
      cmod = pc.x;
      carg = pc.y + fj;
    } else {
      for (int bb = 0; bb < NB; ++bb) {
        const double2 v = bb < nb ? c[(size_t)(b0 + bb) * g.M + j] : make_double2(0.0, 0.0);
        cjr[bb] = (T)v.x;
        cji[bb] = (T)v.y;
      }
    }
    for (int a0 = ia; a0 <= ib; a0 += 61) {
      const int a1 = a0 + 60 < ib ? a0 + 60 : ib;  // intervals [a0, a1] in this pass
      const int rl = a0 - 1 + lane;                 // ray held by this lane
      const int rc = rl < 0 ? 0 : (rl < g.R ? rl : g.R - 1);
      const T dl = D[base + rc], al = A[base + rc], pl = Pp[base + rc], gl = G[base + rc];
      const int cl = rec.cidx[base + rc];
      const IvRec<T> iv = build_interval<T>(g, rl, a0, a1, m0, npts, zs0, dl, al, pl, gl, cl);
      T zr = iv.zr, c0 = iv.c0, c1 = iv.c1, c2 = iv.c2, c3 = iv.c3, q0 = iv.q0, q1 = iv.q1, q2 = iv.q2, q3 = iv.q3;
      if constexpr (POLAR) {
        q0 *= cmod;
        q1 *= cmod;
        q2 *= cmod;
        q3 *= cmod;
      }
      const int mlo = iv.mlo, mhi = iv.mhi;  // owned points [m0 + mlo, m0 + mhi)
      constexpr bool kF64 = std::is_same<T, double>::value;
      int nm = (nm0 + n * mlo) & pmask;
      // offset of point m above the interval's first ray; FP32 steps by h
      T tau;
      if constexpr (kF64) tau = 0.0;
      else tau = (float)mlo * (float)g.h - zr;
      const T hstep = kF64 ? T(0) : (T)g.h;
      // FP32: the phase in turns from the deviation's coefficients scaled to
      // turns once per interval (range phase folded into the constant), and the
      // grid phase (n m' mod P) / P carried as a float: multiples of 1/P below
      // one and their sums are exact in FP32, so fract(gt + n/P) equals it at
      // the next point
      float gt = 0.0f, gstep = 0.0f, e0 = 0.0f, e1 = 0.0f, e2 = 0.0f, e3 = 0.0f;
      if constexpr (!kF64) {
        const float il = (float)inv_lam, invP = 1.0f / (float)g.P;
        gt = (float)nm * invP;
        gstep = (float)(n & pmask) * invP;
        e0 = c0 * il + (POLAR ? carg : fj);
        e1 = c1 * il;
        e2 = c2 * il;
        e3 = c3 * il;
      }
      if constexpr (POLAR) {
        // point m of the row sits at byte 8 (m + m / 8) = (9 m) & ~7 (the
        // padding every 8 points keeps a step's lanes, about rho points
        // apart, in different banks): the loop counts 9 m, and the wave's
        // row offset is OR-ed in
        char* const lds_b = reinterpret_cast<char*>(polar_acc);
        const unsigned wb = (unsigned)w * wstride;
        const unsigned m9e = 9u * (unsigned)mhi;
        for (unsigned m9 = 9u * (unsigned)mlo; m9 < m9e; m9 += 9u, tau += hstep) {
          const float turns = __builtin_amdgcn_fractf(gt + (((e3 * tau + e2) * tau + e1) * tau + e0));
          const float sn = __builtin_amdgcn_sinf(turns);  // argument in revolutions
          const float cs = __builtin_amdgcn_cosf(turns);
          gt = __builtin_amdgcn_fractf(gt + gstep);
          const T a = ((q3 * tau + q2) * tau + q1) * tau + q0;
          C2* const pa = reinterpret_cast<C2*>(lds_b + ((m9 & ~7u) | wb));
          C2 v = *pa;
          v.x = fma_t(a, cs, v.x);
          v.y = fma_t(a, sn, v.y);
          *pa = v;
        }
        continue;
      }
      for (int m = mlo; m < mhi; ++m, tau += hstep) {
        T sn, cs;
        if constexpr (kF64) {
          tau = (double)m * g.h - zr;
          const T dps = ((c3 * tau + c2) * tau + c1) * tau + c0;
          phase_of<T>(nm, g, fj, fjd, dps, inv_lam, sn, cs);
          nm = (nm + n) & pmask;
        } else {
          const float turns = __builtin_amdgcn_fractf(gt + (((e3 * tau + e2) * tau + e1) * tau + e0));
          sn = __builtin_amdgcn_sinf(turns);  // argument in revolutions
          cs = __builtin_amdgcn_cosf(turns);
          gt = __builtin_amdgcn_fractf(gt + gstep);
        }
        const T a = ((q3 * tau + q2) * tau + q1) * tau + q0;
        const T ea = a * cs, eb = a * sn;  // a e^{i phase}
        if constexpr (TABLE) {
          typename CplxOf<T>::type v;
          v.x = ea;
          v.y = eb;
          tab[(size_t)j * g.N + m0 + m] = v;
          continue;
        }
        const int pm = m + (m >> 3);
        for (int bb = 0; bb < NB; ++bb) {
          // lanes of one step own different points; LDS keeps the wavefront's accesses in order
          C2 v = acc[bb * row + pm];
          v.x = fma_t(cjr[bb], ea, fma_t(-cji[bb], eb, v.x));
          v.y = fma_t(cjr[bb], eb, fma_t(cji[bb], ea, v.y));
          acc[bb * row + pm] = v;
        }
      }
    }
  }
  if constexpr (TABLE) return;
  __syncthreads();
  const C2* acc0 = POLAR ? reinterpret_cast<const C2*>(polar_acc) : reinterpret_cast<const C2*>(lds_raw);
  for (int bb = 0; bb < nb; ++bb) {
    for (int m = threadIdx.x; m < npts; m += blockDim.x) {
      const int pm = m + (m >> 3);
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < kWaves; ++k) {
        const C2 v = POLAR ? acc0[(size_t)k * (wstride / sizeof(C2)) + pm] : acc0[((size_t)k * NB + bb) * row + pm];
        sr += (double)v.x;
        si += (double)v.y;
      }
      part[((size_t)(b0 + bb) * gridDim.y + gi) * g.N + m0 + m] = make_double2(sr, si);
    }
  }
}

// Native vector types for non-temporal loads.
typedef float F4 __attribute__((ext_vector_type(4)));
typedef double D2 __attribute__((ext_vector_type(2)));

// Sum over modes for one screen with the points' owners mapped in LDS.
// Same grid, mode split and passes as the interval-walk kernel, but after
// building its records a pass (1) stores them in the wavefront's LDS, (2)
// marks for each point of the super-tile the lane whose interval owns it
// (the owner lane writes its own point range: disjoint, no conflict), and
// (3) lets lane l evaluate points l, l + 64, ... of the super-tile from the
// owner's record.  Every lane then does the same number of evaluations per
// pass, and each lane accumulates its points in registers across modes; the
// wavefronts' sums meet in LDS at the end and are added in a fixed order.
//
// FP32 (batches of fields) asks for 5 wavefronts per SIMD (96 VGPRs, no
// spills; at the compiler's own choice 101 VGPRs and 4): 4-field batch on the
// random medium 71.3 -> 68.4 ms per 400 screens.  FP64 keeps the compiler's
// choice (fewer registers spill there).
template <typename T, int NB, int SUBMAX>
__global__ void __launch_bounds__(64 * kWaves, (std::is_same<T, float>::value ? 5 : 1)) superpose_own_kernel(Geometry g, DevModes modes, DevRecords rec,
                                                                    const double2* __restrict__ c,
                                                                    double2* __restrict__ part, Epi ep, int sub,
                                                                    int batch) {
  struct alignas(16) LRec {
    T zr, c0, c1, c2, c3, q0, q1, q2, q3;
  };
  extern __shared__ double2 lds_raw[];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int gi = blockIdx.y;
  const int jstep = (int)gridDim.y * kWaves;
  const int b0 = (int)blockIdx.z * NB;
  const int nb = batch - b0 < NB ? batch - b0 : NB;
  const int t0 = (int)blockIdx.x * sub;
  const int t1 = t0 + sub < g.T ? t0 + sub : g.T;
  const int npts = (t1 - t0) * 64;
  const int nsub = t1 - t0;
  const int m0 = t0 * 64;
  char* wb = reinterpret_cast<char*>(lds_raw) + (size_t)w * (64 * sizeof(LRec) + SUBMAX * 64 * sizeof(int));
  LRec* recs = reinterpret_cast<LRec*>(wb);
  int* own = reinterpret_cast<int*>(wb + 64 * sizeof(LRec));
  T ar[NB][SUBMAX], ai[NB][SUBMAX];
  for (int bb = 0; bb < NB; ++bb)
    for (int u = 0; u < SUBMAX; ++u) ar[bb][u] = ai[bb][u] = T(0);
  const double inv_lam = 1.0 / g.lam;
  const T* __restrict__ D = static_cast<const T*>(rec.D);
  const T* __restrict__ Pp = static_cast<const T*>(rec.Pp);
  const T* __restrict__ G = static_cast<const T*>(rec.G);
  const T* __restrict__ A = static_cast<const T*>(rec.A);
  const int pmask = g.P - 1;
  const int mp0 = m0 + ep.mprime_off;
  const double zs0 = g.z_a + (double)m0 * g.h;
  for (int j = gi * kWaves + w; j < g.M; j += jstep) {
    if (rec.mflag[j] & 1) continue;  // folded mode
    const int* ts = rec.tstart + (size_t)j * (g.T + 1);
    const int lo = ts[t0], hi = ts[t1];
    const int ia = lo > 0 ? lo : 0;
    const int ib = hi < g.R - 2 ? hi : g.R - 2;
    if (ia > ib) continue;
    const size_t base = (size_t)j * g.R;
    const int n = j - (g.M >> 1);
    const int nml = (n * mp0 + n * lane) & pmask;  // grid phase index of point `lane`
    T cjr[NB], cji[NB];
    for (int bb = 0; bb < NB; ++bb) {
      const double2 v = bb < nb ? c[(size_t)(b0 + bb) * g.M + j] : make_double2(0.0, 0.0);
      cjr[bb] = (T)v.x;
      cji[bb] = (T)v.y;
    }
    const T fj = (T)modes.frac[j];
    const double fjd = modes.frac[j];
    for (int a0 = ia; a0 <= ib; a0 += 61) {
      const int a1 = a0 + 60 < ib ? a0 + 60 : ib;
      const int rl = a0 - 1 + lane;
      const bool in = rl >= 0 && rl < g.R;
      const T dl = in ? D[base + rl] : T(0);
      const T al = in ? A[base + rl] : T(-1);
      const T pl = in ? Pp[base + rl] : T(0);
      const T gl = in ? G[base + rl] : T(0);
      const int cl = in ? rec.cidx[base + rl] : 0;
      const IvRec<T> iv = build_interval<T>(g, rl, a0, a1, m0, npts, zs0, dl, al, pl, gl, cl);
      for (int u = 0; u < SUBMAX; ++u)
        if (u < nsub) own[u * 64 + lane] = -1;
      recs[lane] = LRec{iv.zr, iv.c0, iv.c1, iv.c2, iv.c3, iv.q0, iv.q1, iv.q2, iv.q3};
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int m = iv.mlo; m < iv.mhi; ++m) own[m] = lane;
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < SUBMAX; ++u) {
        if (u >= nsub) break;  // uniform
        const int pt = u * 64 + lane;
        const int o = own[pt];
        if (o < 0) continue;
        const LRec R = recs[o];
        T tau;
        if constexpr (std::is_same<T, double>::value) tau = (double)pt * g.h - R.zr;
        else tau = (float)pt * (float)g.h - R.zr;
        const T dps = ((R.c3 * tau + R.c2) * tau + R.c1) * tau + R.c0;
        const T a = ((R.q3 * tau + R.q2) * tau + R.q1) * tau + R.q0;
        T sn, cs;
        phase_of<T>((nml + n * 64 * u) & pmask, g, fj, fjd, dps, inv_lam, sn, cs);
        const T ea = a * cs, eb = a * sn;  // a e^{i phase}
        for (int bb = 0; bb < NB; ++bb) {
          ar[bb][u] = fma_t(cjr[bb], ea, fma_t(-cji[bb], eb, ar[bb][u]));
          ai[bb][u] = fma_t(cjr[bb], eb, fma_t(cji[bb], ea, ai[bb][u]));
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();  // the next pass rewrites own and recs
    }
  }
  // the wavefronts' sums, added in the order 0, 1, 2, 3
  __syncthreads();
  using C2 = typename CplxOf<T>::type;
  C2* red = reinterpret_cast<C2*>(lds_raw);  // [kWaves][NB][SUBMAX * 64]
  for (int bb = 0; bb < NB; ++bb)
    for (int u = 0; u < SUBMAX; ++u)
      if (u < nsub) {
        C2 v;
        v.x = ar[bb][u];
        v.y = ai[bb][u];
        red[((size_t)w * NB + bb) * (SUBMAX * 64) + u * 64 + lane] = v;
      }
  __syncthreads();
  for (int bb = 0; bb < nb; ++bb) {
    for (int m = threadIdx.x; m < npts; m += blockDim.x) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < kWaves; ++k) {
        const C2 v = red[((size_t)k * NB + bb) * (SUBMAX * 64) + m];
        sr += (double)v.x;
        si += (double)v.y;
      }
      part[((size_t)(b0 + bb) * gridDim.y + gi) * g.N + m0 + m] = make_double2(sr, si);
    }
  }
}

// One screen from the mode-function matrix: part[gi][m] = sum over the
// group's modes of c_j T[j][m], in the same grid/partial layout as the
// superposition (a streaming read of T, coalesced along m).
template <typename T>
__device__ inline void apply_matrix_body(const Geometry& g, const typename CplxOf<T>::type* __restrict__ tab,
                                         const double2* __restrict__ c, double2* __restrict__ part, int sb, int gi,
                                         int groups, int sub, double2* red) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int jstep = groups * kWaves;
  const int m0 = sb * sub * 64;
  T acc_re[kSub], acc_im[kSub];
  for (int u = 0; u < kSub; ++u) acc_re[u] = acc_im[u] = T(0);
#pragma unroll 2
  for (int j = gi * kWaves + w; j < g.M; j += jstep) {
    const double2 cj = c[j];
    const T cr = (T)cj.x, ci = (T)cj.y;
    const typename CplxOf<T>::type* col = tab + (size_t)j * g.N + m0 + lane;
    for (int u = 0; u < kSub; ++u) {
      if (u < sub) {
        typename CplxOf<T>::type v;
        if constexpr (std::is_same<T, double>::value) {
          const D2 d = __builtin_nontemporal_load(reinterpret_cast<const D2*>(col + u * 64));
          v.x = d.x;
          v.y = d.y;
        } else {
          v = col[u * 64];
        }
        acc_re[u] += cr * v.x - ci * v.y;
        acc_im[u] += cr * v.y + ci * v.x;
      }
    }
  }
  for (int u = 0; u < kSub; ++u) red[(w * kSub + u) * 64 + lane] = make_double2((double)acc_re[u], (double)acc_im[u]);
  __syncthreads();
  if (w == 0) {
    for (int u = 0; u < sub; ++u) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k < kWaves; ++k) {
        const double2 v = red[(k * kSub + u) * 64 + lane];
        sr += v.x;
        si += v.y;
      }
      part[(size_t)gi * g.N + m0 + u * 64 + lane] = make_double2(sr, si);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(64 * kWaves) apply_matrix_kernel(Geometry g,
                                                                   const typename CplxOf<T>::type* __restrict__ tab,
                                                                   const double2* __restrict__ c,
                                                                   double2* __restrict__ part, int sub) {
  extern __shared__ double2 red[];
  apply_matrix_body<T>(g, tab, c, part, blockIdx.x, blockIdx.y, gridDim.y, sub, red);
}

// The same product for complex64 T with 16-byte loads: lane l of a
// wavefront reads points m0 + 128 u + 2 l and + 1 (two complex64 in one
// float4), u < 4, so a workgroup covers 512 points and each load moves 1 KB
// per wavefront.  In the per-stage kernels the mode loop is not unrolled
// (U = 1): at 57 VGPRs eight wavefronts per SIMD keep enough loads in flight
// (unrolled by 4: 102 VGPRs, four wavefronts, the 64-problem batch 1.486 ->
// 1.469 s without).  The persistent kernel, whose other stages hold more
// registers anyway, requests U modes' loads at once.  The terms are added in
// the same order either way.  N % 512 == 0.
template <int U>
__device__ inline void apply_c64_body(const Geometry& g, const float4* __restrict__ tab,
                                      const double2* __restrict__ c, double2* __restrict__ part, int bx, int gi,
                                      int groups, float2* red) {  // red: [kWaves][4][64][2] pairs of (re, im)
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int jstep = groups * kWaves;
  const int m0 = bx * 512;
  float ar[4][2], ai[4][2];
  for (int u = 0; u < 4; ++u) ar[u][0] = ar[u][1] = ai[u][0] = ai[u][1] = 0.0f;
  const size_t row4 = (size_t)g.N / 2;  // float4 per row of T
  int j = gi * kWaves + w;
  if constexpr (U > 1) {
#pragma unroll 1
    for (; j + (U - 1) * jstep < g.M; j += U * jstep) {
      F4 v[U][4];
      float cr[U], ci[U];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const double2 cj = c[j + t * jstep];
        cr[t] = (float)cj.x;
        ci[t] = (float)cj.y;
        const float4* col = tab + (size_t)(j + t * jstep) * row4 + m0 / 2 + lane;
#pragma unroll
        for (int u = 0; u < 4; ++u) v[t][u] = __builtin_nontemporal_load(reinterpret_cast<const F4*>(col + u * 64));
      }
#pragma unroll
      for (int t = 0; t < U; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ar[u][0] += cr[t] * v[t][u].x - ci[t] * v[t][u].y;
          ai[u][0] += cr[t] * v[t][u].y + ci[t] * v[t][u].x;
          ar[u][1] += cr[t] * v[t][u].z - ci[t] * v[t][u].w;
          ai[u][1] += cr[t] * v[t][u].w + ci[t] * v[t][u].z;
        }
    }
  }
#pragma unroll 1
  for (; j < g.M; j += jstep) {
    const double2 cj = c[j];
    const float cr = (float)cj.x, ci = (float)cj.y;
    const float4* col = tab + (size_t)j * row4 + m0 / 2 + lane;
    for (int u = 0; u < 4; ++u) {
      // T is streamed once per screen: non-temporal loads keep it out of the caches
      const F4 v = __builtin_nontemporal_load(reinterpret_cast<const F4*>(col + u * 64));
      ar[u][0] += cr * v.x - ci * v.y;
      ai[u][0] += cr * v.y + ci * v.x;
      ar[u][1] += cr * v.z - ci * v.w;
      ai[u][1] += cr * v.w + ci * v.z;
    }
  }
  for (int u = 0; u < 4; ++u)
    for (int h = 0; h < 2; ++h)
      red[((w * 4 + u) * 64 + lane) * 2 + h] = make_float2(ar[u][h], ai[u][h]);
  __syncthreads();
  // points m0 + 128 u + 2 l + h, summed over the wavefronts in order (in FP64)
  for (int idx = threadIdx.x; idx < 512; idx += blockDim.x) {
    const int u = idx >> 7, l = (idx >> 1) & 63, h = idx & 1;
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < kWaves; ++k) {
      const float2 v = red[((k * 4 + u) * 64 + l) * 2 + h];
      sr += (double)v.x;
      si += (double)v.y;
    }
    part[(size_t)gi * g.N + m0 + idx] = make_double2(sr, si);
  }
}

__global__ void __launch_bounds__(64 * kWaves) apply_matrix_c64_kernel(Geometry g, const float4* __restrict__ tab,
                                                                       const double2* __restrict__ c,
                                                                       double2* __restrict__ part) {
  extern __shared__ double2 red[];
  apply_c64_body<1>(g, tab, c, part, blockIdx.x, blockIdx.y, gridDim.y, reinterpret_cast<float2*>(red));
}

// Sum of the mode-group partials in a fixed order (four threads per point,
// each over every fourth group, then combined in order), exit taper, field
// and history writes, for field blockIdx.y of the batch (part is
// [batch][groups][N] of PT = double2 or float2).  The last block of field 0
// accumulates the screen's diagnostics; a mode is significant when its
// energy summed over the batch exceeds caustic_tol^2 times the largest.
constexpr int kFinThreads = 512;  // 128 points per workgroup, 4 threads per point
constexpr int kFinWaves = kFinThreads / 64;
constexpr int kDiagSlots = 8;  // modes per thread and chunk in the diagnostics
// Threads per workgroup of the persistent multi-problem kernel: the FFT and
// product bodies' own workgroup size (the epilogue body takes any).
constexpr int kPersistThreads = 64 * kWaves;
constexpr int kPersistUnroll = 4;  // modes of the product whose loads a wavefront issues together

// Diagnostics of a screen, by one workgroup: the largest mode energy
// (summed over the batch), then the counts, with wavefront reductions and
// the wavefronts combined in order.  A thread takes modes j0 + k *
// blockDim.x, k < kDiagSlots, of each chunk of kDiagSlots * blockDim.x
// modes, with the loads of all of them issued together (kOne, one field:
// the energy is one load; several fields: energy, the modes' energies
// summed over the batch by the panel kernels of the batched product, when
// given, else the sums here); when one chunk covers the M modes (M <= 4096 at
// 512 threads), their energies and flags stay in registers for the count of
// significant modes, so the workgroup waits for memory about once instead of
// once per loop round.
template <bool kOne>
__device__ inline void diag_body(const Geometry& g, const DevRecords& rec, const double2* __restrict__ c, int batch,
                                 unsigned long long* __restrict__ counters, const Epi& ep,
                                 const double* __restrict__ energy) {
  __shared__ double sm[kFinWaves];
  __shared__ unsigned long long cnt[kFinWaves][10];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nt = (int)blockDim.x, nw = nt >> 6;
  // a thread's sums fit 32 bits, 64-bit from the wavefront on; counts 3 and
  // 9 (significant modes) wait for the threshold below
  unsigned v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double emax = 0.0, e[kDiagSlots];
  int fl[kDiagSlots];
  for (int j0 = 0; j0 < g.M; j0 += kDiagSlots * nt) {
#pragma unroll
    for (int k = 0; k < kDiagSlots; ++k) {
      const int j = j0 + k * nt + (int)threadIdx.x;
      int f = 0;
      double ej = 0.0;
      if (j < g.M) {
        f = rec.mflag[j];
        const int4 w = *reinterpret_cast<const int4*>(rec.mwork + 4 * (size_t)j);  // 16-byte aligned rows
        v[0] += rec.mcaus[j];
        v[1] += rec.mdead[j];
        v[2] += f & 1;
        v[8] += (f >> 2) & 1;
        v[4] += (unsigned)w.x;
        v[5] += (unsigned)w.y;
        v[6] += (unsigned)w.z;
        v[7] += (unsigned)w.w;
        if constexpr (kOne) {
          const double2 cj = c[j];
          ej = cj.x * cj.x + cj.y * cj.y;
        } else {
          ej = energy ? energy[j] : batch_energy(c, g.M, j, batch);
        }
      }
      e[k] = ej;
      fl[k] = f;
      emax = fmax(emax, ej);
    }
  }
  // Wavefront reductions (cross-lane DPP steps, no LDS round trips): the
  // largest energy and the eight counts that do not depend on the threshold
  // first, the two that do (each at most M: 32 bits) after it.  As 64-bit
  // shuffle chains one after another they took about 3 us per screen.
  constexpr int kFree[8] = {0, 1, 2, 4, 5, 6, 7, 8};
  unsigned long long w64[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) w64[i] = __ockl_wfred_add_u64(v[kFree[i]]);
  emax = __ockl_wfred_max_f64(emax);
  if (lane == 0) {
    sm[wv] = emax;
#pragma unroll
    for (int i = 0; i < 8; ++i) cnt[wv][kFree[i]] = w64[i];
  }
  __syncthreads();
  emax = 0.0;
  for (int k = 0; k < nw; ++k) emax = fmax(emax, sm[k]);
  const double thr = ep.caustic_tol * ep.caustic_tol * emax;
  unsigned sig = 0, sig_dead = 0;
  if (g.M <= kDiagSlots * nt) {
#pragma unroll
    for (int k = 0; k < kDiagSlots; ++k)
      if (fl[k] && e[k] > thr) {
        if (fl[k] & 3) ++sig;       // caustic or folded
        if (fl[k] & 4) ++sig_dead;  // no live ray
      }
  } else {
    for (int j = threadIdx.x; j < g.M; j += nt) {
      const int f = rec.mflag[j];
      if (f && (!kOne && energy ? energy[j] : batch_energy(c, g.M, j, kOne ? 1 : batch)) > thr) {
        if (f & 3) ++sig;
        if (f & 4) ++sig_dead;
      }
    }
  }
  sig = __ockl_wfred_add_u32(sig);
  sig_dead = __ockl_wfred_add_u32(sig_dead);
  if (lane == 0) {
    cnt[wv][3] = sig;
    cnt[wv][9] = sig_dead;
  }
  __syncthreads();
  // counters[0..3]: count 0..3; [4]: screens; [5..10]: count 4..9 (one
  // lane each, one atomic instruction)
  if ((int)threadIdx.x <= 10) {
    const int k = threadIdx.x;
    unsigned long long t = 0;
    if (k == 4) {
      t = 1;
    } else {
      const int src = k < 4 ? k : k - 1;
      for (int w = 0; w < nw; ++w) t += cnt[w][src];
    }
    atomicAdd(&counters[k], t);
  }
}

template <typename PT>
__device__ inline void finalize_body(const Geometry& g, const DevRecords& rec, const double2* __restrict__ c,
                                     const PT* __restrict__ part, int groups, int batch, double2* __restrict__ out,
                                     double2* __restrict__ hist, unsigned long long* __restrict__ counters,
                                     const Epi& ep, int bx, int nbx, int b,
                                     const double* __restrict__ energy = nullptr) {
  if (bx + 1 < nbx) {
    const int sub = threadIdx.x & 3;
    const PT* pb = part + (size_t)b * groups * g.N;
    // the workgroup's kFinThreads / 4 points, blockDim.x / 4 at a time
    for (int p0 = 0; p0 < kFinThreads / 4; p0 += (int)blockDim.x / 4) {
      const int m = bx * (kFinThreads / 4) + p0 + (threadIdx.x >> 2);
      double sr = 0.0, si = 0.0;
      if (m < g.N) {
#pragma unroll 4
        for (int k = sub; k < groups; k += 4) {
          const PT v = pb[(size_t)k * g.N + m];
          sr += (double)v.x;
          si += (double)v.y;
        }
      }
      // combine the four partial sums in the order 0, 1, 2, 3
      const double r1 = __shfl_down(sr, 1, 4), i1 = __shfl_down(si, 1, 4);
      const double r2 = __shfl_down(sr, 2, 4), i2 = __shfl_down(si, 2, 4);
      const double r3 = __shfl_down(sr, 3, 4), i3 = __shfl_down(si, 3, 4);
      if (sub == 0 && m < g.N) {
        const double tr = ((sr + r1) + r2) + r3, ti = ((si + i1) + i2) + i3;
        const double wz = taper(g, ep, g.z_a + (double)m * g.h);
        const double2 val = make_double2(wz * tr, wz * ti);
        out[(size_t)b * g.N + m] = val;
        if (hist) hist[(size_t)b * g.N + m] = val;
      }
    }
    return;
  }
  if (b != 0) return;
  // the last workgroup of field 0: the screen's diagnostics
  if (batch == 1)
    diag_body<true>(g, rec, c, 1, counters, ep, nullptr);
  else
    diag_body<false>(g, rec, c, batch, counters, ep, energy);
}

template <typename PT>
__global__ void __launch_bounds__(kFinThreads) finalize_kernel(Geometry g, DevRecords rec,
                                                               const double2* __restrict__ c,
                                                               const PT* __restrict__ part, int groups, int batch,
                                                               double2* __restrict__ out, double2* __restrict__ hist,
                                                               unsigned long long* __restrict__ counters, Epi ep,
                                                               const double* __restrict__ energy) {
  finalize_body<PT>(g, rec, c, part, groups, batch, out, hist, counters, ep, blockIdx.x, gridDim.x, blockIdx.y,
                    energy);
}

// The matrix product and the epilogue of one screen for many problems, one
// launch each: workgroup b runs local workgroup map[b] & 0xfffff of problem
// map[b] >> 20 (product: local = gi * (N / 512) + point block).
__global__ void __launch_bounds__(64 * kWaves) apply_c64_multi(const MultiProblem* __restrict__ mp,
                                                               const unsigned* __restrict__ map) {
  extern __shared__ double2 red[];
  const unsigned e = map[blockIdx.x];
  const MultiProblem& p = mp[e >> 20];
  const int local = (int)(e & 0xfffff);
  if (p.fp64) {
    const int nsb = p.g.T / p.sub;
    apply_matrix_body<double>(p.g, p.tmat64, p.c, p.part, local % nsb, local / nsb, p.groups, p.sub, red);
  } else {
    const int nx = p.g.N >> 9;
    apply_c64_body<1>(p.g, p.tmat, p.c, p.part, local % nx, local / nx, p.groups, reinterpret_cast<float2*>(red));
  }
}

__global__ void __launch_bounds__(kFinThreads) finalize_multi(const MultiProblem* __restrict__ mp,
                                                              const unsigned* __restrict__ map, int step) {
  const unsigned e = map[blockIdx.x];
  const MultiProblem& p = mp[e >> 20];
  double2* hist = p.hist ? p.hist + (size_t)step * p.g.N : nullptr;
  finalize_body<double2>(p.g, p.rec, p.c, p.part, p.groups, 1, p.u, hist, p.counters, p.ep, (int)(e & 0xfffff),
                         (p.g.N + kFinThreads / 4 - 1) / (kFinThreads / 4) + 1, 0);
}

// Every screen step of every problem of a group in one launch: a grid of
// workgroups that are all resident at once (cooperative launch) walks the
// stages of each step in order (FFT columns, FFT rows, matrix product,
// epilogue), with a grid-wide barrier between stages.  Within a stage the
// workgroups take the stage's map entries one at a time from a counter
// (ctr[4 q + stage], zero at the start), so that entries of unequal cost
// (problems of different sizes) spread as they do over a launch's
// workgroups.  n[q] holds the number of map entries of each stage at step
// q.  The same device bodies as the per-stage kernels, entry for entry, so
// the fields are those of the per-stage launches bit for bit.
template <typename F>
__device__ inline void take_items(int* __restrict__ ctr, int count, F&& body) {
  __shared__ int item;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(ctr, 1);
    __syncthreads();
    const int i = item;
    __syncthreads();  // every thread has read item before it changes
    if (i >= count) break;  // uniform over the workgroup
    body(i);
    __syncthreads();  // the LDS of this entry is free for the next one
  }
}

__global__ void __launch_bounds__(kPersistThreads) multi_persistent(const MultiProblem* __restrict__ mp,
                                                                    const unsigned* __restrict__ map_cols,
                                                                    const unsigned* __restrict__ map_rows,
                                                                    const unsigned* __restrict__ map_apply,
                                                                    const unsigned* __restrict__ map_fin,
                                                                    const int4* __restrict__ n, int* __restrict__ ctr,
                                                                    int qmax) {
  extern __shared__ double2 L[];
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int q = 0; q < qmax; ++q) {
    const int4 cnt = n[q];
    take_items(ctr + 4 * q, cnt.x, [&](int i) {
      const unsigned e = map_cols[i];
      const MultiProblem& p = mp[e >> 20];
      fftb::fft_cols_body(q == 0 ? p.u_in : p.u, p.Y, p.tw, p.g.N, p.g.bc, p.g.P, p.g.P1, p.g.P2, p.logP1, p.CA,
                          (int)(e & 0xfffff), L);
    });
    grid.sync();
    take_items(ctr + 4 * q + 1, cnt.y, [&](int i) {
      const unsigned e = map_rows[i];
      const MultiProblem& p = mp[e >> 20];
      fftb::fft_rows_body(p.Y, p.c, p.tw, p.g.P, p.g.P1, p.g.P2, p.logP2, p.RB, p.g.M, (int)(e & 0xfffff), L);
    });
    grid.sync();
    take_items(ctr + 4 * q + 2, cnt.z, [&](int i) {
      const unsigned e = map_apply[i];
      const MultiProblem& p = mp[e >> 20];
      const int local = (int)(e & 0xfffff);
      if (p.fp64) {
        const int nsb = p.g.T / p.sub;
        apply_matrix_body<double>(p.g, p.tmat64, p.c, p.part, local % nsb, local / nsb, p.groups, p.sub, L);
      } else {
        const int nx = p.g.N >> 9;
        apply_c64_body<kPersistUnroll>(p.g, p.tmat, p.c, p.part, local % nx, local / nx, p.groups,
                                       reinterpret_cast<float2*>(L));
      }
    });
    grid.sync();
    take_items(ctr + 4 * q + 3, cnt.w, [&](int i) {
      const unsigned e = map_fin[i];
      const MultiProblem& p = mp[e >> 20];
      double2* hist = p.hist ? p.hist + (size_t)q * p.g.N : nullptr;
      finalize_body<double2>(p.g, p.rec, p.c, p.part, p.groups, 1, p.u, hist, p.counters, p.ep, (int)(e & 0xfffff),
                             (p.g.N + kFinThreads / 4 - 1) / (kFinThreads / 4) + 1, 0);
    });
    grid.sync();
  }
}

__global__ void zero_ints(int* __restrict__ a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

}  // namespace

// Mode groups (second grid dimension): enough workgroups to give every CU
// several wavefronts per SIMD.
int superpose_sub(const Geometry& g) { return g.T < kSub ? g.T : kSub; }

static int groups_for(const Geometry& g, int sub) {
  const int tiles = (g.T + sub - 1) / sub;
  int groups = (256 * 4 * 6) / (tiles * kWaves);
  if (groups < 1) groups = 1;
  const int maxg = (g.M + kWaves - 1) / kWaves;
  if (groups > maxg) groups = maxg;
  if (groups > 128) groups = 128;
  return groups;
}

int superpose_groups(const Geometry& g) { return groups_for(g, superpose_sub(g)); }

// Interval-owner sum: a pass handles 61 intervals, so a super-tile spans
// about 56 ray spacings (rho points each): most lanes own an interval and
// the tile still fits one pass unless rays crowd (random medium, N = 8192:
// 39.2 us per screen against 42.2 us at 48 spacings, 45.7 at 40 and 49.6 at
// 64, where a second pass is common); at most 448 points (FP32: the one-field
// accumulator rows) or 256 (FP64) for the LDS accumulators.
static int iv_sub(const Geometry& g, int precision) {
  int s = (56 * g.rho) / 64;
  const int smax = precision == SWKB_FP64 ? 4 : (int)kPolarTiles;
  if (s > smax) s = smax;
  if (s < 1) s = 1;
  return g.T < s ? g.T : s;
}

// Mode groups of the complex64 matrix product: about 512 workgroups of 512
// points (two per CU), each wavefront streaming every (4 G)-th row of T.
// Measured on the duct (N = 16384, M = 4096): 16 groups 6.7 TB/s, 48 groups
// 6.3 TB/s; a plain streaming read of the same bytes reaches 7.05 TB/s.
static int c64_groups(const Geometry& g) {
  int G = 512 / (g.N / 512 > 0 ? g.N / 512 : 1);
  const int maxg = (g.M + kWaves - 1) / kWaves;
  if (G > maxg) G = maxg;
  return G < 1 ? 1 : G;
}

int partial_groups(const Geometry& g) {
  int m = superpose_groups(g);
  m = c64_groups(g) > m ? c64_groups(g) : m;
  for (int s = 1; s <= 8; ++s) m = groups_for(g, s) > m ? groups_for(g, s) : m;
  return m;
}

// Which sum kernel (measured on the MI355X, random medium N = 8192): for one
// FP32 field the interval walk (16.5 ms per 400 screens against 22.7 ms with
// the owner map); for FP64 and for batches of fields, whose points carry more
// work per evaluation, the owner map (batch of 4: 83.0 against 86.8 ms per run).
template <typename T, int NB, int SUBMAX>
static void launch_sum(const swkb_plan_s& pl, const dim3& grid, const DevModes& md, const Epi& ep, int sub, int batch,
                       hipStream_t st) {
  if constexpr (std::is_same<T, float>::value && NB == 1) {
    if (!pl.cpol) return;  // reported by launch_superpose
    // the accumulator rows are the kernel's static LDS (at most kPolarTiles
    // tiles: launch_superpose checks)
    hipLaunchKernelGGL((superpose_iv_kernel<T, NB, false>), dim3(grid.x, grid.y, 1), dim3(64 * kWaves), 0, st,
                       pl.g, md, pl.rec, pl.c, pl.cpol, pl.part, static_cast<typename CplxOf<T>::type*>(nullptr), ep,
                       sub, batch);
  } else {
    struct alignas(16) LRec {
      T v[9];
    };
    const size_t work = (size_t)kWaves * (64 * sizeof(LRec) + SUBMAX * 64 * sizeof(int));
    const size_t red = sizeof(T) * 2 * (size_t)kWaves * NB * SUBMAX * 64;
    const dim3 g3(grid.x, grid.y, (batch + NB - 1) / NB);
    hipLaunchKernelGGL((superpose_own_kernel<T, NB, SUBMAX>), g3, dim3(64 * kWaves), work > red ? work : red, st,
                       pl.g, md, pl.rec, pl.c, pl.part, ep, sub, batch);
  }
}

Epi epi_of(const swkb_plan_s& pl) {
  Epi ep;
  ep.absorber_bot = pl.p.absorber_bot;
  ep.absorber_top = pl.p.absorber_top;
  ep.caustic_tol = pl.p.caustic_tol;
  ep.mprime_off = pl.g.bc == SWKB_BC_PERIODIC ? 0 : pl.g.N;
  return ep;
}

hipError_t launch_superpose(const swkb_plan_s& pl, double2* out, double2* hist, int batch, hipStream_t st) {
  const Geometry& g = pl.g;
  const Epi ep = epi_of(pl);
  // the one-field FP32 sum reads the modes in polar form and accumulates in
  // rows of at most kPolarTiles tiles
  if (pl.precision != SWKB_FP64 && batch == 1 && !pl.cpol) return hipErrorInvalidValue;
  // batches keep the accumulators of NB fields in LDS: 256-point super-tiles
  int sub = iv_sub(g, pl.precision);
  if (batch > 1 && sub > 4) sub = 4;
  if (pl.precision != SWKB_FP64 && batch == 1 && sub > (int)kPolarTiles) return hipErrorInvalidValue;
  const int groups = groups_for(g, sub);
  DevModes md{pl.xi, pl.pbar, pl.e1r, pl.frac};
  const dim3 grid((g.T + sub - 1) / sub, groups);
  if (pl.precision == SWKB_FP64) {
    if (batch == 1) launch_sum<double, 1, 4>(pl, grid, md, ep, sub, batch, st);
    else launch_sum<double, 2, 4>(pl, grid, md, ep, sub, batch, st);
  } else {
    if (batch == 1) launch_sum<float, 1, 8>(pl, grid, md, ep, sub, batch, st);
    else launch_sum<float, 4, 4>(pl, grid, md, ep, sub, batch, st);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finalize_kernel<double2>, dim3((g.N + kFinThreads / 4 - 1) / (kFinThreads / 4) + 1, batch), dim3(kFinThreads), 0, st, g, pl.rec, pl.c,
                     pl.part, groups, batch, out, hist, pl.counters, ep, nullptr);
  return hipGetLastError();
}

hipError_t launch_build_matrix(const swkb_plan_s& pl, hipStream_t st) {
  const Geometry& g = pl.g;
  const Epi ep = epi_of(pl);
  const int sub = iv_sub(g, pl.precision);
  const int groups = groups_for(g, sub);
  DevModes md{pl.xi, pl.pbar, pl.e1r, pl.frac};
  const dim3 grid((g.T + sub - 1) / sub, groups);
  // points a mode does not reach stay zero
  const size_t bytes = (size_t)g.N * g.M * (pl.precision == SWKB_FP64 ? sizeof(double2) : sizeof(float2));
  hipError_t e = hipMemsetAsync(pl.tmat, 0, bytes, st);
  if (e != hipSuccess) return e;
  if (pl.precision == SWKB_FP64)
    hipLaunchKernelGGL((superpose_iv_kernel<double, 1, true>), grid, dim3(64 * kWaves), 0, st, g, md, pl.rec, pl.c,
                       nullptr, pl.part, static_cast<double2*>(pl.tmat), ep, sub, 1);
  else
    hipLaunchKernelGGL((superpose_iv_kernel<float, 1, true>), grid, dim3(64 * kWaves), 0, st, g, md, pl.rec, pl.c,
                       nullptr, pl.part, static_cast<float2*>(pl.tmat), ep, sub, 1);
  return hipGetLastError();
}

hipError_t launch_apply_matrix(const swkb_plan_s& pl, double2* out, double2* hist, int batch, hipStream_t st) {
  const Geometry& g = pl.g;
  const Epi ep = epi_of(pl);
  const int sub = superpose_sub(g);
  if (batch == 1 && pl.precision != SWKB_FP64 && g.N % 512 == 0) {
    const int groups = c64_groups(g);  // 512-point workgroups
    hipLaunchKernelGGL(apply_matrix_c64_kernel, dim3(g.N / 512, groups), dim3(64 * kWaves),
                       sizeof(float2) * kWaves * 4 * 64 * 2, st, g, static_cast<const float4*>(pl.tmat), pl.c,
                       pl.part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel<double2>, dim3((g.N + kFinThreads / 4 - 1) / (kFinThreads / 4) + 1, 1), dim3(kFinThreads), 0, st, g, pl.rec, pl.c,
                       pl.part, groups, 1, out, hist, pl.counters, ep, nullptr);
    return hipGetLastError();
  }
  if (batch == 1) {
    const int groups = superpose_groups(g);
    const size_t red = sizeof(double2) * 64 * kWaves * kSub;
    const dim3 grid(g.T / sub, groups);
    if (pl.precision == SWKB_FP64)
      hipLaunchKernelGGL(apply_matrix_kernel<double>, grid, dim3(64 * kWaves), red, st, g,
                         static_cast<const double2*>(pl.tmat), pl.c, pl.part, sub);
    else
      hipLaunchKernelGGL(apply_matrix_kernel<float>, grid, dim3(64 * kWaves), red, st, g,
                         static_cast<const float2*>(pl.tmat), pl.c, pl.part, sub);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel<double2>, dim3((g.N + kFinThreads / 4 - 1) / (kFinThreads / 4) + 1, 1), dim3(kFinThreads), 0, st, g, pl.rec, pl.c,
                       pl.part, groups, 1, out, hist, pl.counters, ep, nullptr);
    return hipGetLastError();
  }
  // several fields: one complex matrix product U[b][m] = sum_j C[b][j] T[j][m]
  // on the matrix cores, mode-group partials summed in FP64 by the epilogue
  int groups = 1;
  hipError_t e = launch_batch_product(pl, batch, st, &groups);
  if (e != hipSuccess) return e;
  const dim3 fin(finalize_blocks(g), batch);
  if (pl.precision == SWKB_FP64)
    hipLaunchKernelGGL(finalize_kernel<double2>, fin, dim3(kFinThreads), 0, st, g, pl.rec, pl.c, pl.part, groups,
                       batch, out, hist, pl.counters, ep, pl.menergy);
  else
    hipLaunchKernelGGL(finalize_kernel<float2>, fin, dim3(kFinThreads), 0, st, g, pl.rec, pl.c,
                       reinterpret_cast<const float2*>(pl.part), groups, batch, out, hist, pl.counters, ep,
                       pl.menergy);
  return hipGetLastError();
}

int finalize_blocks(const Geometry& g) { return (g.N + kFinThreads / 4 - 1) / (kFinThreads / 4) + 1; }

int apply_multi_groups(const Geometry& g) { return c64_groups(g); }

hipError_t launch_apply_multi(const MultiProblem* mp, const unsigned* map_apply, int n_apply,
                              const unsigned* map_fin, int n_fin, int step, hipStream_t st) {
  if (n_apply > 0) {
    hipLaunchKernelGGL(apply_c64_multi, dim3(n_apply), dim3(64 * kWaves), apply_lds_bytes(), st,
                       mp, map_apply);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (n_fin > 0) {
    hipLaunchKernelGGL(finalize_multi, dim3(n_fin), dim3(kFinThreads), 0, st, mp, map_fin, step);
    return hipGetLastError();
  }
  return hipSuccess;
}


// One cooperative launch for every screen step of a group (see
// multi_persistent): the largest grid whose workgroups all fit on the device
// at once, at most max_blocks; *blocks_out gets the grid size.  ctr: 4 qmax
// ints of device memory for the stage counters.
hipError_t launch_multi_persistent(const MultiProblem* mp, const unsigned* map_cols, const unsigned* map_rows,
                                   const unsigned* map_apply, const unsigned* map_fin, const int4* n, int* ctr,
                                   int qmax, size_t lds, int max_blocks, hipStream_t st, int* blocks_out) {
  int dev = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(multi_persistent),
                                                     kPersistThreads, lds);
  if (e != hipSuccess) return e;
  int blocks = per_cu * prop.multiProcessorCount;
  if (max_blocks > 0 && blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) return hipErrorInvalidConfiguration;
  if (blocks_out) *blocks_out = blocks;
  // the stage counters start at zero (a kernel, not a memset: callers may capture this)
  hipLaunchKernelGGL(zero_ints, dim3((4 * qmax + 255) / 256), dim3(256), 0, st, ctr, 4 * qmax);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&mp, (void*)&map_cols, (void*)&map_rows, (void*)&map_apply, (void*)&map_fin, (void*)&n,
                  (void*)&ctr, (void*)&qmax};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(multi_persistent), dim3(blocks),
                                    dim3(kPersistThreads), args, (unsigned)lds, st);
}

size_t apply_lds_bytes() {
  const size_t c64 = sizeof(float2) * kWaves * 4 * 64 * 2, f64 = sizeof(double2) * 64 * kWaves * kSub;
  return c64 > f64 ? c64 : f64;
}

// The FP64 product's single-problem blocking: 64-point tiles per workgroup
// and mode groups.
int apply_f64_sub(const Geometry& g) { return superpose_sub(g); }
int apply_f64_groups(const Geometry& g) { return superpose_groups(g); }

}  // namespace swkb
