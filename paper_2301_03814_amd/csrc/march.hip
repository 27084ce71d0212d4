// Step 2 of a screen: WKB across the screen, one ray per (mode, launch
// point), and the per-mode bookkeeping the interpolation needs.
//
// Rays follow the characteristic system of the eikonal and transport
// equations (Appendix A, eqs. charsys, charsys_s), reparametrised by the
// range x (dt = dx / (2 psi_x); Sec. 2.1.2 admits any eikonal/transport
// solver) and marched with S classical RK4 steps so that every ray lands
// on x_{q+1}.  With p = psi_x = sqrt(eps - q^2), q = psi_z:
//   dz/dx = q/p,   dq/dx = eps_z / (2p),
//   dZs/dx = (eps Qs - q eps_z Zs / 2) / p^3,
//   dQs/dx = (eps_zz / (2p) - eps_z^2 / (4p^3)) Zs + q eps_z / (2p^3) Qs,
// where Zs = dz/ds, Qs = dq/ds at fixed x carry the ray-tube width.  The
// transport amplitude on arrival is a = sqrt(p0 / (p Zs)) (the Jacobian
// J = X_t Z_s - Z_t X_s of Appendix A with A = A0 sqrt(J0/J)).
//
// Phase split: psi = xi (z - z0') + pbar (x - x_q) + dpsi.  The first term
// is exact on the grid (an integer number of 1/P turns), the second is one
// FP64 number per mode, and only the small deviation dpsi is marched:
//   d dpsi/dx = ((eps - eps_ref_n) - (q - xi)(q + xi)) / (p + pbar) + q (q - xi) / p
// (= eps/p - xi q/p - pbar, written in small quantities).  State per ray:
// dz = z - s, dq = q - xi, dpsi in T (FP32 in the mixed path); the ray-tube
// variations Zs, Qs are accumulated in FP64 in both precisions and the
// amplitude on arrival is formed in FP64.  In the mixed path each RK4 step
// starts from the FP64 tube rounded to FP32, forms its stages and its
// increment in FP32 (their coefficients come from the FP32 ray state) and
// adds the increment in FP64: an increment is ~1e-2 of Zs, so the tube keeps
// about 1e-9 relative accuracy where an FP32 state would round by ~6e-8 a
// step -- the ray-Jacobian amplitude near turning points of the x-march
// (p -> 0, where 1/p^3 drives the tube) stays at FP64 accuracy.
//
// Ray r of mode n starts at s_r = z_a + (r rho - E) h with q = xi_n
// (Sec. 2.1.2 initial conditions), Zs = 1, Qs = 0.  A ray is dead when
// p^2 <= p2_floor at launch or at any stage, caustic when Zs <= 0 at any
// stage; dead and caustic rays do not contribute.
#include "medium.h"

// The compiler's indexed buffer load of four dwords (descriptor, index,
// byte offset, scalar byte offset, cache bits), named by its intrinsic.
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ f32x4 struct_buffer_load_f32x4(i32x4 rsrc, int vindex, int voffset, int soffset, int aux)
    __asm("llvm.amdgcn.struct.buffer.load.v4f32");

namespace swkb {
namespace {

struct ModeC {
  double xi, omx2;  // xi, 1 - xi^2
  double pbar, e1r; // reference p and eps - 1 of the mode
  double pb2;       // pbar^2 = 1 - xi^2 + e1r
};

template <typename T>
struct Deriv {
  T dz, dq, dps;
  T Zs, Qs;
};

enum { kLive = 0, kDeadLaunch = 1, kDead = 2, kCaustic = 3 };

// Work of one ray: RK4 stage evaluations, direct medium evaluations,
// Gaussian terms inside their cutoff, medium values read from a table (a
// medium with kTableReads sets the last from the ray's evaluation count at
// the end of the march instead of counting each read).
struct Work {
  int rhs = 0, med = 0, terms = 0, tab = 0;
};

// Wavefront-uniform constants of a march, computed once on the host.
struct MarchK {
  double hx, h6;   // RK4 step dx / S and hx / 6
  double inv_h;    // 1 / h
  double inv_dzt;  // 1 / dz_t of the medium table (table march only), and in FP32:
  float inv_dz, half_inv_dz, inv_dz2, two_dz, dz_sq;  // 1/dz_t, 1/(2 dz_t), 1/dz_t^2, 2 dz_t, dz_t^2
};

template <typename T>
__device__ inline T fast_rsqrt(T x);
template <>
__device__ inline double fast_rsqrt<double>(double x) { return 1.0 / sqrt(x); }
template <>
__device__ inline float fast_rsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }

template <typename T>
__device__ inline T fast_rcp(T x);
template <>
__device__ inline double fast_rcp<double>(double x) { return 1.0 / x; }
template <>
__device__ inline float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// Mode constants of the march in T (wavefront-uniform: one mode per wavefront).
template <typename T>
struct ModeT {
  T xi, e1r, pb2, pbar, omx2;
};

template <typename T>
__device__ inline ModeT<T> mode_in(const ModeC& mc) {
  return ModeT<T>{(T)mc.xi, (T)mc.e1r, (T)mc.pb2, (T)mc.pbar, (T)mc.omx2};
}

// Medium evaluated through the generic device function (any kind, mirror).
template <typename T>
struct GenericMedium {
  static constexpr bool kTableReads = false;
  DevMedium md;
  double x_q, hx2;  // stage k sits at x_q + k * hx2
  double s;         // launch height of this lane's ray
  // stage heights are carried as the displacement dz itself
  __device__ static T pos(T dz) { return dz; }
  __device__ static T pos_scale(T h) { return h; }
  __device__ static T advance(T p, T hs, T kdz) { return p + hs * kdz; }
  __device__ Med<T> eval(int k, T dz, Work& c) const {
    ++c.med;
    return medium_eval<T>(md, x_q + k * hx2, s, dz, c.terms);
  }
  __device__ static constexpr T hz_scale() { return T(1); }
  __device__ static constexpr T hzz_scale() { return T(1); }
};

// Gaussian-sum medium from the per-screen tables (wavefront-uniform, read
// through scalar loads): for stage k and bump i,
//   ax = a_i exp(-(x_k - cx_i)^2 / (2 s_i^2)),  cut = 64 s_i^2 - (x_k - cx_i)^2
// (stage[k * nl + i]); nh = -1/(2 s_i^2) (times log2 e in FP32), is2 = 1/s_i^2
// (term[i]); czl = cz_i - z_w relative to the wavefront's reference height.
// A bump contributes when (z - cz)^2 <= cut, i.e. inside its 8-sigma disc.
template <typename T>
struct T2 { T x, y; };

// e^x for a Gaussian term inside its 8-sigma cutoff (x in [-32, 0]).
// FP32: the hardware exp2 (the tables carry the factor log2 e).  FP64:
// Cody-Waite reduction x = k ln2/64 + r, with ln2/64 split into a 32-bit head
// (k ln2/64_head exact for |k| < 2^21) and the remainder, |r| <= ln2/128;
// e^r from its Taylor polynomial of degree 5 by Horner; then
// e^x = 2^(k >> 6) 2^((k & 63) / 64) e^r with the 64 powers 2^(j/64) from a
// table in LDS (filled by the kernel with the device exp2).  Relative error
// at most 2.9e-16 over [-32, 0] with correctly rounded table entries (the
// FMAs emulated with one exact rounding each, against a 50-digit exp:
// tests/test_exp_constants.py), plus the table's own rounding; no overflow
// or underflow there.
__device__ inline double exp_gauss(double x, const double* __restrict__ pow2_64) {
  constexpr double k64InvLn2 = 92.33248261689366;
  constexpr double kLn2Head = 0.01083042469326756;     // 0x1.62e42fee00000p-7
  constexpr double kLn2Tail = 2.9815858269852933e-12;  // ln2/64 - kLn2Head
  // 1/k!, k = 5 .. 0
  constexpr double kC[6] = {0.008333333333333333, 0.041666666666666664, 0.16666666666666666, 0.5, 1.0, 1.0};
  const double kf = rint(x * k64InvLn2);
  double r = fma(-kf, kLn2Head, x);
  r = fma(-kf, kLn2Tail, r);
  double p = kC[0];
#pragma unroll
  for (int i = 1; i < 6; ++i) p = fma(p, r, kC[i]);
  const int k = (int)kf;
  return ldexp(pow2_64[k & 63] * p, k >> 6);
}

template <typename T>
struct GaussMedium {
  static constexpr bool kTableReads = false;
  const T2<T>* __restrict__ stage;
  const T2<T>* __restrict__ term;
  const T* __restrict__ czl;
  int nl;
  T zl0;  // launch height of this lane's ray relative to the wavefront reference
  const double* __restrict__ pow2_64 = nullptr;  // FP64: 2^(j/64), j < 64, in LDS
  __device__ static T pos(T dz) { return dz; }
  __device__ static T pos_scale(T h) { return h; }
  __device__ static T advance(T p, T hs, T kdz) { return p + hs * kdz; }
  __device__ inline void bump(T z, T c, T2<T> ac, T2<T> tk, T& dn, T& nz, T& nzz, int& nterms) const {
    const T ddz = z - c;
    const T d2 = ddz * ddz;
    if (d2 > ac.y) return;
    ++nterms;
    T ex;
    if constexpr (std::is_same<T, double>::value) ex = exp_gauss(d2 * tk.x, pow2_64);
    else ex = __builtin_amdgcn_exp2f(d2 * tk.x);
    const T gg = ac.x * ex;
    dn += gg;
    const T t = tk.y * gg;
    nz -= ddz * t;
    nzz += (d2 * tk.y - T(1)) * t;
  }
  __device__ Med<T> eval(int k, T dz, Work& c) const {
    ++c.med;
    int& nterms = c.terms;
    const T z = zl0 + dz;
    const T2<T>* __restrict__ st = stage + k * nl;
    T dn = T(0), nz = T(0), nzz = T(0);
    int i = 0;
    // four bumps per iteration: their table entries are fetched together
    for (; i + 4 <= nl; i += 4) {
      const T c0 = czl[i], c1 = czl[i + 1], c2 = czl[i + 2], c3 = czl[i + 3];
      const T2<T> a0 = st[i], a1 = st[i + 1], a2 = st[i + 2], a3 = st[i + 3];
      const T2<T> t0 = term[i], t1 = term[i + 1], t2 = term[i + 2], t3 = term[i + 3];
      this->bump(z, c0, a0, t0, dn, nz, nzz, nterms);
      this->bump(z, c1, a1, t1, dn, nz, nzz, nterms);
      this->bump(z, c2, a2, t2, dn, nz, nzz, nterms);
      this->bump(z, c3, a3, t3, dn, nz, nzz, nterms);
    }
    for (; i < nl; ++i) this->bump(z, czl[i], st[i], term[i], dn, nz, nzz, nterms);
    return from_index<T>(dn, nz, nzz);
  }
  __device__ static constexpr T hz_scale() { return T(1); }
  __device__ static constexpr T hzz_scale() { return T(1); }
};

// Gaussian-sum medium read from a per-screen table (mixed path).  At each
// RK4 stage position x_k of the screen, eps - 1 is the cubic Hermite
// interpolant in z between nodes z_lo + i dz_t of its FP64 values and
// z-derivatives; eps_z / 2 and eps_zz / 2 come from the interpolant's
// derivatives.  Per interval the table holds power-form coefficients in
// u = (z - z_i)/dz_t, p(u) = c0 + c1 u + c2 u^2 + c3 u^3, as one float4.
// The interpolation error is of order dz_t^4 max|eps^(4)| in eps,
// dz_t^3 max|eps^(4)| in eps_z and dz_t^2 max|eps^(4)| in eps_zz; with
// dz_t = s_min / 40 and bumps of relative height 1e-2 the first two stay at
// the FP32 rounding of a direct evaluation (random medium: 1e-11 against an
// FP32 ulp of 5e-10 in eps - 1, 3e-7 relative in eps_z) and eps_zz, which
// only enters the ray-tube amplitude, within 1e-4 relative.  Heights
// outside the table fall back to the direct evaluation.
//
// The table row of a stage is wavefront-uniform; an interval's entry is read
// by a buffer load indexed by the interval (the descriptor: the row's base,
// a 16-byte stride and the row length as the record count), which takes the
// interval index as it is, without a per-lane address computation, and whose
// hardware range check agrees with the caller's own test.
constexpr int kBufferWord3 = 0x00020000;  // 32-bit data format, CDNA buffer descriptor word 3

__device__ inline f32x4 row_load(const float4* row, unsigned n, unsigned i) {
  const unsigned long long a = (unsigned long long)row;
  i32x4 r;
  r.x = (int)(unsigned)a;
  r.y = (int)((unsigned)(a >> 32) | (16u << 16));  // base bits 32..47, stride 16 bytes
  r.z = (int)n;
  r.w = kBufferWord3;
  return struct_buffer_load_f32x4(r, (int)i, 0, 0, 0);
}

// eval returns hz = p' and hzz = p''/2 in node units; hz_scale() and
// hzz_scale() take them to eps_z / 2 and eps_zz / 2, so that the scales
// ride on products the right-hand side forms anyway.
//
// Stage heights are carried as the table coordinate t = dz / dz_t + tl
// itself (node spacings above node j0): a stage's height is then one FMA
// from the step's first, t + (h / dz_t) k_dz, and the direct evaluation
// recovers dz = (t - tl) dz_t.
template <bool kHold>
struct TableMedium {
  static constexpr bool kTableReads = true;
  const float4* __restrict__ ta;  // [(2S+1)][ni]
  unsigned ni;                    // intervals
  float inv_dz, half_inv_dz;      // 1/dz_t, 1/(2 dz_t)
  float inv_dz2;                  // 1/dz_t^2
  float dzt, two_dz, dz_sq;       // dz_t, 2 dz_t, dz_t^2 (direct values into node units)
  int j0;      // node at or below the wavefront's reference height z_w
  float tl;    // this lane's launch height above node j0, in node spacings
  GaussMedium<float> direct;
  __device__ float pos(float dz) const { return dz * inv_dz + tl; }
  __device__ float pos_scale(float h) const { return h * inv_dz; }
  __device__ static float advance(float t, float hs, float kdz) { return t + hs * kdz; }
  // kHold: keep the entry last read (interval held_iv of the previous
  // evaluation's row, ~0 if none).  RK4 stages 2 and 3 share a range
  // position, and so do stage 4 and the next step's stage 1 (and the launch
  // with the first stage, the last stage with the arrival); between such
  // stages a ray moves by far less than a table interval, so the second
  // usually finds its entry held and a wavefront reads only for the lanes
  // that do not.
  mutable f32x4 held;
  mutable unsigned held_iv = ~0u;
  template <bool kSameRow>
  __device__ Med<float> eval(int k, float t, Work& c) const {
    // node index floor(t) in one instruction (a saturating conversion, like
    // the one of floorf(t) to int) and the offset t - floor(t) in another
    int ti;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(ti) : "v"(t));
    // unsigned wrap sends heights below the table (and saturated conversions) out of range too
    const unsigned iv = (unsigned)j0 + (unsigned)ti;
    if (!(iv < ni)) {
      held_iv = ~0u;
      Med<float> m = direct.eval(k, (t - tl) * dzt, c);
      m.hz *= two_dz;
      m.hzz *= dz_sq;
      return m;
    }
    const float u = __builtin_amdgcn_fractf(t);
    if (!(kHold && kSameRow) || iv != held_iv) {
      held = row_load(ta + (size_t)k * ni, ni, iv);
      held_iv = iv;
    }
    const f32x4 a = held;
    // Horner for p, p' and p''/2 together
    float p = a.w * u + a.z;
    float d1 = a.w * u + p;         // 2 c3 u + c2
    const float d2 = a.w * u + d1;  // 3 c3 u + c2 = p''/2
    p = p * u + a.y;
    d1 = d1 * u + p;                // 3 c3 u^2 + 2 c2 u + c1 = p'
    p = p * u + a.x;
    Med<float> m;
    m.e1 = p;
    m.hz = d1;
    m.hzz = d2;
    return m;
  }
  __device__ float hz_scale() const { return half_inv_dz; }
  __device__ float hzz_scale() const { return inv_dz2; }
};

// Right-hand side at stage k, the n-th evaluation (n = 1..4) of RK4 step i,
// at the stage height pos (in the medium's coordinate).  Returns false when
// the ray stops there, with st = kCaustic (Z_s <= 0 at the stage) or else
// kDead (p^2 <= p2_floor), plus 4 (4 i + n - 1); the medium is evaluated in
// either case, so that both tests are taken on one branch that a wavefront
// of live rays skips.
// Medium at stage k; kSameRow: the previous evaluation was on the same row
// (same range position), which a table medium may use.
template <bool kSameRow, typename MED, typename POS>
__device__ inline auto eval_medium(const MED& med, int k, POS pos, Work& c) {
  if constexpr (MED::kTableReads) return med.template eval<kSameRow>(k, pos, c);
  else return med.eval(k, pos, c);
}

template <bool kSameRow, typename T, typename MED, typename POS>
__device__ inline bool rhs(const MED& med, const ModeT<T>& mc, int k, int n, int i, POS pos, T dq, T Zs, T Qs,
                          T p2_floor, Deriv<T>& d, Work& c, int& st) {
  const Med<T> m = eval_medium<kSameRow>(med, k, pos, c);
  const T xi = mc.xi;
  const T w = dq * (T(2) * xi + dq);          // q^2 - xi^2
  const T num = (m.e1 - mc.e1r) - w;          // p^2 - pbar^2, in small quantities
  const T p2 = num + mc.pb2;
  const bool ok = (Zs > T(0)) & (p2 > p2_floor);
  if (__builtin_expect(!ok, 0)) {
    st = (Zs > T(0) ? kDead : kCaustic) + 4 * (4 * i + n - 1);
    return false;
  }
  const T ip = fast_rsqrt<T>(p2);
  const T q = xi + dq;
  d.dz = q * ip;
  d.dps = num * fast_rcp<T>(p2 * ip + mc.pbar) + dq * d.dz;
  d.dq = m.hz * (med.hz_scale() * ip);        // (eps_z/2) / p
  // ray-tube variations:
  //   Z_s' = (eps Q_s - q (eps_z/2) Z_s) / p^3,
  //   Q_s' = ((eps_zz/2) - (eps_z/2)^2 / p^2) Z_s / p + q (eps_z/2) Q_s / p^3
  const T ip2 = ip * ip, ip3 = ip2 * ip;
  const T qa = q * (ip2 * d.dq);              // q (eps_z/2) / p^3
  d.Zs = (ip3 + ip3 * m.e1) * Qs - qa * Zs;
  d.Qs = (m.hzz * med.hzz_scale() - d.dq * d.dq) * ip * Zs + qa * Qs;
  return true;
}

// First grid index m in [0, N] with z_m = z_a + m h >= key (N + 1 if none,
// 0 for an empty key), with the FP64 comparisons of the bracket search.
__device__ inline int first_point_at_or_above(const Geometry& g, double key, double inv_h) {
  if (key == -INFINITY) return 0;
  const double x = (key - g.z_a) * inv_h;
  int ci = x <= 0.0 ? 0 : (x >= (double)(g.N + 1) ? g.N + 1 : (int)ceil(x));
  // exact decisions with the same arithmetic as z_m = z_a + m h.  The
  // estimate's rounding is a few 1e-11 grid steps here (|x| <= 2^17), so it
  // is exact unless x lies that close to an integer: the two neighbouring
  // decisions confirm it, and the stepping loops (z_m increases with m)
  // correct it otherwise
  auto reaches = [&](int m) { return g.z_a + (double)m * g.h >= key; };
  const bool high = ci > 0 && reaches(ci - 1);
  const bool low = ci <= g.N && !reaches(ci);
  if (__builtin_expect(high || low, 0)) {
    while (ci > 0 && reaches(ci - 1)) --ci;
    while (ci <= g.N && !reaches(ci)) ++ci;
  }
  return ci;
}

// Transport amplitude sqrt(p0 / (p Zs)) = sqrt(p0 / p) Zs^(-1/2) with the
// ray tube's factor in FP64: Zs^(-1/2) from the hardware estimate refined by
// two Newton steps y <- y (3 - Zs y^2) / 2 (each doubles the correct bits of
// the estimate, which has at least 22, so the result is FP64-accurate); the
// slowness ratio p0 / p in T (the launch and arrival slownesses are T
// quantities; in FP32 from the hardware square root and reciprocal square
// root, within a few ulp, as the FP32 amplitude that is stored).
template <typename T>
__device__ inline double tube_amplitude(T p02, T p2, double Zs) {
  if constexpr (std::is_same<T, double>::value) {
    return sqrt(sqrt(p02) / (sqrt(p2) * Zs));
  } else {
    double y = __builtin_amdgcn_rsq(Zs);
    y = y * (1.5 - 0.5 * Zs * y * y);
    y = y * (1.5 - 0.5 * Zs * y * y);
    return (double)__builtin_amdgcn_sqrtf(__builtin_amdgcn_sqrtf(p02) * fast_rsqrt<T>(p2)) * y;
  }
}

// One wavefront lane per ray: RK4 across the screen.  Writes the arrival
// record and returns the lane's status and work counts.
template <typename T, typename MED>
__device__ inline void march_ray(const MED& med, const ModeC& mc, const Geometry& g, const MarchK& mk, bool active,
                                 size_t o, double s_launch, const DevRecords& rec, int& st, Work& c) {
  T dz = T(0), dq = T(0), dps = T(0);
  double Zs = 1.0, Qs = 0.0;  // ray tube, accumulated in FP64
  double amp = 0.0;
  st = kLive;
  if (!active) return;
  const ModeT<T> mt = mode_in<T>(mc);
  const Med<T> m0 = eval_medium<false>(med, 0, med.pos(T(0)), c);
  int evals = 1;  // medium evaluations of this ray
  const T p02 = mt.omx2 + m0.e1;
  const T pfl = (T)g.p2_floor;
  if (!(p02 > pfl)) {
    st = kDeadLaunch;
  } else {
    const T hh = (T)(0.5 * mk.hx), hf = (T)mk.hx, h6 = (T)mk.h6;
    const double h6d = (double)h6;
    // stage offsets in the medium's coordinate
    const auto hh_p = med.pos_scale(hh), hf_p = med.pos_scale(hf);
    Deriv<T> k1, k2, k3, k4;
    for (int i = 0; i < g.S; ++i) {
      const T zs = (T)Zs, qs = (T)Qs;  // the step's tube in T
      const auto p1 = med.pos(dz);
      if (!rhs<true, T>(med, mt, 2 * i, 1, i, p1, dq, zs, qs, pfl, k1, c, st)) break;
      if (!rhs<false, T>(med, mt, 2 * i + 1, 2, i, med.advance(p1, hh_p, k1.dz), dq + hh * k1.dq, zs + hh * k1.Zs,
                         qs + hh * k1.Qs, pfl, k2, c, st))
        break;
      if (!rhs<true, T>(med, mt, 2 * i + 1, 3, i, med.advance(p1, hh_p, k2.dz), dq + hh * k2.dq, zs + hh * k2.Zs,
                        qs + hh * k2.Qs, pfl, k3, c, st))
        break;
      if (!rhs<false, T>(med, mt, 2 * i + 2, 4, i, med.advance(p1, hf_p, k3.dz), dq + hf * k3.dq, zs + hf * k3.Zs,
                         qs + hf * k3.Qs, pfl, k4, c, st))
        break;
      dz += h6 * (k1.dz + T(2) * k2.dz + T(2) * k3.dz + k4.dz);
      dq += h6 * (k1.dq + T(2) * k2.dq + T(2) * k3.dq + k4.dq);
      dps += h6 * (k1.dps + T(2) * k2.dps + T(2) * k3.dps + k4.dps);
      // the step's weighted slope sum in T; its product with h/6 (exact in
      // FP64 for T = float) and the sum in FP64
      Zs = fma(h6d, (double)(k1.Zs + T(2) * k2.Zs + T(2) * k3.Zs + k4.Zs), Zs);
      Qs = fma(h6d, (double)(k1.Qs + T(2) * k2.Qs + T(2) * k3.Qs + k4.Qs), Qs);
    }
    // completed steps (4 evaluations each), and the evaluations of the step
    // where the ray stopped
    if (st == kLive) {
      c.rhs = 4 * g.S;
      evals += c.rhs;
    } else {
      c.rhs = (st >> 2) & ~3;
      evals += (st >> 2) + 1;
      st &= 3;
    }
    if (st == kLive) {
      if (!(Zs > 0.0)) {
        st = kCaustic;
      } else {
        ++evals;
        const Med<T> m1 = eval_medium<true>(med, 2 * g.S, med.pos(dz), c);
        const T xi = mt.xi;
        const T p2 = mt.omx2 + m1.e1 - dq * (T(2) * xi + dq);
        if (!(p2 > pfl)) st = kDead;
        else amp = tube_amplitude<T>(p02, p2, Zs);
      }
    }
  }
  if constexpr (MED::kTableReads) c.tab = evals - c.med;
  static_cast<T*>(rec.D)[o] = dz;
  static_cast<T*>(rec.Pp)[o] = dps;
  static_cast<T*>(rec.G)[o] = dq;
  static_cast<T*>(rec.A)[o] = st == kLive ? (T)amp : (T)(-st);
  // first grid point at or above the arrival (the scan's running maximum of these gives the brackets)
  rec.cz[o] = st == kLive ? first_point_at_or_above(g, s_launch + (double)dz, mk.inv_h) : 0;
}

// Wavefront sums of the lanes' work counts (the device library's wavefront
// reduction, all 64 lanes taking part).  With S <= 250 a lane makes at most
// 4 S + 2 < 1024 evaluations, so the RK4 and table counts of 64 lanes fit 16
// bits each and share one reduction; the direct-evaluation counts are reduced
// only when some lane has any.
extern "C" __device__ unsigned int __ockl_wfred_add_u32(unsigned int);

__device__ inline void wave_counts(int* __restrict__ wcount, size_t slot, int lane, bool active, int st, Work c,
                                   int S) {
  const unsigned long long bc = __ballot(active && st == kCaustic);
  const unsigned long long bd = __ballot(active && (st == kDead || st == kDeadLaunch));
  if (S <= 250) {
    // sums at most 64 (4 S + 2) = 64128 < 2^16 per field, so the word stays below 2^32
    const unsigned rt = __ockl_wfred_add_u32((unsigned)c.rhs | ((unsigned)c.tab << 16));
    c.rhs = (int)(rt & 0xffffu);
    c.tab = (int)(rt >> 16);
  } else {
    c.rhs = (int)__ockl_wfred_add_u32((unsigned)c.rhs);
    c.tab = (int)__ockl_wfred_add_u32((unsigned)c.tab);
  }
  if (__ballot(c.med != 0 || c.terms != 0)) {
    c.med = (int)__ockl_wfred_add_u32((unsigned)c.med);
    c.terms = (int)__ockl_wfred_add_u32((unsigned)c.terms);
  }
  if (lane == 0) {
    int* wc = wcount + kWaveCounts * slot;
    wc[0] = __popcll(bc);
    wc[1] = __popcll(bd);
    wc[2] = c.rhs;
    wc[3] = c.med;
    wc[4] = c.terms;
    wc[5] = c.tab;
  }
}

// Wavefronts of the Gaussian-sum marches.  A mode's first F = R / 64
// wavefront positions are full (64 rays each).  Its last T = R mod 64 rays
// start at the launch heights of position F whatever the mode, so the tails
// of floor(64 / T) modes share one wavefront, mode after mode in segments of
// T lanes (random medium: R = 1091, a mode's eighteenth wavefront would
// otherwise march 3 rays on 64 lanes, 5.6 % of all wavefronts).  Every ray
// takes the same arithmetic either way; only its mode index becomes a lane
// value on a tail wavefront.
__host__ __device__ inline long long packed_march_waves(const Geometry& g) {
  const int T = g.R & 63;
  const long long full = (long long)g.M * (g.R >> 6);
  if (!T) return full;
  const int per = 64 / T;
  return full + (g.M + per - 1) / per;
}

// A lane's ray on the packed layout: mode j, wavefront position w, ray
// rl within the position (r = 64 w + rl).
struct RayLane {
  int j, w, rl;
  bool active;
  bool lead;  // tail wavefront: first lane of its mode's segment
};

// Counts of a tail wavefront: the first lane of each segment sums its T
// lanes (T - 1 lane reads each) and writes its mode's slot of position F.
__device__ inline void tail_counts(int* __restrict__ wcount, int wpm, const RayLane& rl, int lane, int T, int st,
                                   Work c) {
  const unsigned long long bc = __ballot(rl.active && st == kCaustic);
  const unsigned long long bd = __ballot(rl.active && (st == kDead || st == kDeadLaunch));
  int v0 = c.rhs, v1 = c.med, v2 = c.terms, v3 = c.tab;
  for (int k = 1; k < T; ++k) {
    v0 += __shfl(c.rhs, lane + k);
    v1 += __shfl(c.med, lane + k);
    v2 += __shfl(c.terms, lane + k);
    v3 += __shfl(c.tab, lane + k);
  }
  if (rl.lead && rl.active) {
    const unsigned long long seg = (1ull << T) - 1;
    int* wc = wcount + kWaveCounts * ((size_t)rl.j * wpm + rl.w);
    wc[0] = __popcll((bc >> lane) & seg);
    wc[1] = __popcll((bd >> lane) & seg);
    wc[2] = v0;
    wc[3] = v1;
    wc[4] = v2;
    wc[5] = v3;
  }
}

// Wavefront `wave` of the packed layout (kPack: full positions first, then
// the tails) or of one mode per wavefront position (ceil(R / 64) per mode).
// Returns false when the wavefront has no ray (uniform).  One march body
// serves full and tail wavefronts, the mode index a lane value: inlined once
// per kind, the table march's register allocation spilled inside the step
// loop.  The FP64 march keeps one mode per wavefront: with the mode index a
// lane value it spilled 56 bytes a lane inside its step loop (HBM writes per
// launch 80 -> 176 MB).
template <bool kPack>
__device__ inline bool ray_lane(const Geometry& g, int wave, int lane, int wpm, RayLane& rl, bool& tail) {
  if constexpr (!kPack) {
    tail = false;
    const int j = wave / wpm;
    if (j >= g.M) return false;
    rl.j = j;
    rl.w = wave - j * wpm;
    rl.rl = lane;
    rl.active = rl.w * 64 + lane < g.R;
    rl.lead = lane == 0;
    return true;
  }
  const int F = g.R >> 6;
  tail = wave >= g.M * F;
  if (!tail) {
    const int j = wave / F;
    rl.j = j;
    rl.w = wave - j * F;
    rl.rl = lane;
    rl.active = true;
    rl.lead = lane == 0;
    return true;
  }
  const int T = g.R & 63;
  if (!T) return false;
  const int per = 64 / T;
  const int tw = wave - g.M * F;
  if (tw * per >= g.M) return false;
  const int seg = lane / T;
  rl.j = tw * per + seg;
  rl.w = F;
  rl.rl = lane - seg * T;
  rl.active = seg < per && rl.j < g.M;
  rl.lead = rl.rl == 0;
  if (!rl.active) rl.j = g.M - 1;  // loads stay in range; nothing is marched or written
  return true;
}

// Packed layout for the FP32 Gaussian-sum march without the table.
template <typename T>
constexpr bool packs_tails() { return !std::is_same<T, double>::value; }

__device__ inline ModeC load_mode(const DevModes& modes, int j) {
  ModeC mc;
  mc.xi = modes.xi[j];
  mc.omx2 = 1.0 - mc.xi * mc.xi;
  mc.pbar = modes.pbar[j];
  mc.e1r = modes.e1r[j];
  mc.pb2 = mc.omx2 + mc.e1r;
  return mc;
}

// Any medium kind, ground mirror allowed.  Wavefront w of the grid marches
// rays w_in_mode * 64 + lane of mode j.
template <typename T>
__global__ void __launch_bounds__(256) march_kernel(Geometry g, MarchK mk, DevMedium md, DevModes modes,
                                                    DevRecords rec, int* __restrict__ wcount, double x_q,
                                                    int waves_per_mode) {
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int j = wave / waves_per_mode;
  if (j >= g.M) return;  // uniform per wavefront
  const int w = wave - j * waves_per_mode;
  const int r = w * 64 + lane;
  const bool active = r < g.R;
  const ModeC mc = load_mode(modes, j);
  GenericMedium<T> med;
  med.md = md;
  med.x_q = x_q;
  med.hx2 = 0.5 * mk.hx;
  med.s = g.z_a + (double)(r * g.rho - g.E) * g.h;
  int st;
  Work c;
  march_ray<T>(med, mc, g, mk, active, (size_t)j * g.R + r, g.z_a + (double)(r * g.rho - g.E) * g.h, rec, st, c);
  wave_counts(wcount, (size_t)j * waves_per_mode + w, lane, active, st, c, g.S);
}

// Per-screen Gaussian tables in device memory.
template <typename T>
struct GaussTabs {
  const T2<T>* stage;  // [(2S+1)][nl]
  const T2<T>* term;   // [nl]
  const T* czl;        // [waves_per_mode][nl]: cz_i - z_w per wavefront position w
  int nl;
};

// Gaussian-sum medium without a mirror.  Bump heights are relative to each
// wavefront's first launch height z_w, so FP32 never carries an absolute
// coordinate; all table reads are wavefront-uniform.
// FP64 asks for 5 wavefronts per SIMD (96 VGPRs and a 36-byte spill outside
// the bump loop; at the compiler's choice 101 VGPRs and 4): random medium,
// 1448 -> 1404 us per screen.
template <typename T>
__device__ __forceinline__ void march_gauss_lane(const Geometry& g, const MarchK& mk, const GaussTabs<T>& tabs,
                                                 const DevModes& modes, const DevRecords& rec,
                                                 int* __restrict__ wcount, int waves_per_mode,
                                                 const double* pow2_64, int wave, int lane) {
  RayLane rl;
  bool tail;
  if (!ray_lane<packs_tails<T>()>(g, wave, lane, waves_per_mode, rl, tail)) return;  // uniform per wavefront
  const int w = __builtin_amdgcn_readfirstlane(rl.w);
  const int r = w * 64 + rl.rl;
  const ModeC mc = load_mode(modes, rl.j);
  GaussMedium<T> med;
  med.pow2_64 = pow2_64;
  med.stage = tabs.stage;
  med.term = tabs.term;
  med.czl = tabs.czl + (size_t)w * tabs.nl;
  med.nl = tabs.nl;
  med.zl0 = (T)((double)(rl.rl * g.rho) * g.h);
  int st;
  Work c;
  march_ray<T>(med, mc, g, mk, rl.active, (size_t)rl.j * g.R + r, g.z_a + (double)(r * g.rho - g.E) * g.h, rec,
               st, c);
  if (tail) tail_counts(wcount, waves_per_mode, rl, lane, g.R & 63, st, c);
  else wave_counts(wcount, (size_t)__builtin_amdgcn_readfirstlane(rl.j) * waves_per_mode + w, lane, rl.active, st, c,
                   g.S);
}

template <typename T>
__global__ void __launch_bounds__(256, (std::is_same<T, double>::value ? 5 : 1)) march_gauss_kernel(Geometry g, MarchK mk, GaussTabs<T> tabs,
                                                          DevModes modes, DevRecords rec, int* __restrict__ wcount,
                                                          int waves_per_mode) {
  __shared__ double pow2_64[64];
  if constexpr (std::is_same<T, double>::value) {
    if (threadIdx.x < 64) pow2_64[threadIdx.x] = exp2((double)threadIdx.x * (1.0 / 64.0));
    __syncthreads();
  }
  const int wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int lane = threadIdx.x & 63;
  march_gauss_lane<T>(g, mk, tabs, modes, rec, wcount, waves_per_mode, pow2_64, wave, lane);
}

// Per-screen medium table of the mixed Gaussian-sum march.  Node values at
// height z_lo + i dz_t and stage x_q + k hx/2: eps - 1 and its z-derivative,
// from the same candidate bumps and 8-sigma cutoff as the direct
// evaluation, in FP64.  With g_i the bump value and d = z - cz_i:
//   n - 1 = sum g_i,  n_z = -sum d g_i / s_i^2,  eps - 1 = (n-1)(n+1),  eps_z = 2 n n_z.
// Each block computes 256 consecutive nodes and writes the 255 intervals
// between them (blocks overlap by one node).  Cubic Hermite coefficients
// from node values f and slopes d = dz_t f' at both ends (D = f1 - f0):
//   c0 = f0, c1 = d0, c2 = 3 D - 2 d0 - d1, c3 = -2 D + d0 + d1.
constexpr int kTabBumps = 256;  // bumps staged in LDS per pass
constexpr int kTabNodes = 256;  // nodes per block

__global__ void __launch_bounds__(kTabNodes) medium_table_kernel(const double* __restrict__ prm,
                                                                 const int* __restrict__ list, int nl, double x_q,
                                                                 double hx2, double z_lo, double dzt, int ni,
                                                                 float4* __restrict__ ta) {
  // per bump at this stage: a e^{-(x - cx)^2 / (2 s^2)}, 64 s^2 - (x - cx)^2, cz, 1/s^2
  __shared__ double4 sb[kTabBumps];
  __shared__ double2 nv[kTabNodes];  // eps - 1, dz_t eps_z at this block's nodes
  const int i = blockIdx.x * (kTabNodes - 1) + threadIdx.x;  // node
  const double x = x_q + blockIdx.y * hx2, z = z_lo + i * dzt;
  double dn = 0.0, n1 = 0.0;
  for (int t0 = 0; t0 < nl; t0 += kTabBumps) {
    const int cnt = nl - t0 < kTabBumps ? nl - t0 : kTabBumps;
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const double* b = prm + 1 + 4 * list[t0 + t];
      const double ddx = x - b[2], s2 = b[1] * b[1];
      sb[t] = make_double4(b[0] * exp(-0.5 * ddx * ddx / s2), 64.0 * s2 - ddx * ddx, b[3], 1.0 / s2);
    }
    __syncthreads();
    for (int t = 0; t < cnt; ++t) {
      const double4 b = sb[t];
      const double ddz = z - b.z, dz2 = ddz * ddz;
      if (dz2 > b.y) continue;  // outside the 8-sigma disc
      const double d2 = dz2 * b.w;
      const double gg = b.x * exp(-0.5 * d2);
      dn += gg;
      n1 -= ddz * b.w * gg;
    }
  }
  const double n = 1.0 + dn;
  nv[threadIdx.x] = make_double2(dn * (2.0 + dn), dzt * 2.0 * n * n1);
  __syncthreads();
  if (threadIdx.x >= kTabNodes - 1 || i >= ni) return;
  const double2 p = nv[threadIdx.x], q = nv[threadIdx.x + 1];
  const double D = q.x - p.x;
  const size_t o = (size_t)blockIdx.y * ni + i;
  ta[o] = make_float4((float)p.x, (float)p.y, (float)(3.0 * D - 2.0 * p.y - q.y), (float)(-2.0 * D + p.y + q.y));
}

// Mixed-path Gaussian-sum march through the screen's medium table.
template <bool kHold, bool kPack>
__device__ __forceinline__ void march_table_lane(const Geometry& g, const MarchK& mk, const GaussTabs<float>& tabs,
                                                 const MedTab& mt, const DevModes& modes, const DevRecords& rec,
                                                 int* __restrict__ wcount, int waves_per_mode, int wave, int lane) {
  RayLane rl;
  bool tail;
  if (!ray_lane<kPack>(g, wave, lane, waves_per_mode, rl, tail)) return;  // uniform per wavefront
  const int j = rl.j, w = __builtin_amdgcn_readfirstlane(rl.w);
  const int r = w * 64 + rl.rl;
  const ModeC mc = load_mode(modes, j);
  TableMedium<kHold> med;
  med.direct.stage = tabs.stage;
  med.direct.term = tabs.term;
  med.direct.czl = tabs.czl + (size_t)w * tabs.nl;
  med.direct.nl = tabs.nl;
  med.direct.zl0 = (float)((double)(rl.rl * g.rho) * g.h);
  med.ni = (unsigned)(mt.n - 1);
  med.ta = mt.tab;
  med.inv_dz = mk.inv_dz;
  med.half_inv_dz = mk.half_inv_dz;
  med.inv_dz2 = mk.inv_dz2;
  med.dzt = 0.5f * mk.two_dz;
  med.two_dz = mk.two_dz;
  med.dz_sq = mk.dz_sq;
  const double rel = (g.z_a + (double)(w * 64 * g.rho - g.E) * g.h) - mt.z_lo;  // z_w above the table's base
  med.j0 = (int)floor(rel * mk.inv_dzt);
  med.tl = (float)((rel - (double)med.j0 * mt.dz + (double)(rl.rl * g.rho) * g.h) * mk.inv_dzt);
  int st;
  Work c;
  march_ray<float>(med, mc, g, mk, rl.active, (size_t)j * g.R + r, g.z_a + (double)(r * g.rho - g.E) * g.h, rec,
                   st, c);
  if (tail) tail_counts(wcount, waves_per_mode, rl, lane, g.R & 63, st, c);
  else wave_counts(wcount, (size_t)__builtin_amdgcn_readfirstlane(j) * waves_per_mode + w, lane, kPack || rl.active,
                   st, c, g.S);
}

template <bool kHold, bool kPack>
__device__ __forceinline__ void march_table_body(const Geometry& g, const MarchK& mk, const GaussTabs<float>& tabs,
                                        const MedTab& mt, const DevModes& modes, const DevRecords& rec,
                                        int* __restrict__ wcount, int waves_per_mode) {
  const int wave = __builtin_amdgcn_readfirstlane((int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
  const int lane = threadIdx.x & 63;
  march_table_lane<kHold, kPack>(g, mk, tabs, mt, modes, rec, wcount, waves_per_mode, wave, lane);
}

// Two launch shapes of the same march.  Beside the one-field FP32 sum the
// march keeps the table entry it last read (half the table reads of a step;
// the reads, about 27 cache lines per wavefront load, kept the texture data
// path 82 % busy) and asks for 7 wavefronts per SIMD: 67 VGPRs without
// spills (at 8, the held entry and the RK4 slopes spill to scratch inside the
// step loop): random medium N = 8192, march 94.5 -> 88.5 us, step 53.6 ->
// 52.3 ms per 400 screens.  Beside the sum of several fields (the owner-map
// kernel, 4 wavefronts per SIMD) the march crowds that sum out of the CUs it
// shares when it asks for more wavefronts or holds more registers, so there
// the compiler's own choice runs without the held entry: 4 fields, 80.2 ->
// 71.6 ms per 400 screens (held entry: 73.3 ms).  That shape also keeps one
// mode per wavefront: the packed tails took it from 62 to 67 VGPRs, 7
// wavefronts per SIMD instead of 8 (4 fields: 67.9 -> 74.5 ms).
//
// Both take their arguments as one structure and read each field where it
// is used, through the argument segment: the compiler loads by-value kernel
// arguments on entry, which would hold the record pointers and the count
// buffer (used only after the march) in scalar registers across it and
// spill them to vector lanes.
struct TableMarchArgs {
  Geometry g;
  MarchK mk;
  GaussTabs<float> tabs;
  MedTab mt;
  DevModes modes;
  DevRecords rec;
  int* wcount;
  int waves_per_mode;
};

__device__ inline const TableMarchArgs& table_args() {
  return *(const TableMarchArgs*)__builtin_amdgcn_kernarg_segment_ptr();
}

__global__ void __launch_bounds__(256, 7) march_table_kernel(TableMarchArgs) {
  const TableMarchArgs& a = table_args();
  march_table_body<true, true>(a.g, a.mk, a.tabs, a.mt, a.modes, a.rec, a.wcount, a.waves_per_mode);
}

__global__ void __launch_bounds__(256) march_table_batch_kernel(TableMarchArgs) {
  const TableMarchArgs& a = table_args();
  march_table_body<false, false>(a.g, a.mk, a.tabs, a.mt, a.modes, a.rec, a.wcount, a.waves_per_mode);
}

// One workgroup per mode: running maximum of live arrival heights (search
// keys), the first grid point at or above each key, the fold test (live
// arrivals must increase strictly), the per-tile search windows and the
// mode's ray counts.  Each thread takes `run` consecutive rays (run =
// ceil(R / 128), at most 9; longer ray sets are taken in several chunks):
// the thread's maximum, a workgroup exclusive prefix maximum over threads
// plus the carry of the previous chunk, then the thread's keys in order.
//
// Ray r owns the grid points [ci_r, ci_{r+1}), ci_r = smallest m in [0, N]
// with z_m >= key_r (N + 1 if none; 0 for an empty key): those are the
// points whose largest r' with key_{r'} <= z_m is r.  Tile t (first point
// 64 t) therefore starts in the interval of ray r - 1 for
// ceil(ci_{r-1} / 64) <= t < ceil(ci_r / 64) (ci_{-1} = 0), and tiles at or
// above ceil(ci_{R-1} / 64) in that of ray R - 1.
// 128 threads with up to 9 rays each: the per-wavefront prefix and count
// work is spread over more rays (random medium, 1091 rays per mode: 18.3 ->
// 16.4 us per screen against 256 threads with 5 rays; 64 threads with 18:
// 19.8 us)
constexpr int kScanThreads = 128;
constexpr int kScanRun = 9;  // most consecutive rays per thread

template <typename T>
__global__ void __launch_bounds__(kScanThreads) scan_kernel(Geometry g, DevRecords rec,
                                                            const int* __restrict__ wcount, int waves_per_mode) {
  // the chunk's rays staged in LDS so that global loads and stores stay
  // coalesced: sA, sD (T) and sC, sI (int) of kScanThreads * run entries each,
  // sized by the launch (scan_lds_bytes) so that as many workgroups as
  // possible are resident at once
  extern __shared__ double scan_lds[];
  __shared__ double wtot[kScanThreads / 64];
  __shared__ int wci[kScanThreads / 64];
  __shared__ int sfold;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = blockIdx.x;
  const size_t base = (size_t)j * g.R;
  int* __restrict__ ts = rec.tstart + (size_t)j * (g.T + 1);
  const T* __restrict__ A = static_cast<const T*>(rec.A) + base;
  const T* __restrict__ D = static_cast<const T*>(rec.D) + base;
  const int* __restrict__ CZ = rec.cz + base;
  int run = (g.R + kScanThreads - 1) / kScanThreads;
  if (run > kScanRun) run = kScanRun;
  const int chunk = kScanThreads * run;
  T* sA = reinterpret_cast<T*>(scan_lds);
  T* sD = sA + chunk;
  int* sC = reinterpret_cast<int*>(sD + chunk);
  int* sI = sC + chunk;
  if (tid == 0) sfold = 0;
  // the mode's per-wavefront counts, loaded now so that their latency
  // overlaps the scan's
  int v[kWaveCounts] = {0, 0, 0, 0, 0, 0};
  if (tid < 64)
    for (int w = tid; w < waves_per_mode; w += 64)
      for (int k = 0; k < kWaveCounts; ++k) v[k] += wcount[kWaveCounts * ((size_t)j * waves_per_mode + w) + k];
  double carry = -INFINITY;  // key of the last ray before this chunk
  int carry_ci = 0;          // its first point
  bool fold = false;
  for (int c0 = 0; c0 < g.R; c0 += kScanThreads * run) {
    const int n = g.R - c0 < kScanThreads * run ? g.R - c0 : kScanThreads * run;
    for (int i = tid; i < n; i += kScanThreads) {
      sA[i] = A[c0 + i];
      sD[i] = D[c0 + i];
      sC[i] = CZ[c0 + i];
    }
    __syncthreads();
    const int l0 = tid * run;  // this thread's first ray in the chunk
    // the thread's rays: arrival height of live rays (-inf otherwise) and the
    // first grid point at or above it (computed by the march)
    double Z[kScanRun];
    int cz[kScanRun];
    double lmax = -INFINITY;
    int lci = 0;
#pragma unroll
    for (int i = 0; i < kScanRun; ++i) {
      const int l = l0 + i;
      const bool live = i < run && l < n && sA[l < n ? l : 0] > T(0);
      Z[i] = live ? (g.z_a + (double)((c0 + l) * g.rho - g.E) * g.h) + (double)sD[l] : -INFINITY;
      cz[i] = live ? sC[l] : 0;
      lmax = fmax(lmax, Z[i]);
      lci = cz[i] > lci ? cz[i] : lci;
    }
    // workgroup exclusive prefix maxima of (height, first point)
    double incl = lmax;
    int icl = lci;
    for (int off = 1; off < 64; off <<= 1) {
      const double v = __shfl_up(incl, off, 64);
      const int vi = __shfl_up(icl, off, 64);
      if (lane >= off) {
        incl = fmax(incl, v);
        icl = vi > icl ? vi : icl;
      }
    }
    if (lane == 63) {
      wtot[wv] = incl;
      wci[wv] = icl;
    }
    __syncthreads();
    double key = __shfl_up(incl, 1, 64);
    int ci = __shfl_up(icl, 1, 64);
    if (lane == 0) {
      key = -INFINITY;
      ci = 0;
    }
    for (int k = 0; k < wv; ++k) {
      key = fmax(key, wtot[k]);
      ci = wci[k] > ci ? wci[k] : ci;
    }
    key = fmax(carry, key);  // key of ray c0 + l0 - 1 and its first point
    ci = carry_ci > ci ? carry_ci : ci;
#pragma unroll
    for (int i = 0; i < kScanRun; ++i) {
      const int l = l0 + i;
      if (i < run && l < n) {
        if (Z[i] != -INFINITY && !(Z[i] > key)) fold = true;
        key = fmax(key, Z[i]);
        const int ci_prev = ci;
        ci = cz[i] > ci ? cz[i] : ci;
        sI[l] = ci;
        for (int t = (ci_prev + 63) >> 6; t < ((ci + 63) >> 6) && t <= g.T; ++t) ts[t] = c0 + l - 1;
      }
    }
    double tot = carry;
    int tci = carry_ci;
    for (int k = 0; k < kScanThreads / 64; ++k) {
      tot = fmax(tot, wtot[k]);
      tci = wci[k] > tci ? wci[k] : tci;
    }
    __syncthreads();  // sI complete; wtot, wci are rewritten by the next chunk
    for (int i = tid; i < n; i += kScanThreads) rec.cidx[base + c0 + i] = sI[i];
    carry = tot;
    carry_ci = tci;
    __syncthreads();  // the staging arrays are refilled by the next chunk
  }
  // the last ray of the mode is R - 1: carry holds its key, carry_ci its first point
  for (int t = ((carry_ci + 63) >> 6) + tid; t <= g.T; t += kScanThreads) ts[t] = g.R - 1;
  if (fold) sfold = 1;
  // counts
  if (tid < 64) {
    for (int k = 0; k < kWaveCounts; ++k) v[k] = (int)__ockl_wfred_add_u32((unsigned)v[k]);
    if (tid == 0) {
      rec.mcaus[j] = v[0];
      rec.mdead[j] = v[1];
      rec.mwork[4 * j] = v[2];
      rec.mwork[4 * j + 1] = v[3];
      rec.mwork[4 * j + 2] = v[4];
      rec.mwork[4 * j + 3] = v[5];
    }
  }
  __syncthreads();
  if (tid == 0) rec.mflag[j] = (sfold ? 1 : 0) | (rec.mcaus[j] > 0 ? 2 : 0) | (rec.mdead[j] >= g.R ? 4 : 0);
}

// Full records in FP64 for the stage entry point.
template <typename T>
__global__ void export_kernel(Geometry g, DevModes modes, DevRecords rec, double* __restrict__ Z,
                              double* __restrict__ psi, double* __restrict__ qz, double* __restrict__ amp,
                              int* __restrict__ flag, double z0p) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)g.M * g.R) return;
  const int j = (int)(i / g.R), r = (int)(i - (size_t)j * g.R);
  const double xi = modes.xi[j];
  const double s = g.z_a + (double)(r * g.rho - g.E) * g.h;
  const double zz = s + (double)static_cast<const T*>(rec.D)[i];
  const double a = (double)static_cast<const T*>(rec.A)[i];
  Z[i] = zz;
  psi[i] = xi * (zz - z0p) + modes.pbar[j] * g.dx + (double)static_cast<const T*>(rec.Pp)[i];
  qz[i] = xi + (double)static_cast<const T*>(rec.G)[i];
  amp[i] = a > 0.0 ? a : 0.0;
  flag[i] = a > 0.0 ? 0 : (int)(-a);
}

DevMedium medium_for(const swkb_plan_s& pl, int q) {
  DevMedium md;
  md.kind = pl.p.medium_kind;
  md.mirror = pl.g.bc != SWKB_BC_PERIODIC;
  md.z_a = pl.g.z_a;
  md.prm = pl.mprm;
  md.list = nullptr;
  md.nlist = 0;
  if (md.kind == SWKB_MEDIUM_GAUSSSUM) {
    md.list = pl.glist + pl.goff[q];
    md.nlist = pl.goff[q + 1] - pl.goff[q];
  }
  return md;
}

DevModes modes_of(const swkb_plan_s& pl) {
  DevModes m;
  m.xi = pl.xi;
  m.pbar = pl.pbar;
  m.e1r = pl.e1r;
  m.frac = pl.frac;
  return m;
}

}  // namespace

int waves_per_mode(const Geometry& g) { return (g.R + 63) / 64; }

static hipError_t launch_march_rays(const swkb_plan_s& pl, int q, hipStream_t st) {
  const Geometry& g = pl.g;
  const int wpm = waves_per_mode(g);
  const long long waves = (long long)wpm * g.M;
  const dim3 grid((unsigned)((waves + 3) / 4));
  // the FP32 Gaussian-sum marches share tail wavefronts between modes
  const dim3 pgrid((unsigned)((packed_march_waves(g) + 3) / 4));
  const double x_q = pl.p.x0 + q * pl.p.dx;
  int* wcount = pl.wcount;
  MarchK mk;
  mk.hx = g.dx / g.S;
  mk.h6 = mk.hx / 6.0;
  mk.inv_h = 1.0 / g.h;
  mk.inv_dzt = pl.mtab.tab ? 1.0 / pl.mtab.dz : 0.0;
  mk.inv_dz = (float)mk.inv_dzt;
  mk.half_inv_dz = pl.mtab.tab ? (float)(0.5 / pl.mtab.dz) : 0.0f;
  mk.inv_dz2 = pl.mtab.tab ? (float)(1.0 / (pl.mtab.dz * pl.mtab.dz)) : 0.0f;
  mk.two_dz = (float)(2.0 * pl.mtab.dz);
  mk.dz_sq = (float)(pl.mtab.dz * pl.mtab.dz);
  if (pl.gfast) {
    const int nl = pl.goff[q + 1] - pl.goff[q];
    const size_t off = (size_t)pl.goff[q];
    const size_t nst = (size_t)(2 * pl.tab_S + 1);  // table stride per screen
    if (pl.precision == SWKB_FP64) {
      GaussTabs<double> t{reinterpret_cast<const T2<double>*>(pl.gstage) + off * nst,
                          reinterpret_cast<const T2<double>*>(pl.gterm) + off,
                          static_cast<const double*>(pl.gczl) + off * wpm, nl};
      hipLaunchKernelGGL(march_gauss_kernel<double>, grid, dim3(256), 0, st, g, mk, t, modes_of(pl), pl.rec,
                         wcount, wpm);
    } else if (pl.mtab.tab) {
      GaussTabs<float> t{reinterpret_cast<const T2<float>*>(pl.gstage) + off * nst,
                         reinterpret_cast<const T2<float>*>(pl.gterm) + off,
                         static_cast<const float*>(pl.gczl) + off * wpm, nl};
      // reads the table launch_medium_table built for screen q
      const TableMarchArgs a{g, mk, t, pl.mtab, modes_of(pl), pl.rec, wcount, wpm};
      if (pl.sum_fields > 1)
        hipLaunchKernelGGL(march_table_batch_kernel, grid, dim3(256), 0, st, a);
      else
        hipLaunchKernelGGL(march_table_kernel, pgrid, dim3(256), 0, st, a);
    } else {
      GaussTabs<float> t{reinterpret_cast<const T2<float>*>(pl.gstage) + off * nst,
                         reinterpret_cast<const T2<float>*>(pl.gterm) + off,
                         static_cast<const float*>(pl.gczl) + off * wpm, nl};
      hipLaunchKernelGGL(march_gauss_kernel<float>, pgrid, dim3(256), 0, st, g, mk, t, modes_of(pl), pl.rec,
                         wcount, wpm);
    }
    return hipGetLastError();
  }
  if (pl.precision == SWKB_FP64)
    hipLaunchKernelGGL(march_kernel<double>, grid, dim3(256), 0, st, g, mk, medium_for(pl, q), modes_of(pl),
                       pl.rec, wcount, x_q, wpm);
  else
    hipLaunchKernelGGL(march_kernel<float>, grid, dim3(256), 0, st, g, mk, medium_for(pl, q), modes_of(pl),
                       pl.rec, wcount, x_q, wpm);
  return hipGetLastError();
}

namespace {

// Launch amplitudes of a patch (Sec. 2.4: initial amplitude S^p(z) w_j / N):
// the transport factor of every live ray r of every mode times W[r]; a ray
// with W[r] = 0 lies outside the patch and is not launched (dead at launch).
template <typename T>
__global__ void launch_window_kernel(T* __restrict__ A, const double* __restrict__ W, int R, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = W[i % (size_t)R];
  const T a = A[i];
  if (w > 0.0) {
    if (a > T(0)) A[i] = (T)((double)a * w);
  } else if (a > T(0)) {
    A[i] = (T)(-kDeadLaunch);
  }
}

}  // namespace

hipError_t launch_march(const swkb_plan_s& pl, int q, hipStream_t st) {
  const hipError_t e = launch_march_rays(pl, q, st);
  if (e != hipSuccess || !pl.lwin) return e;
  const size_t n = (size_t)pl.g.M * pl.g.R;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (pl.precision == SWKB_FP64)
    hipLaunchKernelGGL(launch_window_kernel<double>, grid, dim3(256), 0, st, static_cast<double*>(pl.rec.A), pl.lwin,
                       pl.g.R, n);
  else
    hipLaunchKernelGGL(launch_window_kernel<float>, grid, dim3(256), 0, st, static_cast<float*>(pl.rec.A), pl.lwin,
                       pl.g.R, n);
  return hipGetLastError();
}

hipError_t launch_medium_table(const swkb_plan_s& pl, int q, hipStream_t st) {
  const MedTab& mt = pl.mtab;
  if (!mt.tab || !pl.gfast || pl.precision == SWKB_FP64) return hipSuccess;
  const int nl = pl.goff[q + 1] - pl.goff[q];
  const double x_q = pl.p.x0 + q * pl.p.dx, hx2 = 0.5 * pl.p.dx / pl.tab_S;
  const int ni = mt.n - 1;  // intervals; a block writes kTabNodes - 1 of them
  hipLaunchKernelGGL(medium_table_kernel, dim3((ni + kTabNodes - 2) / (kTabNodes - 1), 2 * pl.tab_S + 1),
                     dim3(kTabNodes), 0, st, pl.mprm, pl.glist + pl.goff[q], nl, x_q, hx2, mt.z_lo, mt.dz, ni,
                     const_cast<float4*>(mt.tab));
  return hipGetLastError();
}

// Dynamic LDS of the scan: four arrays of kScanThreads * run entries.
static size_t scan_lds_bytes(const Geometry& g, size_t tsize) {
  int run = (g.R + kScanThreads - 1) / kScanThreads;
  if (run > kScanRun) run = kScanRun;
  return (size_t)kScanThreads * run * (2 * tsize + 2 * sizeof(int));
}

hipError_t launch_scan(const swkb_plan_s& pl, hipStream_t st) {
  const Geometry& g = pl.g;
  const int wpm = waves_per_mode(g);
  const int* wcount = pl.wcount;
  if (pl.precision == SWKB_FP64)
    hipLaunchKernelGGL(scan_kernel<double>, dim3(g.M), dim3(kScanThreads), scan_lds_bytes(g, sizeof(double)), st, g,
                       pl.rec, wcount, wpm);
  else
    hipLaunchKernelGGL(scan_kernel<float>, dim3(g.M), dim3(kScanThreads), scan_lds_bytes(g, sizeof(float)), st, g,
                       pl.rec, wcount, wpm);
  return hipGetLastError();
}

hipError_t launch_export_rays(const swkb_plan_s& pl, int q, double* Z, double* psi, double* qz, double* amp,
                              int* flag, hipStream_t st) {
  (void)q;
  const Geometry& g = pl.g;
  const size_t n = (size_t)g.M * g.R;
  const double z0p = g.bc == SWKB_BC_PERIODIC ? g.z_a : g.z_a - (g.z_b - g.z_a);
  const dim3 grid((unsigned)((n + 255) / 256));
  if (pl.precision == SWKB_FP64)
    hipLaunchKernelGGL(export_kernel<double>, grid, dim3(256), 0, st, g, modes_of(pl), pl.rec, Z, psi, qz, amp,
                       flag, z0p);
  else
    hipLaunchKernelGGL(export_kernel<float>, grid, dim3(256), 0, st, g, modes_of(pl), pl.rec, Z, psi, qz, amp,
                       flag, z0p);
  return hipGetLastError();
}

}  // namespace swkb
