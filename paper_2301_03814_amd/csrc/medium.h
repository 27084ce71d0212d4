// Device evaluation of the medium seen by the rays: eps - 1, eps_z / 2 and
// eps_zz / 2 at (x, z), z = s + dz with s the ray's launch height (the ray
// system uses the derivatives only halved).
//
// T = double: everything in FP64.
// T = float : the small deviation dz and the medium are evaluated in FP32,
//             with the large coordinates (x, s, centres) differenced in FP64
//             first so that no FP32 quantity carries an absolute coordinate.
//
// The ground mirror reflects eps about z_a (Sec. 2.3): eps~(z) = eps(2 z_a - z)
// for z < z_a, so eps_z changes sign there.
#pragma once

#include "swkb_internal.h"

namespace swkb {

template <typename T>
struct Med {
  T e1, hz, hzz;  // eps - 1, (d eps / dz) / 2, (d^2 eps / dz^2) / 2
};

template <typename T>
__device__ inline T dev_exp(T x);
template <>
__device__ inline double dev_exp<double>(double x) { return exp(x); }
template <>
__device__ inline float dev_exp<float>(float x) { return __expf(x); }

template <typename T>
__device__ inline T dev_log1p(T x);
template <>
__device__ inline double dev_log1p<double>(double x) { return log1p(x); }
template <>
__device__ inline float dev_log1p<float>(float x) { return log1pf(x); }

// Refractive-index deviation dn = n - 1 and its z-derivatives -> eps terms.
template <typename T>
__device__ inline Med<T> from_index(T dn, T nz, T nzz) {
  const T n = T(1) + dn;
  Med<T> m;
  m.e1 = dn * (T(2) + dn);
  m.hz = n * nz;
  m.hzz = nz * nz + n * nzz;
  return m;
}

// zrel = z - zref with zref a coordinate given in FP64 (exact difference
// first, then the small deviation dz added in T).
template <typename T>
__device__ inline T rel(double s, double zref, T dz) {
  return (T)(s - zref) + dz;
}

// nterms is incremented by the number of Gaussian terms evaluated inside
// their cutoff (work accounting only).
template <typename T>
__device__ inline Med<T> medium_eval(const DevMedium& md, double x, double s, T dz, int& nterms) {
  // reflection about the ground
  bool flip = false;
  if (md.mirror) {
    const T zr = rel<T>(s, md.z_a, dz);
    if (zr < T(0)) {
      flip = true;
      // reflected height 2 z_a - z: deviation relative to 2 z_a - s is -dz
      s = 2.0 * md.z_a - s;
      dz = -dz;
    }
  }
  const double* p = md.prm;
  Med<T> m;
  switch (md.kind) {
    case SWKB_MEDIUM_LINEAR: {
      // eps - 1 = (eps0 - 1) + g z
      const T g = (T)p[1];
      m.e1 = (T)((p[0] - 1.0) + p[1] * s) + g * dz;
      m.hz = T(0.5) * g;
      m.hzz = T(0);
      break;
    }
    case SWKB_MEDIUM_EXPGAUSS: {
      const T a = (T)p[1], b = (T)p[2];
      const T d = rel<T>(s, p[3], dz);
      const T gg = a * dev_exp<T>(-b * d * d);
      m.e1 = (T)(p[0] - 1.0) + gg;
      m.hz = -b * d * gg;
      m.hzz = (T(2) * b * b * d * d - b) * gg;
      break;
    }
    case SWKB_MEDIUM_GAUSSSUM: {
      T dn = T(0), nz = T(0), nzz = T(0);
      for (int i = 0; i < md.nlist; ++i) {
        const int j = md.list[i];
        const double* q = p + 1 + 4 * j;
        const T a = (T)q[0], sg = (T)q[1];
        const T ddx = (T)(x - q[2]);
        const T ddz = rel<T>(s, q[3], dz);
        const T r2 = ddx * ddx + ddz * ddz;
        const T s2 = sg * sg;
        if (r2 > T(64) * s2) continue;
        ++nterms;
        const T is2 = T(1) / s2;
        const T gg = a * dev_exp<T>(-r2 * T(0.5) * is2);
        dn += gg;
        nz -= ddz * is2 * gg;
        nzz += (ddz * ddz * is2 - T(1)) * is2 * gg;
      }
      m = from_index<T>(dn, nz, nzz);
      break;
    }
    default: {  // SWKB_MEDIUM_MPROFILE
      const double M0 = p[0], g1 = p[1], g2 = p[2], d = p[3], w = p[4], sc = p[5];
      const T y = rel<T>(s, d, dz) / (T)w;
      const T ey = dev_exp<T>(-(y > T(0) ? y : -y));
      const T sp = (y > T(0) ? y : T(0)) + dev_log1p<T>(ey);  // log(1 + e^y)
      const T sig = y > T(0) ? T(1) / (T(1) + ey) : ey / (T(1) + ey);
      const T dg = (T)(g2 - g1);
      // n - 1 = sc M, M = M0 + g1 z + (g2 - g1) w softplus(y)
      const T Mv = (T)(M0 + g1 * s) + (T)g1 * dz + dg * (T)w * sp;
      const T dn = (T)sc * Mv;
      const T nz = (T)sc * ((T)g1 + dg * sig);
      const T nzz = (T)sc * dg * sig * (T(1) - sig) / (T)w;
      m = from_index<T>(dn, nz, nzz);
      break;
    }
  }
  if (flip) m.hz = -m.hz;
  return m;
}

}  // namespace swkb
