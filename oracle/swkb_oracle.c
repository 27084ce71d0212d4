/*
 * swkb_oracle.c -- plain FP64 CPU screened-WKB (S-WKB), the parity oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call this code; the GPU library never
 * links, loads or calls it, and the two share no source, header or table.
 *
 * What it computes (Bruno & Maas, "WKB across caustics: the screened-WKB
 * method"): the field on screen q+1 from the field on screen q, for the 2D
 * Helmholtz problem  Delta u + k^2 eps(x,z) u = 0  (Sec. 2, eq. helmholtz_3D),
 * by the steps of Algorithm 1 ("Screened WKB"), taken in the paper's order:
 *
 *   1. vertical DFT of the field on the screen (Sec. 2.1.1, eqs. fft_eq and
 *      ifft_eq; the 1/N of ifft_eq is folded into the mode amplitudes);
 *   2. per Fourier mode n, a plane wave with vertical slowness
 *      xi_n = 2 pi n / (k P h) (eq. fourier_psi and the initial conditions of
 *      Sec. 2.1.2), carried across the screen by WKB: rays of the
 *      characteristic system (Appendix A, eqs. charsys and charsys_s) for the
 *      eikonal phase psi and the transport amplitude A (eqs.
 *      first_order_system_1/2);
 *   3. interpolation of psi_n and A_n from the ray arrivals to the uniform grid
 *      of the next screen (Sec. 2.1.2, which leaves the scheme open);
 *   4. the sum over modes (eq. ray_bundle_q_plus_1), repeated per screen.
 *
 * Readings taken where the paper is silent or garbled (listed with reasons
 * in the design notes):
 *   - DFT phase origin z0' and normalisation: w_n = sum_m v_m e^{-2 pi i n m/P},
 *     amplitude of mode n = w_n / P; modes n in [-M/2, M/2).
 *   - Rays are marched in the range variable x instead of the ray parameter t
 *     (dt = dx / (2 psi_x); Sec. 2.1.2 allows any eikonal/transport solver),
 *     with S uniform RK4 steps so that every ray lands on x_{q+1}.  State
 *     (z, q = psi_z, psi, Z_s = dz/ds|_x, Q_s = dq/ds|_x); psi_x = p is
 *     eliminated by the eikonal p^2 = eps - q^2.
 *   - Amplitude: the Jacobian of Appendix A read as J = X_t Z_s - Z_t X_s
 *     with Delta Psi = J_t / (2J), so A = A0 sqrt(J0/J); in the x-march this
 *     is a = sqrt(p0 / (p Z_s)).
 *   - Launch set: s_r = z_a + (r rho - E) h, r = 0..R-1; rays whose
 *     p^2 <= p2_floor at launch or at any RK4 stage are dead, rays with
 *     Z_s <= 0 at any stage are caustic (dead and counted).
 *   - Interpolation: psi by cubic Hermite with slopes q (psi_z = q at fixed
 *     x), amplitude by 4-point Lagrange (linear when a neighbour is missing),
 *     between consecutive live rays; a mode whose live arrivals are not
 *     strictly increasing in z is folded and contributes nothing.
 *   - Ground mirror (Sec. 2.3): P = 2N, odd (Dirichlet) or even (Neumann)
 *     extension of the field about z_a and eps reflected about z_a.
 *   - Open ends: cos^2 taper of the field after each screen.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MEDIUM_LINEAR 0
#define OR_MEDIUM_EXPGAUSS 1
#define OR_MEDIUM_GAUSSSUM 2
#define OR_MEDIUM_MPROFILE 3

#define OR_BC_PERIODIC 0
#define OR_BC_DIRICHLET 1
#define OR_BC_NEUMANN 2

#define OR_RAY_LIVE 0
#define OR_RAY_DEAD_LAUNCH 1
#define OR_RAY_DEAD 2
#define OR_RAY_CAUSTIC 3

#define OR_ERR_ARG -1

/* Problem description; field meanings as in workloads/__init__.py. */
typedef struct {
  double k, z_a, z_b;
  int32_t n_z, n_modes;
  double x0, dx;
  int32_t n_screens, rk4_steps, ray_stride, launch_ext_cells;
  double p2_floor;
  int32_t bc;
  double absorber_bot, absorber_top;
  int32_t medium_kind, n_medium_params;
  const double* medium_params;
  double caustic_tol; /* a caustic/folded mode counts as significant when |c_n| > caustic_tol max|c| */
} or_params;

typedef struct {
  int64_t caustic_rays;  /* rays with Z_s <= 0 at some stage              */
  int64_t dead_rays;     /* rays dead at launch or on the way             */
  int64_t folded_modes;  /* modes whose live arrivals are not increasing  */
  int64_t significant;   /* caustic/folded modes with |c_n| > caustic_tol max|c| */
  int64_t evanescent_modes;       /* modes of which no ray arrived live       */
  int64_t significant_evanescent; /* of those, modes with |c_n| > caustic_tol max|c| */
} or_counters;

typedef struct { double z, q, psi, Zs, Qs; } ray_state;

/* ---------------------------------------------------------------- medium */

static double softplus(double y) { return y > 0.0 ? y + log1p(exp(-y)) : log1p(exp(y)); }

/* eps(x,z) and its z-derivatives for the un-reflected medium. */
static void medium_raw(const or_params* P, double x, double z, double* e, double* ez, double* ezz) {
  const double* m = P->medium_params;
  switch (P->medium_kind) {
    case OR_MEDIUM_LINEAR:
      *e = m[0] + m[1] * z;
      *ez = m[1];
      *ezz = 0.0;
      break;
    case OR_MEDIUM_EXPGAUSS: { /* eps = eps0 + a exp(-b (z - zc)^2), the paper's model of Sec. 3 */
      double d = z - m[3];
      double g = m[1] * exp(-m[2] * d * d);
      *e = m[0] + g;
      *ez = -2.0 * m[2] * d * g;
      *ezz = (4.0 * m[2] * m[2] * d * d - 2.0 * m[2]) * g;
      break;
    }
    case OR_MEDIUM_GAUSSSUM: { /* n = 1 + sum_j a_j exp(-r^2 / (2 s_j^2)), r^2 <= 64 s_j^2 */
      int ng = (int)m[0];
      double n = 1.0, nz = 0.0, nzz = 0.0;
      for (int j = 0; j < ng; ++j) {
        double a = m[1 + 4 * j], s = m[2 + 4 * j], cx = m[3 + 4 * j], cz = m[4 + 4 * j];
        double ddx = x - cx, ddz = z - cz;
        double r2 = ddx * ddx + ddz * ddz;
        if (r2 > 64.0 * s * s) continue;
        double g = a * exp(-r2 / (2.0 * s * s));
        n += g;
        nz += -ddz / (s * s) * g;
        nzz += (ddz * ddz / (s * s * s * s) - 1.0 / (s * s)) * g;
      }
      *e = n * n;
      *ez = 2.0 * n * nz;
      *ezz = 2.0 * (nz * nz + n * nzz);
      break;
    }
    case OR_MEDIUM_MPROFILE: { /* n = 1 + scale (M0 + g1 z + (g2-g1) w softplus((z-d)/w)) */
      double M0 = m[0], g1 = m[1], g2 = m[2], d = m[3], w = m[4], sc = m[5];
      double y = (z - d) / w;
      double sig = 1.0 / (1.0 + exp(-y));
      double M = M0 + g1 * z + (g2 - g1) * w * softplus(y);
      double Mz = g1 + (g2 - g1) * sig;
      double Mzz = (g2 - g1) * sig * (1.0 - sig) / w;
      double n = 1.0 + sc * M, nz = sc * Mz, nzz = sc * Mzz;
      *e = n * n;
      *ez = 2.0 * n * nz;
      *ezz = 2.0 * (nz * nz + n * nzz);
      break;
    }
    default:
      *e = NAN; *ez = NAN; *ezz = NAN;
  }
}

/* Medium seen by the rays: reflected about the ground z_a for the mirror
 * boundary conditions (Sec. 2.3, reflected permittivity). */
static void medium(const or_params* P, double x, double z, double* e, double* ez, double* ezz) {
  if (P->bc != OR_BC_PERIODIC && z < P->z_a) {
    medium_raw(P, x, 2.0 * P->z_a - z, e, ez, ezz);
    *ez = -*ez;
  } else {
    medium_raw(P, x, z, e, ez, ezz);
  }
}

/* ---------------------------------------------------------------- layout */

static int fft_len(const or_params* P) { return P->bc == OR_BC_PERIODIC ? P->n_z : 2 * P->n_z; }
static double grid_h(const or_params* P) { return (P->z_b - P->z_a) / P->n_z; }
/* DFT phase origin z0' = z_a (periodic) or z_a - L (mirror). */
static double phase_origin(const or_params* P) {
  return P->bc == OR_BC_PERIODIC ? P->z_a : P->z_a - (P->z_b - P->z_a);
}
int or_num_rays(const or_params* P) {
  int n = P->n_z, rho = P->ray_stride, e = P->launch_ext_cells;
  return (n + 2 * e + rho - 1) / rho + 1;
}
/* vertical slowness of mode index j (n = j - M/2): xi = 2 pi n / (k P h) */
static double mode_xi(const or_params* P, int j) {
  int n = j - P->n_modes / 2;
  return 2.0 * M_PI * n / (P->k * fft_len(P) * grid_h(P));
}

static int check(const or_params* P) {
  if (!P || !(P->k > 0) || !(P->z_b > P->z_a) || P->n_z < 4 || P->n_modes < 2 || (P->n_modes & 1)) return OR_ERR_ARG;
  if (P->n_modes > fft_len(P) || P->rk4_steps < 1 || P->ray_stride < 1 || P->launch_ext_cells < 0) return OR_ERR_ARG;
  if (P->bc < 0 || P->bc > 2 || P->medium_kind < 0 || P->medium_kind > 3 || !P->medium_params) return OR_ERR_ARG;
  return 0;
}

/* ------------------------------------------------------- step 1: the DFT */

/* The periodic vector v (length P) whose DFT gives the modes: v = u
 * (periodic), or the odd/even extension about z_a for the ground mirror:
 * v[N+m] = u[m], v[N-m] = -/+ u[m] (m = 1..N-1), v[0] = 0 (image of z_b,
 * which lies under the top absorber), v[N] = u[0] (0 for Dirichlet). */
static void extend(const or_params* P, const double* u, double* v) {
  int N = P->n_z;
  if (P->bc == OR_BC_PERIODIC) {
    memcpy(v, u, sizeof(double) * 2 * N);
    return;
  }
  double sgn = P->bc == OR_BC_DIRICHLET ? -1.0 : 1.0;
  for (int m = 0; m < N; ++m) {
    v[2 * (N + m)] = u[2 * m];
    v[2 * (N + m) + 1] = u[2 * m + 1];
  }
  for (int m = 1; m < N; ++m) {
    v[2 * (N - m)] = sgn * u[2 * m];
    v[2 * (N - m) + 1] = sgn * u[2 * m + 1];
  }
  v[0] = v[1] = 0.0;
  if (P->bc == OR_BC_DIRICHLET) v[2 * N] = v[2 * N + 1] = 0.0;
}

/* Mode amplitudes c_j = (1/P) sum_{m=0}^{P-1} v_m exp(-2 pi i n m / P),
 * n = j - M/2: the DFT written out (eq. fft_eq), the angle reduced exactly
 * through the integer (n m) mod P. */
int or_modes(const or_params* P, const double* u, double* c) {
  if (check(P)) return OR_ERR_ARG;
  int PP = fft_len(P), M = P->n_modes;
  double* v = (double*)malloc(sizeof(double) * 2 * PP);
  double* cs = (double*)malloc(sizeof(double) * 2 * PP);
  extend(P, u, v);
  for (int j = 0; j < PP; ++j) {
    cs[2 * j] = cos(2.0 * M_PI * j / PP);
    cs[2 * j + 1] = sin(2.0 * M_PI * j / PP);
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < M; ++j) {
    long long n = j - M / 2;
    double re = 0.0, im = 0.0;
    for (int m = 0; m < PP; ++m) {
      long long t = ((n * m) % PP + PP) % PP;
      double cr = cs[2 * t], ci = -cs[2 * t + 1];
      re += v[2 * m] * cr - v[2 * m + 1] * ci;
      im += v[2 * m] * ci + v[2 * m + 1] * cr;
    }
    c[2 * j] = re / PP;
    c[2 * j + 1] = im / PP;
  }
  free(v);
  free(cs);
  return 0;
}

/* --------------------------------------------- step 2: rays of one mode */

/* Right-hand side of the characteristic system (Appendix A, charsys and
 * its s-derivative charsys_s) rewritten with x as the independent variable
 * (dt = dx / (2p)):
 *   dz/dx = q/p,  dq/dx = eps_z/(2p),  dpsi/dx = eps/p,
 *   dZs/dx = (eps Qs - q eps_z Zs / 2) / p^3,
 *   dQs/dx = (eps_zz/(2p) - eps_z^2/(4p^3)) Zs + q eps_z/(2p^3) Qs,
 * with p = sqrt(eps - q^2) (the eikonal, eq. first_order_system_1). */
static int rhs(const or_params* P, double x, const ray_state* y, ray_state* d) {
  if (y->Zs <= 0.0) return OR_RAY_CAUSTIC;
  double e, ez, ezz;
  medium(P, x, y->z, &e, &ez, &ezz);
  double p2 = e - y->q * y->q;
  if (!(p2 > P->p2_floor)) return OR_RAY_DEAD;
  double p = sqrt(p2);
  double p3 = p2 * p;
  d->z = y->q / p;
  d->q = ez / (2.0 * p);
  d->psi = e / p;
  d->Zs = (e * y->Qs - 0.5 * y->q * ez * y->Zs) / p3;
  d->Qs = (ezz / (2.0 * p) - ez * ez / (4.0 * p3)) * y->Zs + (y->q * ez / (2.0 * p3)) * y->Qs;
  return OR_RAY_LIVE;
}

static void axpy(ray_state* o, const ray_state* y, double h, const ray_state* d) {
  o->z = y->z + h * d->z;
  o->q = y->q + h * d->q;
  o->psi = y->psi + h * d->psi;
  o->Zs = y->Zs + h * d->Zs;
  o->Qs = y->Qs + h * d->Qs;
}

/* March all R rays of mode j across the screen [x_q, x_q + dx] with S
 * classical RK4 steps.  Initial conditions per ray (Sec. 2.1.2 and the
 * variational ICs Z_s = 1, Q_s = 0): z = s_r, q = xi_n,
 * psi = xi_n (s_r - z0'), p0 = sqrt(eps(x_q, s_r) - xi_n^2).
 * Arrival: Z, psi, q and a = sqrt(p0 / (p Z_s)).  flag: OR_RAY_*. */
int or_march_mode(const or_params* P, double x_q, int j, double* Z, double* psi, double* q,
                  double* amp, int32_t* flag) {
  if (check(P) || j < 0 || j >= P->n_modes) return OR_ERR_ARG;
  int R = or_num_rays(P), S = P->rk4_steps;
  double h = grid_h(P), xi = mode_xi(P, j), z0p = phase_origin(P);
  double dxs = P->dx / S;
  for (int r = 0; r < R; ++r) {
    double s = P->z_a + (double)(r * P->ray_stride - P->launch_ext_cells) * h;
    double e, ez, ezz;
    medium(P, x_q, s, &e, &ez, &ezz);
    double p02 = e - xi * xi;
    Z[r] = s; psi[r] = xi * (s - z0p); q[r] = xi; amp[r] = 0.0;
    if (!(p02 > P->p2_floor)) { flag[r] = OR_RAY_DEAD_LAUNCH; continue; }
    double p0 = sqrt(p02);
    ray_state y = {s, xi, xi * (s - z0p), 1.0, 0.0}, k1, k2, k3, k4, t;
    int st = OR_RAY_LIVE;
    for (int i = 0; i < S && st == OR_RAY_LIVE; ++i) {
      double x = x_q + i * dxs;
      if ((st = rhs(P, x, &y, &k1))) break;
      axpy(&t, &y, 0.5 * dxs, &k1);
      if ((st = rhs(P, x + 0.5 * dxs, &t, &k2))) break;
      axpy(&t, &y, 0.5 * dxs, &k2);
      if ((st = rhs(P, x + 0.5 * dxs, &t, &k3))) break;
      axpy(&t, &y, dxs, &k3);
      if ((st = rhs(P, x + dxs, &t, &k4))) break;
      y.z += dxs / 6.0 * (k1.z + 2.0 * k2.z + 2.0 * k3.z + k4.z);
      y.q += dxs / 6.0 * (k1.q + 2.0 * k2.q + 2.0 * k3.q + k4.q);
      y.psi += dxs / 6.0 * (k1.psi + 2.0 * k2.psi + 2.0 * k3.psi + k4.psi);
      y.Zs += dxs / 6.0 * (k1.Zs + 2.0 * k2.Zs + 2.0 * k3.Zs + k4.Zs);
      y.Qs += dxs / 6.0 * (k1.Qs + 2.0 * k2.Qs + 2.0 * k3.Qs + k4.Qs);
    }
    if (st == OR_RAY_LIVE) {
      if (y.Zs <= 0.0) {
        st = OR_RAY_CAUSTIC;
      } else {
        medium(P, x_q + P->dx, y.z, &e, &ez, &ezz);
        double p2 = e - y.q * y.q;
        if (!(p2 > P->p2_floor)) st = OR_RAY_DEAD;
        else amp[r] = sqrt(p0 / (sqrt(p2) * y.Zs));
      }
    }
    Z[r] = y.z; psi[r] = y.psi; q[r] = y.q;
    flag[r] = st;
  }
  return 0;
}

/* --------------------------------- step 3: interpolation onto the grid */

/* A mode is folded when its live arrivals are not strictly increasing in z. */
static int folded(int R, const double* Z, const int32_t* flag) {
  int have = 0;
  double last = 0.0;
  for (int r = 0; r < R; ++r) {
    if (flag[r] != OR_RAY_LIVE) continue;
    if (have && !(Z[r] > last)) return 1;
    last = Z[r];
    have = 1;
  }
  return 0;
}

/* Search keys: the running maximum of live arrivals (minus infinity before
 * the first live ray), non-decreasing by construction. */
static void search_keys(int R, const double* Z, const int32_t* flag, double* key) {
  double run = -INFINITY;
  for (int r = 0; r < R; ++r) {
    if (flag[r] == OR_RAY_LIVE) run = Z[r];
    key[r] = run;
  }
}

/* psi and a of one mode at height z.  The bracket is the largest r with
 * key_r <= z; it contributes only if rays r and r+1 are both live.
 * psi: cubic Hermite with end slopes q_r, q_{r+1}.  a: Lagrange through
 * r-1..r+2 when all four are live, else linear through r, r+1.
 * Returns 0 where the mode has no bracket. */
static int interp_at(int R, const double* Z, const double* psi, const double* q, const double* amp,
                     const int32_t* flag, const double* key, double z, double* out_psi, double* out_a) {
  if (R < 2 || !(key[0] <= z)) return 0;
  int lo = 0, hi = R - 1; /* key[lo] <= z; find largest such index */
  if (key[hi] <= z) lo = hi;
  else {
    while (hi - lo > 1) {
      int mid = (lo + hi) / 2;
      if (key[mid] <= z) lo = mid; else hi = mid;
    }
  }
  int r = lo;
  if (r >= R - 1 || flag[r] != OR_RAY_LIVE || flag[r + 1] != OR_RAY_LIVE) return 0;
  double H = Z[r + 1] - Z[r];
  double t = (z - Z[r]) / H;
  double t2 = t * t, t3 = t2 * t;
  double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t, h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
  *out_psi = h00 * psi[r] + h10 * H * q[r] + h01 * psi[r + 1] + h11 * H * q[r + 1];
  if (r >= 1 && r + 2 < R && flag[r - 1] == OR_RAY_LIVE && flag[r + 2] == OR_RAY_LIVE) {
    double x0 = Z[r - 1], x1 = Z[r], x2 = Z[r + 1], x3 = Z[r + 2];
    double l0 = (z - x1) * (z - x2) * (z - x3) / ((x0 - x1) * (x0 - x2) * (x0 - x3));
    double l1 = (z - x0) * (z - x2) * (z - x3) / ((x1 - x0) * (x1 - x2) * (x1 - x3));
    double l2 = (z - x0) * (z - x1) * (z - x3) / ((x2 - x0) * (x2 - x1) * (x2 - x3));
    double l3 = (z - x0) * (z - x1) * (z - x2) / ((x3 - x0) * (x3 - x1) * (x3 - x2));
    *out_a = l0 * amp[r - 1] + l1 * amp[r] + l2 * amp[r + 1] + l3 * amp[r + 2];
  } else {
    *out_a = (1.0 - t) * amp[r] + t * amp[r + 1];
  }
  return 1;
}

/* Interpolate one mode's records onto n points (for unit tests). */
int or_interp(int R, const double* Z, const double* psi, const double* q, const double* amp,
              const int32_t* flag, int n, const double* z, double* out_psi, double* out_a, int32_t* has) {
  double* key = (double*)malloc(sizeof(double) * (R > 0 ? R : 1));
  int fold = folded(R, Z, flag);
  search_keys(R, Z, flag, key);
  for (int i = 0; i < n; ++i) {
    out_psi[i] = 0.0; out_a[i] = 0.0;
    has[i] = fold ? 0 : interp_at(R, Z, psi, q, amp, flag, key, z[i], &out_psi[i], &out_a[i]);
  }
  free(key);
  return fold;
}

/* ----------------------------------------- one screen: steps 1 through 4 */

/* Absorbing taper W(z): cos^2(pi/2 d/D) inside a layer of thickness D at an
 * open end, d the depth into the layer; 1 elsewhere. */
static double taper(const or_params* P, double z) {
  double w = 1.0;
  if (P->absorber_bot > 0.0 && z < P->z_a + P->absorber_bot) {
    double d = (P->z_a + P->absorber_bot - z) / P->absorber_bot;
    double c = cos(0.5 * M_PI * d);
    w *= c * c;
  }
  if (P->absorber_top > 0.0 && z > P->z_b - P->absorber_top) {
    double d = (z - (P->z_b - P->absorber_top)) / P->absorber_top;
    double c = cos(0.5 * M_PI * d);
    w *= c * c;
  }
  return w;
}

/* u_out (screen q+1) from u_in (screen q). */
int or_screen(const or_params* P, int q, const double* u_in, double* u_out, or_counters* cnt) {
  if (check(P)) return OR_ERR_ARG;
  int N = P->n_z, M = P->n_modes, R = or_num_rays(P);
  double h = grid_h(P), x_q = P->x0 + q * P->dx, k = P->k;
  double* c = (double*)malloc(sizeof(double) * 2 * M);
  or_modes(P, u_in, c);
  size_t MR = (size_t)M * R;
  double* Z = (double*)malloc(sizeof(double) * MR);
  double* psi = (double*)malloc(sizeof(double) * MR);
  double* qq = (double*)malloc(sizeof(double) * MR);
  double* amp = (double*)malloc(sizeof(double) * MR);
  double* key = (double*)malloc(sizeof(double) * MR);
  int32_t* flag = (int32_t*)malloc(sizeof(int32_t) * MR);
  int32_t* fold = (int32_t*)malloc(sizeof(int32_t) * M);
  int32_t* caus = (int32_t*)malloc(sizeof(int32_t) * M);
  int32_t* nolive = (int32_t*)malloc(sizeof(int32_t) * M);
  int64_t n_caustic = 0, n_dead = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : n_caustic, n_dead)
  for (int j = 0; j < M; ++j) {
    size_t o = (size_t)j * R;
    or_march_mode(P, x_q, j, Z + o, psi + o, qq + o, amp + o, flag + o);
    fold[j] = folded(R, Z + o, flag + o);
    search_keys(R, Z + o, flag + o, key + o);
    caus[j] = fold[j];
    int dead_here = 0;
    for (int r = 0; r < R; ++r) {
      if (flag[o + r] == OR_RAY_CAUSTIC) { ++n_caustic; caus[j] = 1; }
      if (flag[o + r] == OR_RAY_DEAD || flag[o + r] == OR_RAY_DEAD_LAUNCH) { ++n_dead; ++dead_here; }
    }
    nolive[j] = dead_here == R; /* every ray evanescent: the mode carries nothing across */
  }
  if (cnt) {
    double cmax = 0.0;
    for (int j = 0; j < M; ++j) cmax = fmax(cmax, hypot(c[2 * j], c[2 * j + 1]));
    cnt->caustic_rays += n_caustic;
    cnt->dead_rays += n_dead;
    for (int j = 0; j < M; ++j) {
      cnt->folded_modes += fold[j];
      if (caus[j] && hypot(c[2 * j], c[2 * j + 1]) > P->caustic_tol * cmax) cnt->significant++;
      cnt->evanescent_modes += nolive[j];
      if (nolive[j] && hypot(c[2 * j], c[2 * j + 1]) > P->caustic_tol * cmax) cnt->significant_evanescent++;
    }
  }
  /* step 4: u'(z_m) = sum_n c_n a_n(z_m) exp(i k psi_n(z_m)), summed in mode order */
#pragma omp parallel for schedule(static)
  for (int m = 0; m < N; ++m) {
    double z = P->z_a + m * h;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < M; ++j) {
      if (fold[j]) continue;
      size_t o = (size_t)j * R;
      double ps, a;
      if (!interp_at(R, Z + o, psi + o, qq + o, amp + o, flag + o, key + o, z, &ps, &a)) continue;
      double ph = k * ps;
      double er = a * cos(ph), ei = a * sin(ph);
      re += c[2 * j] * er - c[2 * j + 1] * ei;
      im += c[2 * j] * ei + c[2 * j + 1] * er;
    }
    double w = taper(P, z);
    u_out[2 * m] = w * re;
    u_out[2 * m + 1] = w * im;
  }
  free(c); free(Z); free(psi); free(qq); free(amp); free(key); free(flag); free(fold); free(caus); free(nolive);
  return 0;
}

/* Screens q_begin .. q_end-1: hist[(q - q_begin) * N] receives u on screen q+1. */
int or_run(const or_params* P, const double* u0, int q_begin, int q_end, double* hist, or_counters* cnt) {
  if (check(P) || q_end < q_begin) return OR_ERR_ARG;
  int N = P->n_z;
  const double* cur = u0;
  for (int q = q_begin; q < q_end; ++q) {
    double* out = hist + (size_t)(q - q_begin) * 2 * N;
    or_screen(P, q, cur, out, cnt);
    cur = out;
  }
  return 0;
}

/* The exit taper alone: u (N complex values on the grid z_a + m h) times
 * W(z_m), as applied at the end of a screen step. */
int or_taper(const or_params* P, double* u) {
  if (check(P)) return OR_ERR_ARG;
  double h = grid_h(P);
  for (int m = 0; m < P->n_z; ++m) {
    double w = taper(P, P->z_a + m * h);
    u[2 * m] *= w;
    u[2 * m + 1] *= w;
  }
  return 0;
}

/* Medium evaluation as the rays see it (for unit tests). */
int or_medium(const or_params* P, int n, const double* x, const double* z, double* e, double* ez, double* ezz) {
  if (check(P)) return OR_ERR_ARG;
  for (int i = 0; i < n; ++i) medium(P, x[i], z[i], &e[i], &ez[i], &ezz[i]);
  return 0;
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
