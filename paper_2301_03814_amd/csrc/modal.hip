// Separation-of-variables reference for media that do not depend on x (the
// paper's reference method, Sec. 3.1, eqs. series_sol, phi_equation,
// series_init, sl_expansion):
//   u(x, z) = sum_i a_i e^{i alpha_i x} phi_i(z),
//   phi_i'' + k^2 eps phi_i = alpha_i^2 phi_i,   a = projections of u0.
// The Sturm-Liouville operator is discretised Fourier-spectrally on the
// screen grid (periodic), or on the doubled grid of the ground mirror with
// eps reflected about z_a and the field extended oddly (Dirichlet) or evenly
// (Neumann), and diagonalised as a dense symmetric matrix with rocSOLVER
// (dsyevd, FP64).  Eigenvectors are orthonormal, so a = Phi^T u0; modes with
// alpha_i^2 < 0 decay as e^{-sqrt(-alpha_i^2) x}.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cmath>
#include <string>

#include "medium.h"

namespace swkb {
namespace {

// A[i][j] = D2[i][j] + k^2 eps(z_i) delta_ij with the periodic Fourier-
// spectral second derivative on P points of spacing h (domain P h):
//   D2_jj = -(pi/h)^2/3 - (2 pi/(P h))^2/6,
//   D2_ij = -(-1)^(i-j) 2 (pi/(P h))^2 / sin^2(pi (i-j)/P)   (i != j).
__global__ void operator_kernel(double* __restrict__ A, int P, double h, double k2, DevMedium md, double z0) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  double v;
  if (i == j) {
    const double L = P * h;
    v = -(M_PI / h) * (M_PI / h) / 3.0 - (2.0 * M_PI / L) * (2.0 * M_PI / L) / 6.0;
    int nt = 0;
    const Med<double> m = medium_eval<double>(md, 0.0, z0 + (double)i * h, 0.0, nt);
    v += k2 * (1.0 + m.e1);
  } else {
    const int d = i - j;
    const double s = sinpi((double)d / (double)P);
    const double f = M_PI / (P * h);
    v = ((d & 1) ? 1.0 : -1.0) * 2.0 * f * f / (s * s);
  }
  A[(size_t)j * P + i] = v;  // column-major, symmetric
}

// w = a .* e^{i alpha x}, alpha = sqrt(lambda) (decaying branch when lambda < 0).
__global__ void phase_kernel(const double2* __restrict__ a, const double* __restrict__ lam, double x,
                             double2* __restrict__ w, int P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const double l = lam[i];
  double er, ei;
  if (l >= 0.0) {
    double s, c;
    sincos(sqrt(l) * x, &s, &c);
    er = c;
    ei = s;
  } else {
    er = exp(-sqrt(-l) * x);
    ei = 0.0;
  }
  const double2 v = a[i];
  w[i] = make_double2(v.x * er - v.y * ei, v.x * ei + v.y * er);
}

// Extended initial field on the P-point grid (periodic: u itself; mirror:
// v[N+m] = u[m], v[N-m] = -/+ u[m], v[0] = 0, v[N] = 0 for Dirichlet).
__global__ void extend_kernel(const double2* __restrict__ u, double2* __restrict__ v, int N, int bc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int P = bc == SWKB_BC_PERIODIC ? N : 2 * N;
  if (i >= P) return;
  double2 x;
  if (bc == SWKB_BC_PERIODIC) x = u[i];
  else if (i > N) x = u[i - N];
  else if (i == N) x = bc == SWKB_BC_DIRICHLET ? make_double2(0.0, 0.0) : u[0];
  else if (i == 0) x = make_double2(0.0, 0.0);
  else {
    const double2 y = u[N - i];
    x = bc == SWKB_BC_DIRICHLET ? make_double2(-y.x, -y.y) : y;
  }
  v[i] = x;
}

}  // namespace
}  // namespace swkb

using namespace swkb;

extern "C" swkb_status swkb_modal_reference(const swkb_params* p, const void* u0, const double* xs, int32_t nx,
                                            void* out, void* hip_stream) {
  const size_t need = swkb_workspace_bytes(p);
  if (need == 0) {
    set_error("invalid parameters");
    return SWKB_ERR_ARG;
  }
  if (!u0 || !xs || !out || nx < 1) {
    set_error("NULL argument or nx < 1");
    return SWKB_ERR_ARG;
  }
  if (p->medium_kind == SWKB_MEDIUM_GAUSSSUM) {
    set_error("separation of variables needs a medium that does not depend on x");
    return SWKB_ERR_ARG;
  }
  const int N = p->n_z, bc = p->bc;
  const int P = bc == SWKB_BC_PERIODIC ? N : 2 * N;
  if (P > 16384) {
    set_error("modal reference limited to P <= 16384 grid points");
    return SWKB_ERR_ARG;
  }
  const double h = (p->z_b - p->z_a) / N;
  const double z0 = bc == SWKB_BC_PERIODIC ? p->z_a : p->z_a - (p->z_b - p->z_a);
  hipStream_t st = (hipStream_t)hip_stream;
  double *A = nullptr, *lam = nullptr, *E = nullptr, *mp = nullptr;
  double2 *v = nullptr, *a = nullptr, *w = nullptr, *o = nullptr;
  int* info = nullptr;
  rocblas_handle hb = nullptr;
  swkb_status ret = SWKB_OK;
  std::string why;
  auto ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && ret == SWKB_OK) {
      ret = SWKB_ERR_DEVICE;
      why = std::string(what) + ": " + hipGetErrorString(e);
    }
    return ret == SWKB_OK;
  };
  auto okb = [&](rocblas_status s, const char* what) {
    if (s != rocblas_status_success && ret == SWKB_OK) {
      ret = SWKB_ERR_DEVICE;
      why = std::string(what) + " failed";
    }
    return ret == SWKB_OK;
  };
  const size_t PP = (size_t)P * P;
  if (ok(hipMalloc(&A, sizeof(double) * PP), "hipMalloc") && ok(hipMalloc(&lam, sizeof(double) * P), "hipMalloc") &&
      ok(hipMalloc(&E, sizeof(double) * P), "hipMalloc") &&
      ok(hipMalloc(&mp, sizeof(double) * (p->n_medium_params + 1)), "hipMalloc") &&
      ok(hipMalloc(&v, sizeof(double2) * P), "hipMalloc") && ok(hipMalloc(&a, sizeof(double2) * P), "hipMalloc") &&
      ok(hipMalloc(&w, sizeof(double2) * P), "hipMalloc") && ok(hipMalloc(&o, sizeof(double2) * P), "hipMalloc") &&
      ok(hipMalloc(&info, sizeof(int)), "hipMalloc") &&
      ok(hipMemcpyAsync(mp, p->medium_params, sizeof(double) * p->n_medium_params, hipMemcpyHostToDevice, st),
         "copy") &&
      okb(rocblas_create_handle(&hb), "rocblas_create_handle") && okb(rocblas_set_stream(hb, st), "set_stream")) {
    DevMedium md;
    md.kind = p->medium_kind;
    md.mirror = bc != SWKB_BC_PERIODIC;
    md.z_a = p->z_a;
    md.prm = mp;
    md.list = nullptr;
    md.nlist = 0;
    hipLaunchKernelGGL(operator_kernel, dim3((P + 255) / 256, P), dim3(256), 0, st, A, P, h, p->k * p->k, md, z0);
    ok(hipGetLastError(), "operator");
    if (okb(rocsolver_dsyevd(hb, rocblas_evect_original, rocblas_fill_upper, P, A, P, lam, E, info), "dsyevd")) {
      hipLaunchKernelGGL(extend_kernel, dim3((P + 255) / 256), dim3(256), 0, st, static_cast<const double2*>(u0), v,
                         N, bc);
      ok(hipGetLastError(), "extend");
      // a^T (2 x P) = v^T (2 x P) * Phi (P x P): projections of the initial field
      const double one = 1.0, zero = 0.0;
      okb(rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_none, 2, P, P, &one,
                        reinterpret_cast<const double*>(v), 2, A, P, &zero, reinterpret_cast<double*>(a), 2),
          "dgemm");
      for (int s = 0; s < nx && ret == SWKB_OK; ++s) {
        hipLaunchKernelGGL(phase_kernel, dim3((P + 255) / 256), dim3(256), 0, st, a, lam, xs[s], w, P);
        ok(hipGetLastError(), "phase");
        // u^T (2 x P) = w^T (2 x P) * Phi^T
        okb(rocblas_dgemm(hb, rocblas_operation_none, rocblas_operation_transpose, 2, P, P, &one,
                          reinterpret_cast<const double*>(w), 2, A, P, &zero, reinterpret_cast<double*>(o), 2),
            "dgemm");
        // physical part of the grid
        double2* dst = static_cast<double2*>(out) + (size_t)s * N;
        ok(hipMemcpyAsync(dst, o + (P - N), sizeof(double2) * N, hipMemcpyDeviceToDevice, st), "copy");
      }
      int hinfo = 0;
      if (ok(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st), "copy") &&
          ok(hipStreamSynchronize(st), "sync") && hinfo != 0) {
        ret = SWKB_ERR_DEVICE;
        why = "dsyevd did not converge";
      }
    }
  }
  (void)hipStreamSynchronize(st);
  if (hb) rocblas_destroy_handle(hb);
  (void)hipFree(A);
  (void)hipFree(lam);
  (void)hipFree(E);
  (void)hipFree(mp);
  (void)hipFree(v);
  (void)hipFree(a);
  (void)hipFree(w);
  (void)hipFree(o);
  (void)hipFree(info);
  if (ret != SWKB_OK) set_error(why);
  return ret;
}
