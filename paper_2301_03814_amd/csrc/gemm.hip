// Batched sources through the mode-function matrix: for B fields on one
// screen the sums over modes U[b][m] = sum_j c[b][j] T[j][m] (eq.
// ray_bundle_q_plus_1 with T tabulated once) form one complex matrix product,
// a plain GEMM handed to rocBLAS (matrix cores): zgemm in FP64, cgemm with
// complex64 T and amplitudes in the mixed path.
#include <rocblas/rocblas.h>

#include "swkb_internal.h"

namespace swkb {

hipError_t gemm_fields(const swkb_plan_s& pl, int batch, hipStream_t st) {
  const Geometry& g = pl.g;
  rocblas_handle h = static_cast<rocblas_handle>(pl.blas);
  if (!h) return hipErrorInvalidValue;
  if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorInvalidValue;
  rocblas_status s;
  // column-major views: T is N x M (ld N), C is M x B (ld M), U is N x B (ld N)
  if (pl.precision == SWKB_FP64) {
    const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
    s = rocblas_zgemm(h, rocblas_operation_none, rocblas_operation_none, g.N, batch, g.M, &one,
                      static_cast<const rocblas_double_complex*>(pl.tmat), g.N,
                      reinterpret_cast<const rocblas_double_complex*>(pl.c), g.M, &zero,
                      reinterpret_cast<rocblas_double_complex*>(pl.part), g.N);
  } else {
    hipError_t e = launch_to_c64(pl, batch, st);
    if (e != hipSuccess) return e;
    const rocblas_float_complex one = {1.0f, 0.0f}, zero = {0.0f, 0.0f};
    s = rocblas_cgemm(h, rocblas_operation_none, rocblas_operation_none, g.N, batch, g.M, &one,
                      static_cast<const rocblas_float_complex*>(pl.tmat), g.N,
                      reinterpret_cast<const rocblas_float_complex*>(pl.cf), g.M, &zero,
                      reinterpret_cast<rocblas_float_complex*>(pl.part), g.N);
  }
  return s == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

}  // namespace swkb
