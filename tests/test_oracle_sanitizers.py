"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code; OpenMP off so the runs are serial) and driven through every
medium kind, the periodic grid and both ground mirrors, a ragged ray stride
and launch extension, two modes only, a mode set that reaches the evanescent
edge, and the stage entry points (modes, one mode's rays, interpolation):
any out-of-bounds access, use after free, leak or undefined operation ends
the run with a report and a nonzero status."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdio.h>
#include "swkb_oracle.c"

static double u_re(int m, int n) { return exp(-pow((m - 0.4 * n) / (0.05 * n), 2)); }

static int run_case(const char* name, or_params P, int screens) {
  int N = P.n_z;
  double* u = (double*)calloc(2 * (size_t)N, sizeof(double));
  double* hist = (double*)calloc(2 * (size_t)N * screens, sizeof(double));
  for (int m = 0; m < N; ++m) { u[2 * m] = u_re(m, N); u[2 * m + 1] = 0.3 * u_re(m, N); }
  or_counters c;
  memset(&c, 0, sizeof c);
  int rc = or_run(&P, u, 0, screens, hist, &c);
  /* stage entry points on the same problem */
  int M = P.n_modes, R = or_num_rays(&P);
  double* cm = (double*)calloc(2 * (size_t)M, sizeof(double));
  rc |= or_modes(&P, u, cm);
  double *Z = calloc(R, sizeof(double)), *ps = calloc(R, sizeof(double)), *q = calloc(R, sizeof(double)),
         *a = calloc(R, sizeof(double));
  int32_t* fl = calloc(R, sizeof(int32_t));
  rc |= or_march_mode(&P, P.x0, M - 1, Z, ps, q, a, fl);
  double zz[7], po[7], ao[7];
  int32_t has[7];
  for (int i = 0; i < 7; ++i) zz[i] = P.z_a + (P.z_b - P.z_a) * (i - 1) / 5.0;
  or_interp(R, Z, ps, q, a, fl, 7, zz, po, ao, has);
  double s = 0.0;
  for (size_t i = 0; i < 2 * (size_t)N * screens; ++i) s += hist[i];
  printf("%s rc=%d caustic=%lld dead=%lld checksum=%.6e\n", name, rc, (long long)c.caustic_rays,
         (long long)c.dead_rays, s);
  free(u); free(hist); free(cm); free(Z); free(ps); free(q); free(a); free(fl);
  return rc;
}

int main(void) {
  int rc = 0;
  double lin[2] = {1.0, 0.02};
  or_params P = {.k = 6.283185307179586, .z_a = 0.0, .z_b = 64.0, .n_z = 128, .n_modes = 32, .x0 = 0.0,
                 .dx = 8.0, .n_screens = 3, .rk4_steps = 4, .ray_stride = 1, .launch_ext_cells = 16,
                 .p2_floor = 1e-2, .bc = OR_BC_PERIODIC, .absorber_bot = 8.0, .absorber_top = 8.0,
                 .medium_kind = OR_MEDIUM_LINEAR, .n_medium_params = 2, .medium_params = lin,
                 .caustic_tol = 1e-3};
  rc |= run_case("linear_periodic", P, 3);
  or_params P2 = P; P2.ray_stride = 3; P2.launch_ext_cells = 7; P2.n_modes = 2;
  rc |= run_case("linear_ragged_M2", P2, 2);
  or_params P3 = P; P3.n_modes = 128; /* every mode of the grid, evanescent edge included */
  rc |= run_case("linear_all_modes", P3, 2);
  double mp[6] = {330.0, -0.3, 0.118, 40.0, 1.0, 1e-6};
  or_params P4 = P; P4.k = 125.66370614359172; P4.z_b = 60.0; P4.n_z = 256; P4.n_modes = 64; P4.dx = 100.0;
  P4.medium_kind = OR_MEDIUM_MPROFILE; P4.n_medium_params = 6; P4.medium_params = mp; P4.bc = OR_BC_DIRICHLET;
  P4.absorber_bot = 0.0; P4.absorber_top = 10.0; P4.launch_ext_cells = 32;
  rc |= run_case("duct_dirichlet", P4, 2);
  double eg[4] = {1.0, 0.05, 0.01, 32.0};
  or_params P5 = P; P5.medium_kind = OR_MEDIUM_EXPGAUSS; P5.n_medium_params = 4; P5.medium_params = eg;
  P5.bc = OR_BC_NEUMANN;
  rc |= run_case("expgauss_neumann", P5, 2);
  double gs[1 + 4 * 3] = {3, 0.01, 3.0, 4.0, 30.0, -0.01, 2.0, 12.0, 20.0, 0.005, 4.0, 20.0, 40.0};
  or_params P6 = P; P6.medium_kind = OR_MEDIUM_GAUSSSUM; P6.n_medium_params = 13; P6.medium_params = gs;
  rc |= run_case("gausssum_periodic", P6, 3);
  or_params P7 = P6; P7.bc = OR_BC_DIRICHLET; P7.ray_stride = 2; P7.launch_ext_cells = 9;
  rc |= run_case("gausssum_dirichlet_ragged", P7, 2);
  return rc;
}
"""


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    flags = ["-std=gnu99", "-O1", "-g", "-D_GNU_SOURCE", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wno-unknown-pragmas"]
    subprocess.check_call(["gcc", *flags, "-I", os.path.join(ROOT, "oracle"), "-o", str(exe), str(src), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.strip().splitlines()
    assert len(lines) == 7 and all("rc=0" in ln for ln in lines), r.stdout
