"""Seeded, synthetic workloads for the screened-WKB propagation step.

This module holds problem *descriptions* only: geometry, numerical
parameters, seeded random draws of media and the incident field on the
first screen.  It contains none of the method's arithmetic (no medium
evaluation, no FFT, no ray march, no interpolation, no superposition), so
both the CPU oracle and the GPU library may take their inputs from it
without sharing any of the method.

Every workload is a plain ``dict`` whose keys mirror the fields of the
``swkb_params`` C struct:

    lam, k            wavelength and wavenumber k = 2*pi/lam
    z_a, z_b          vertical extent of a screen (paper Sec. 2, planar screens)
    n_z, n_modes      grid points N on a screen and kept Fourier modes M
    x0, dx, n_screens first screen, screen spacing, number of screen steps
    rk4_steps         RK4 steps S per screen
    ray_stride        launch spacing of rays, in grid cells (rho)
    launch_ext_cells  launch extension E beyond [z_a, z_b], in grid cells
    p2_floor          rays with p^2 = eps - q^2 at or below this are dead
    bc                0 periodic, 1 Dirichlet ground mirror, 2 Neumann mirror
    absorber_bot/top  thickness of the cos^2 taper layers (0 = none)
    caustic_tol       a mode with caustic or crossing rays is reported as an
                      error when |c_n| > caustic_tol * max |c|
    propagator        GPU library only: 0 auto, 1 mode-function matrix, 2 recompute
    max_batch         GPU library only: most fields one batched propagation carries
    medium_kind       MEDIUM_* below;  medium_params: float64 array
    eps_ref           reference permittivity for the phase split
    source            dict(z0, width, xi0) of the incident Gaussian beam

Medium parameter layouts (shared data format; each side parses it itself):

    MEDIUM_LINEAR    [eps0, g]                      eps = eps0 + g z
    MEDIUM_EXPGAUSS  [eps0, a, b, zc]               eps = eps0 + a exp(-b (z-zc)^2)
                                                    (the paper's exponential
                                                    permittivity model, Sec. 3)
    MEDIUM_GAUSSSUM  [n_g, (a, s, cx, cz) * n_g]    n = 1 + sum a exp(-r^2/(2 s^2)),
                                                    terms with r^2 > 64 s^2 dropped,
                                                    eps = n^2
    MEDIUM_MPROFILE  [M0, g1, g2, d, w, scale]      modified refractivity
                                                    M = M0 + g1 z + (g2-g1) w softplus((z-d)/w),
                                                    n = 1 + scale M, eps = n^2
"""
from __future__ import annotations

import math

import numpy as np

MEDIUM_LINEAR = 0
MEDIUM_EXPGAUSS = 1
MEDIUM_GAUSSSUM = 2
MEDIUM_MPROFILE = 3

BC_PERIODIC = 0
BC_DIRICHLET = 1
BC_NEUMANN = 2

PRECISION_FP64 = 0
PRECISION_MIXED = 1


def _base(lam, z_a, z_b, n_z, n_modes, x0, dx, n_screens, rk4_steps, ray_stride,
          launch_ext_cells, bc, absorber_bot, absorber_top, medium_kind,
          medium_params, eps_ref, source, p2_floor=1e-2, caustic_tol=1e-3, propagator=0, max_batch=1,
          name=""):
    return dict(
        name=name,
        lam=float(lam), k=2.0 * math.pi / float(lam),
        z_a=float(z_a), z_b=float(z_b), n_z=int(n_z), n_modes=int(n_modes),
        x0=float(x0), dx=float(dx), n_screens=int(n_screens),
        rk4_steps=int(rk4_steps), ray_stride=int(ray_stride),
        launch_ext_cells=int(launch_ext_cells), p2_floor=float(p2_floor),
        bc=int(bc), absorber_bot=float(absorber_bot), absorber_top=float(absorber_top),
        medium_kind=int(medium_kind),
        medium_params=np.ascontiguousarray(np.asarray(medium_params, dtype=np.float64)),
        eps_ref=float(eps_ref), caustic_tol=float(caustic_tol), propagator=int(propagator),
        max_batch=int(max_batch),
        source=dict(source),
    )


def gaussian_sum_params(seed: int, n_g: int, x_span, z_span, amp=0.01, s_range=(20.0, 80.0)):
    """Seeded smooth random medium: n_g Gaussian bumps of the refractive index.

    Draw order (numpy default_rng): amplitudes a ~ U(-amp, amp), widths
    s ~ U(s_range), centres cx ~ U(x_span), cz ~ U(z_span).
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(-amp, amp, n_g)
    s = rng.uniform(s_range[0], s_range[1], n_g)
    cx = rng.uniform(x_span[0], x_span[1], n_g)
    cz = rng.uniform(z_span[0], z_span[1], n_g)
    out = np.empty(1 + 4 * n_g)
    out[0] = n_g
    out[1:] = np.stack([a, s, cx, cz], axis=1).reshape(-1)
    return out


def duct_params(slope_in=-0.3, depth=40.0, slope_above=0.118, M0=330.0, w=1.0):
    """Surface duct in modified refractivity (M units), corner smoothed over w metres."""
    return np.array([M0, slope_in, slope_above, depth, w, 1e-6])


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the problem statements; the numerical
# parameters (S, rho, E, p2_floor, absorbers) are fixed per workload and shared
# as data by the oracle and the GPU library.
# ---------------------------------------------------------------------------

def linear_caustic(n_screens=32):
    """Linear profile eps = 1 + 0.02 z with an Airy turning point.

    lambda = 1, z in [0, 64], N = 512, M = 128, 32 screens of width 8,
    Gaussian beam of width 4 centred at z = 16 tilted 10 degrees downward
    (xi0 = -n(16) sin 10deg), absorbers of thickness 8 at both ends.
    """
    xi0 = -math.sqrt(1.0 + 0.02 * 16.0) * math.sin(math.radians(10.0))
    return _base(lam=1.0, z_a=0.0, z_b=64.0, n_z=512, n_modes=128, x0=0.0, dx=8.0,
                 n_screens=n_screens, rk4_steps=16, ray_stride=1, launch_ext_cells=128,
                 bc=BC_PERIODIC, absorber_bot=8.0, absorber_top=8.0,
                 medium_kind=MEDIUM_LINEAR, medium_params=[1.0, 0.02], eps_ref=1.0,
                 source=dict(z0=16.0, width=4.0, xi0=xi0), name="linear_caustic_N512")


def random_medium(n_screens=400, n_z=8192, n_modes=2048, height=1000.0, seed=2301,
                  n_gauss=200, x_len=4000.0):
    """Smooth random medium of 200 Gaussian index bumps (seed 2301).

    lambda = 1, domain 4000 (range) x 1000 (height) wavelengths, N = 8192,
    M = 2048, 400 screens of width 10, beam of width 20 at mid-height,
    absorbers of thickness 50 at both ends.
    """
    h = height / n_z
    ext = int(math.ceil(32.0 / h / 8.0)) * 8
    return _base(lam=1.0, z_a=0.0, z_b=height, n_z=n_z, n_modes=n_modes, x0=0.0,
                 dx=10.0, n_screens=n_screens, rk4_steps=8, ray_stride=8,
                 launch_ext_cells=ext, bc=BC_PERIODIC, absorber_bot=50.0, absorber_top=50.0,
                 medium_kind=MEDIUM_GAUSSSUM,
                 medium_params=gaussian_sum_params(seed, n_gauss, (0.0, x_len), (0.0, height)),
                 eps_ref=1.0, source=dict(z0=height / 2.0, width=20.0, xi0=0.0),
                 name=f"random_medium_N{n_z}")


def surface_duct(n_screens=1000, n_z=16384, n_modes=4096, lam=0.05, height=300.0,
                 slope_in=-0.3, depth=40.0, source_z=25.0, beamwidth_deg=1.0, bc=BC_DIRICHLET,
                 ray_stride=8, ext_m=20.0, dx=100.0):
    """Atmospheric surface duct at 6 GHz over a Dirichlet ground.

    lambda = 0.05 m, height 0-300 m, N = 16384, 1000 screens of 100 m,
    M = 4096, Gaussian source at 25 m with a 1 degree half-power beamwidth,
    top absorber H/6.
    """
    h = height / n_z
    ext = int(math.ceil(ext_m / h / ray_stride)) * ray_stride
    k = 2.0 * math.pi / lam
    width = 2.0 * math.sqrt(2.0 * math.log(2.0)) / (k * math.radians(beamwidth_deg))
    mp = duct_params(slope_in=slope_in, depth=depth)
    # reference permittivity of the phase split: the ground-level value (1 + 1e-6 M0)^2
    eps_ref = (1.0 + mp[5] * mp[0]) ** 2
    return _base(lam=lam, z_a=0.0, z_b=height, n_z=n_z, n_modes=n_modes, x0=0.0, dx=dx,
                 n_screens=n_screens, rk4_steps=8, ray_stride=ray_stride, launch_ext_cells=ext,
                 bc=bc, absorber_bot=0.0, absorber_top=height / 6.0,
                 medium_kind=MEDIUM_MPROFILE, medium_params=mp,
                 eps_ref=eps_ref, source=dict(z0=source_z, width=width, xi0=0.0),
                 name=f"surface_duct_N{n_z}")


def duct_batch(seed=4, n_problems=64):
    """Uneven batch of surface-duct problems (seed 4)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_problems):
        f_ghz = rng.uniform(1.0, 10.0)
        depth = rng.uniform(10.0, 100.0)
        slope = rng.uniform(-0.5, -0.1)
        height = rng.uniform(200.0, 500.0)
        rng_km = rng.uniform(10.0, 100.0)
        lam = 0.3 / f_ghz
        nz = 2 ** int(math.ceil(math.log2(16.0 * height * math.sin(math.radians(3.5)) / lam)))
        nz = int(min(max(nz, 2048), 16384))
        h = height / nz
        rho = max(1, int(round(3.0 * lam / h)))
        cfg = surface_duct(n_screens=int(round(rng_km * 1000.0 / 100.0)), n_z=nz,
                           n_modes=nz // 4, lam=lam, height=height, slope_in=slope,
                           depth=depth, ray_stride=rho)
        cfg["name"] = f"duct_batch_{i}"
        out.append(cfg)
    return out


def serving_stream(seed=5, rate=20.0, duration=60.0):
    """Poisson stream of propagation requests: (arrival time, workload)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        nz = int(2 ** rng.integers(10, 16))
        if rng.uniform() < 0.5:
            f_ghz = rng.uniform(1.0, 10.0)
            lam = 0.3 / f_ghz
            height = rng.uniform(200.0, 500.0)
            h = height / nz
            rho = max(1, int(round(3.0 * lam / h)))
            cfg = surface_duct(n_screens=int(round(rng.uniform(10.0, 100.0) * 10.0)), n_z=nz,
                               n_modes=nz // 4, lam=lam, height=height,
                               slope_in=rng.uniform(-0.5, -0.1), depth=rng.uniform(10.0, 100.0),
                               source_z=rng.uniform(5.0, 100.0), ray_stride=rho)
        else:
            height = nz * (1000.0 / 8192.0)
            x_len = rng.uniform(1000.0, 4000.0)
            n_g = max(1, int(round(200 * (height * x_len) / (1000.0 * 4000.0))))
            cfg = random_medium(n_screens=int(round(x_len / 10.0)), n_z=nz, n_modes=nz // 4,
                                height=height, seed=int(rng.integers(1 << 31)), n_gauss=n_g,
                                x_len=x_len)
        reqs.append((t, cfg))
    return reqs


def grid(cfg):
    """Uniform screen grid z_m = z_a + m h, m = 0..N-1 (z_b excluded)."""
    h = (cfg["z_b"] - cfg["z_a"]) / cfg["n_z"]
    return cfg["z_a"] + h * np.arange(cfg["n_z"])


def incident_field(cfg):
    """Incident Gaussian beam on the first screen, complex128[N].

    u0(z) = exp(-((z - z0)/w)^2) exp(i k xi0 (z - z0)); xi0 = n sin(theta)
    fixes the tilt (negative = downward).
    """
    src = cfg["source"]
    z = grid(cfg)
    d = z - src["z0"]
    return np.exp(-(d / src["width"]) ** 2) * np.exp(1j * cfg["k"] * src["xi0"] * d)


def with_overrides(cfg, **kw):
    out = dict(cfg)
    out["source"] = dict(cfg["source"])
    for key, val in kw.items():
        if key == "medium_params":
            val = np.ascontiguousarray(np.asarray(val, dtype=np.float64))
        out[key] = val
    if "lam" in kw:
        out["k"] = 2.0 * math.pi / out["lam"]
    return out
