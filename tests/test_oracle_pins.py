"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test compares the oracle with something other than itself: numpy's
FFT, finite differences, closed-form parabolic rays, the paper's own
characteristic system in the ray parameter t integrated by scipy, the exact
angular spectrum for a homogeneous medium, and the paper's reference method
(separation of variables, Sec. 3.1) as a dense eigensolve.
"""
import math

import numpy as np
import pytest

import workloads as W
from refs import GaussBumps, modal_reference, rel_l2, t_system_ray


def small_linear(**kw):
    cfg = W.with_overrides(W.linear_caustic(), **kw)
    return cfg


# ------------------------------------------------------------ step 1: DFT

@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET, W.BC_NEUMANN])
def test_modes_match_numpy_fft(oracle_mod, bc):
    """Mode amplitudes = numpy FFT of the (extended) field / P, low |n| kept."""
    cfg = small_linear(bc=bc, n_z=256, n_modes=96)
    rng = np.random.default_rng(1)
    u = rng.normal(size=256) + 1j * rng.normal(size=256)
    c = oracle_mod.modes(cfg, u)
    N = cfg["n_z"]
    if bc == W.BC_PERIODIC:
        v = u.copy()
    else:  # extension about z_a written out: index N+m <- u_m, N-m <- -/+ u_m
        sgn = -1.0 if bc == W.BC_DIRICHLET else 1.0
        v = np.zeros(2 * N, complex)
        v[N:] = u
        v[N - np.arange(1, N)] = sgn * u[1:]
        if bc == W.BC_DIRICHLET:
            v[N] = 0.0
    P = v.size
    W_ = np.fft.fft(v) / P
    n = np.arange(-48, 48)
    ref = W_[n % P]
    assert rel_l2(c, ref) < 1e-13
    # brute force on one mode: the definition with the phase origin z0'
    j = 10
    brute = np.sum(v * np.exp(-2j * np.pi * n[j] * np.arange(P) / P)) / P
    assert abs(c[j] - brute) < 1e-13 * np.abs(ref).max()


def test_dft_parseval(oracle_mod):
    """With all modes kept the DFT is unitary up to 1/sqrt(P)."""
    cfg = small_linear(n_z=128, n_modes=128)
    u = np.random.default_rng(2).normal(size=128) + 0j
    c = oracle_mod.modes(cfg, u)
    assert abs(np.sum(np.abs(c) ** 2) * 128 - np.sum(np.abs(u) ** 2)) < 1e-12 * np.sum(np.abs(u) ** 2)


# ---------------------------------------------------------------- medium

def _fd(f, z, h):
    return (f(z - 2 * h) - 8 * f(z - h) + 8 * f(z + h) - f(z + 2 * h)) / (12 * h)


MEDIA = [
    ("linear", W.MEDIUM_LINEAR, [1.0, 0.02], W.BC_PERIODIC),
    ("expgauss", W.MEDIUM_EXPGAUSS, [1.0, 0.05, 0.01, 32.0], W.BC_PERIODIC),
    ("gausssum", W.MEDIUM_GAUSSSUM, W.gaussian_sum_params(7, 12, (0, 200), (0, 64), s_range=(5, 15)), W.BC_PERIODIC),
    ("duct", W.MEDIUM_MPROFILE, W.duct_params(), W.BC_PERIODIC),
    ("duct_mirror", W.MEDIUM_MPROFILE, W.duct_params(), W.BC_DIRICHLET),
]


@pytest.mark.parametrize("name,kind,params,bc", MEDIA)
def test_medium_derivatives_match_finite_differences(oracle_mod, name, kind, params, bc):
    cfg = small_linear(medium_kind=kind, medium_params=params, bc=bc)
    z = np.linspace(3.0, 60.0, 23) if bc == W.BC_PERIODIC else np.linspace(-60.0, -3.0, 23)
    x = np.full_like(z, 37.0)
    e, ez, ezz = oracle_mod.medium(cfg, x, z)
    h = 1e-3
    fe = lambda zz: oracle_mod.medium(cfg, x, zz)[0]
    fez = lambda zz: oracle_mod.medium(cfg, x, zz)[1]
    # five-point differences: truncation O(h^4), rounding ~1e-16 |eps| / h
    assert np.abs(_fd(fe, z, h) - ez).max() < 1e-12 + 1e-8 * np.abs(ez).max()
    assert np.abs(_fd(fez, z, h) - ezz).max() < 1e-14 + 1e-7 * np.abs(ezz).max()
    assert np.abs(ez).max() > 0


def test_medium_closed_forms(oracle_mod):
    # linear
    cfg = small_linear()
    e, ez, ezz = oracle_mod.medium(cfg, 0.0, np.array([0.0, 10.0]))
    assert np.allclose(e, [1.0, 1.2], rtol=0, atol=1e-15) and np.allclose(ez, 0.02) and np.all(ezz == 0)
    # duct: slopes -0.3 M/m well below the corner and +0.118 M/m well above
    cfg = small_linear(medium_kind=W.MEDIUM_MPROFILE, medium_params=W.duct_params())
    z = np.array([0.0, 10.0, 100.0, 200.0])
    e, ez, _ = oracle_mod.medium(cfg, 0.0, z)
    n = np.sqrt(e)
    nz = ez / (2 * n)
    assert abs(n[0] - (1 + 330e-6)) < 1e-15
    assert abs(nz[1] / 1e-6 + 0.3) < 1e-9 and abs(nz[3] / 1e-6 - 0.118) < 1e-9
    # the mirror reflects eps about the ground: eps(-z) = eps(z), eps_z odd
    cfgm = small_linear(medium_kind=W.MEDIUM_MPROFILE, medium_params=W.duct_params(), bc=W.BC_DIRICHLET)
    em, ezm, ezzm = oracle_mod.medium(cfgm, 0.0, -z[1:])
    e2, ez2, ezz2 = oracle_mod.medium(cfgm, 0.0, z[1:])
    assert np.array_equal(em, e2) and np.array_equal(ezm, -ez2) and np.array_equal(ezzm, ezz2)
    # Gaussian sum: value at a lone bump's centre, and the 8-sigma cutoff
    gp = np.array([1, 0.01, 10.0, 50.0, 30.0])
    cfg = small_linear(medium_kind=W.MEDIUM_GAUSSSUM, medium_params=gp)
    e, ez, ezz = oracle_mod.medium(cfg, np.array([50.0, 50.0, 50.0]), np.array([30.0, 30.0 + 79.9, 30.0 + 80.1]))
    assert abs(e[0] - 1.01 ** 2) < 1e-15 and ez[0] == 0.0
    assert abs(ezz[0] - 2 * 1.01 * (-0.01 / 100.0)) < 1e-15
    assert e[1] != 1.0 and e[2] == 1.0


# ------------------------------------------------------------ step 2: rays

def _parabola(g, s, xi, D):
    p0 = math.sqrt(1 + g * s - xi * xi)
    z = s + xi * D / p0 + g * D * D / (4 * p0 * p0)
    q = xi + g * D / (2 * p0)
    t = D / (2 * p0)
    dpsi = 2 * (1 + g * s) * t + 2 * g * xi * t * t + (2.0 / 3.0) * g * g * t ** 3
    Zs = 1 - xi * g * D / (2 * p0 ** 3) - g * g * D * D / (4 * p0 ** 4)
    return z, q, dpsi, 1.0 / math.sqrt(Zs)


@pytest.mark.parametrize("j", [64 - 13, 64, 64 + 20])
def test_rays_match_closed_form_parabolas(oracle_mod, j):
    """eps = 1 + g z: p is constant on a ray, z is a parabola in x, Z_s and
    psi are polynomials; the amplitude is 1/sqrt(Z_s)."""
    g = 0.02
    errs = {}
    for S in (8, 16, 64):
        cfg = small_linear(rk4_steps=S, n_z=128, n_modes=128, launch_ext_cells=16, ray_stride=4)
        rec = oracle_mod.march_mode(cfg, 3, j)
        h = 64.0 / 128
        xi = 2 * math.pi * (j - 64) / (cfg["k"] * 128 * h)
        worst = 0.0
        for r in range(0, rec["Z"].size, 5):
            s = (r * 4 - 16) * h
            if rec["flag"][r] != 0:
                continue
            z, q, dpsi, a = _parabola(g, s, xi, cfg["dx"])
            psi = xi * s + dpsi
            worst = max(worst, abs(rec["Z"][r] - z), abs(rec["q"][r] - q), abs(rec["psi"][r] - psi),
                        abs(rec["a"][r] - a))
        errs[S] = worst
    assert errs[64] < 2e-12
    # fourth-order convergence of the RK4 march
    assert errs[8] / errs[16] > 12.0


MED_T = {
    "expgauss": (W.MEDIUM_EXPGAUSS, [1.0, 0.05, 0.01, 32.0]),
    "bumps_xvarying": (W.MEDIUM_GAUSSSUM, np.array([3, 0.03, 6.0, 30.0, 20.0, -0.02, 9.0, 34.0, 40.0,
                                                    0.025, 12.0, 26.0, 34.0])),
}


@pytest.mark.parametrize("name", sorted(MED_T))
def test_x_march_matches_paper_t_system(oracle_mod, name):
    """The oracle's x-march equals the paper's characteristic system in t with
    the transport law A_t = -Delta Psi A (Cramer rule), rays stopped on the
    next screen; this also fixes the amplitude law a = A0 sqrt(J0/J)."""
    kind, params = MED_T[name]
    cfg = small_linear(medium_kind=kind, medium_params=params, rk4_steps=64, n_z=128, n_modes=128,
                       launch_ext_cells=16, ray_stride=4, x0=20.0)
    if kind == W.MEDIUM_GAUSSSUM:
        def med(x, z):
            return GaussBumps(params)(x, z)
    else:
        e0, a, b, zc = params

        def med(x, z):
            d = z - zc
            gg = a * math.exp(-b * d * d)
            return e0 + gg, 0.0, -2 * b * d * gg, 0.0, 0.0, (4 * b * b * d * d - 2 * b) * gg
    h = 0.5
    for j in (50, 64, 77):
        xi = 2 * math.pi * (j - 64) / (cfg["k"] * 128 * h)
        rec = oracle_mod.march_mode(cfg, 0, j)
        for r in (5, 15, 25, 35):
            s = (r * 4 - 16) * h
            ref = t_system_ray(med, 20.0, s, xi, 0.0, cfg["dx"])
            assert rec["flag"][r] == 0
            assert abs(rec["Z"][r] - ref["Z"]) < 1e-10
            assert abs(rec["q"][r] - ref["q"]) < 1e-10
            assert abs(rec["psi"][r] - ref["psi"]) < 1e-9
            # amplitude: transport ODE along t (Cramer Delta Psi) vs the x-march
            assert abs(rec["a"][r] - ref["A"]) < 1e-9
            assert abs(ref["A"] - math.sqrt(ref["J0"] / ref["J"])) < 1e-9


def test_zs_matches_finite_difference_of_launch_point(oracle_mod):
    """dZ/ds from neighbouring launch points agrees with the variational
    state (recovered from the amplitude a^2 = p0/(p Z_s))."""
    params = MED_T["bumps_xvarying"][1]
    base = small_linear(medium_kind=W.MEDIUM_GAUSSSUM, medium_params=params, rk4_steps=64,
                        n_z=128, n_modes=128, launch_ext_cells=16, ray_stride=4, x0=20.0)
    d = 1e-4
    recs = {sgn: oracle_mod.march_mode(W.with_overrides(base, z_a=sgn * d, z_b=64.0 + sgn * d), 0, 70)
            for sgn in (-1, 0, 1)}
    med = GaussBumps(params)
    xi = 2 * math.pi * 6 / (base["k"] * 64.0)
    for r in (10, 20, 30):
        dZds = (recs[1]["Z"][r] - recs[-1]["Z"][r]) / (2 * d)
        s = (r * 4 - 16) * 0.5
        p0 = math.sqrt(med(20.0, s)[0] - xi * xi)
        Z, q, a = recs[0]["Z"][r], recs[0]["q"][r], recs[0]["a"][r]
        p = math.sqrt(med(20.0 + base["dx"], Z)[0] - q * q)
        Zs = p0 / (p * a * a)
        assert abs(dZds - Zs) < 1e-7


def test_dead_rays_and_caustics_are_flagged(oracle_mod):
    cfg = small_linear()
    rec = oracle_mod.march_mode(cfg, 0, 0)  # xi = -1: evanescent everywhere below z ~ 0.5
    assert np.all(rec["flag"][:100] == oracle_mod.RAY_DEAD_LAUNCH)
    # a very wide screen makes steep upward modes cross (Z_s <= 0)
    wide = small_linear(dx=200.0, rk4_steps=64)
    rec = oracle_mod.march_mode(wide, 0, 64 + 50)
    assert np.any(rec["flag"] == oracle_mod.RAY_CAUSTIC)


# ---------------------------------------------------- step 3: interpolation

def test_interpolation_exact_on_cubics(oracle_mod):
    rng = np.random.default_rng(3)
    Z = np.cumsum(rng.uniform(0.5, 1.5, 12))
    c = rng.normal(size=4)
    psi = c[0] + c[1] * Z + c[2] * Z ** 2 + c[3] * Z ** 3
    q = c[1] + 2 * c[2] * Z + 3 * c[3] * Z ** 2
    d = rng.normal(size=4)
    a = d[0] + d[1] * Z + d[2] * Z ** 2 + d[3] * Z ** 3
    rec = dict(Z=Z, psi=psi, q=q, a=a, flag=np.zeros(12, np.int32))
    z = np.linspace(Z[1], Z[-2] - 1e-9, 50)
    ps, aa, has, fold = oracle_mod.interp(rec, z)
    assert not fold and has.all()
    assert np.abs(ps - (c[0] + c[1] * z + c[2] * z ** 2 + c[3] * z ** 3)).max() < 1e-11
    assert np.abs(aa - (d[0] + d[1] * z + d[2] * z ** 2 + d[3] * z ** 3)).max() < 1e-10
    # first/last interval: linear amplitude; outside the arrivals: no bracket
    zz = np.array([0.5 * (Z[0] + Z[1]), Z[0] - 0.1, Z[-1] + 0.1])
    ps, aa, has, _ = oracle_mod.interp(rec, zz)
    assert has.tolist() == [True, False, False]
    t = (zz[0] - Z[0]) / (Z[1] - Z[0])
    assert abs(aa[0] - ((1 - t) * a[0] + t * a[1])) < 1e-13
    # a dead ray removes both intervals that touch it
    rec2 = dict(rec, flag=np.where(np.arange(12) == 5, 2, 0).astype(np.int32))
    zz = np.array([0.5 * (Z[4] + Z[5]), 0.5 * (Z[5] + Z[6]), 0.5 * (Z[6] + Z[7])])
    _, _, has, _ = oracle_mod.interp(rec2, zz)
    assert has.tolist() == [False, False, True]
    # crossing rays fold the mode
    Zf = Z.copy()
    Zf[7], Zf[8] = Zf[8], Zf[7]
    _, _, has, fold = oracle_mod.interp(dict(rec, Z=Zf), z)
    assert fold and not has.any()


# ------------------------------------------------- whole method, closed forms

def _homog(**kw):
    base = dict(medium_params=[1.0, 0.0], absorber_bot=0.0, absorber_top=0.0)
    base.update(kw)
    cfg = small_linear(**base)
    cfg["source"] = dict(z0=32.0, width=4.0, xi0=cfg["source"]["xi0"])
    return cfg


def _angular_spectrum(cfg, u0, X):
    N, M = cfg["n_z"], cfg["n_modes"]
    n = np.arange(-M // 2, M // 2)
    xi = 2 * np.pi * n / (cfg["k"] * (cfg["z_b"] - cfg["z_a"]))
    live = 1 - xi ** 2 > cfg["p2_floor"]
    c = np.fft.fft(u0)[n % N] / N
    p = np.sqrt(np.where(live, 1 - xi ** 2, 0.0))
    m = np.arange(N)
    return (np.exp(2j * np.pi * np.outer(m, n) / N) * np.where(live, np.exp(1j * cfg["k"] * p * X), 0)) @ c


def test_homogeneous_medium_is_exact_angular_spectrum(oracle_mod):
    """eps = 1: rays are straight, a = 1 and psi is linear, so S-WKB is the
    exact propagator of the kept plane waves, whatever the screen count."""
    cfg = _homog()
    u0 = W.incident_field(cfg)
    hist, cnt = oracle_mod.run(cfg, u0, 0, 4)
    ref = _angular_spectrum(cfg, u0, 32.0)
    assert rel_l2(hist[-1], ref) < 1e-12
    cfg2 = _homog(dx=16.0)
    hist2, _ = oracle_mod.run(cfg2, u0, 0, 2)
    assert rel_l2(hist2[-1], ref) < 1e-12
    assert cnt["caustic_rays"] == 0 and cnt["significant"] == 0


def test_evanescent_mode_carries_nothing_and_is_counted(oracle_mod):
    """A free-space beam aimed at grazing incidence (xi0 = -0.999): the kept
    mode xi = -1 has p^2 = 0 on every ray, so it is dead and contributes
    nothing; every other mode is carried exactly (the launch extension covers
    the drift of the steepest live mode).  The oracle equals the exact
    angular spectrum of the live modes and counts one evanescent mode per
    screen, significant on the first screen only (the next screens' fields
    hold no weight there)."""
    cfg = _homog(launch_ext_cells=400, n_screens=2)
    cfg["source"] = dict(cfg["source"], xi0=-0.999)
    u0 = W.incident_field(cfg)
    hist, cnt = oracle_mod.run(cfg, u0)
    assert rel_l2(hist[-1], _angular_spectrum(cfg, u0, 16.0)) < 1e-12
    assert cnt["evanescent_modes"] == 2 and cnt["significant_evanescent"] == 1
    assert cnt["significant"] == 0
    # the same beam aimed at 30 degrees puts no weight on the dead mode
    cfg2 = _homog(launch_ext_cells=400, n_screens=2)
    cfg2["source"] = dict(cfg2["source"], xi0=-0.5)
    _, cnt2 = oracle_mod.run(cfg2, W.incident_field(cfg2))
    assert cnt2["evanescent_modes"] == 2 and cnt2["significant_evanescent"] == 0


def test_absorber_taper(oracle_mod):
    # every kept mode is covered by rays (drift dx*xi/p < E), so the only
    # difference to the exact propagator is the taper
    cfg = _homog(absorber_bot=8.0, absorber_top=8.0, n_modes=120, launch_ext_cells=256)
    cfg["source"]["z0"] = 12.0
    u0 = W.incident_field(cfg)
    out, _ = oracle_mod.screen(cfg, 0, u0)
    ref = _angular_spectrum(cfg, u0, 8.0)
    z = W.grid(cfg)
    w = np.ones_like(z)
    lo, hi = z < 8.0, z > 56.0
    w[lo] = np.cos(0.5 * np.pi * (8.0 - z[lo]) / 8.0) ** 2
    w[hi] = np.cos(0.5 * np.pi * (z[hi] - 56.0) / 8.0) ** 2
    assert rel_l2(out, w * ref) < 1e-12


def test_linearity_in_the_field(oracle_mod):
    cfg = small_linear()
    rng = np.random.default_rng(4)
    u = W.incident_field(cfg)
    v = np.roll(u, 100) * np.exp(1j * rng.uniform(0, 6.3))
    al, be = 0.3 - 0.7j, 1.1 + 0.2j
    fu, _ = oracle_mod.run(cfg, u, 0, 3)
    fv, _ = oracle_mod.run(cfg, v, 0, 3)
    fw, _ = oracle_mod.run(cfg, al * u + be * v, 0, 3)
    assert rel_l2(fw, al * fu + be * fv) < 1e-13


def test_mirror_equals_periodic_run_of_the_odd_extension(oracle_mod):
    """One screen with the Dirichlet ground mirror equals, on the physical
    half, a periodic run on the doubled domain [z_a - L, z_b] of the
    odd-extended field in a medium even about z_a (Sec. 2.3)."""
    params = [1.0, 0.05, 0.004, 0.0]   # eps even about z_a = 0
    cfg = small_linear(bc=W.BC_DIRICHLET, medium_kind=W.MEDIUM_EXPGAUSS, medium_params=params,
                       n_z=256, n_modes=64, launch_ext_cells=64, ray_stride=2, absorber_top=0.0,
                       absorber_bot=0.0)
    cfg["source"] = dict(z0=12.0, width=3.0, xi0=-0.1)
    u = W.incident_field(cfg)
    out, _ = oracle_mod.screen(cfg, 0, u)
    dbl = small_linear(bc=W.BC_PERIODIC, medium_kind=W.MEDIUM_EXPGAUSS, medium_params=params,
                       n_z=512, n_modes=64, launch_ext_cells=64, ray_stride=2, z_a=-64.0, z_b=64.0,
                       absorber_top=0.0, absorber_bot=0.0)
    v = np.zeros(512, complex)
    v[256:] = u
    v[256 - np.arange(1, 256)] = -u[1:]
    v[256] = 0.0
    out2, _ = oracle_mod.screen(dbl, 0, v)
    assert rel_l2(out, out2[256:]) < 1e-13


# ------------------------------------------- symmetries of the whole method
#
# The mode expansion (Sec. 2.1.1), the characteristic system (Sec. 2.1.2) and
# the interpolation and superposition (Sec. 2.1.3) are built from the medium
# and the field alone, so moving both rigidly in z moves the result with them.
# A slip in an absolute height (the launch grid, the phase origin z_a, a
# record's base point) breaks the translation; a sign slip in xi or q, or a
# one-sided choice in the ray-interval search, breaks the reflection.


def _bumps(seed, amp, s_range, n_g=8, cx=(0.0, 60.0), cz=(85.0, 115.0)):
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(-amp, amp, n_g), rng.uniform(*s_range, n_g), rng.uniform(*cx, n_g),
                     rng.uniform(*cz, n_g)], axis=1)


def _bump_cfg(bumps, n_screens=6):
    """Gaussian-sum medium on [0, 200] (N = 512, M = 128, rho = 8) without
    absorbers; every bump's 8-sigma disc stays inside (37, 163), so the medium
    is homogeneous near both ends of the launch range."""
    cfg = W.random_medium(n_screens=n_screens, n_z=512, n_modes=128, height=200.0)
    prm = np.concatenate([[len(bumps)], np.asarray(bumps, dtype=np.float64).reshape(-1)])
    cfg = W.with_overrides(cfg, medium_params=prm, absorber_bot=0.0, absorber_top=0.0)
    cfg["source"] = dict(z0=92.0, width=8.0, xi0=0.05)
    return cfg


def _band_limited(cfg, seed):
    """Random field of the kept modes n = -M/2 + 1 .. M/2 - 1.  Mode -M/2 is
    left out: its mirror image +M/2 is not kept, so it alone would break the
    reflection."""
    N, M = cfg["n_z"], cfg["n_modes"]
    rng = np.random.default_rng(seed)
    n = np.arange(-M // 2 + 1, M // 2)
    cn = rng.normal(size=n.size) + 1j * rng.normal(size=n.size)
    return np.exp(2j * np.pi * np.outer(np.arange(N), n) / N) @ cn


@pytest.mark.parametrize("k", [8, 40, -24])
def test_translation_moves_the_result(oracle_mod, k):
    """Bumps raised by k cells and the beam rolled by k cells (k a multiple
    of the ray stride, so every ray keeps its place relative to the medium):
    three screens later the field is the rolled field, counters equal."""
    bumps = _bumps(11, 0.02, (3.0, 6.0))
    cfg = _bump_cfg(bumps)
    h = 200.0 / cfg["n_z"]
    assert k % cfg["ray_stride"] == 0
    u = W.incident_field(cfg)
    out, cnt = oracle_mod.run(cfg, u, 0, 3)
    moved = bumps.copy()
    moved[:, 3] += k * h
    out2, cnt2 = oracle_mod.run(_bump_cfg(moved), np.roll(u, k), 0, 3)
    assert rel_l2(out2[-1], np.roll(out[-1], k)) < 1e-12
    assert cnt2 == cnt


@pytest.mark.parametrize("q", [0, 3])
def test_reflection_mirrors_each_screen(oracle_mod, q):
    """Medium and field reflected about the middle of the periodic domain
    (z -> 2 z_a + L - z, grid point m -> -m mod N): one screen of the
    reflected problem gives the reflected output.  With the medium left
    unreflected the result is far off, so the check sees the medium."""
    bumps = _bumps(3, 0.1, (2.0, 4.0))
    refl = bumps.copy()
    refl[:, 3] = 200.0 - refl[:, 3]
    cfg, cfg_r = _bump_cfg(bumps), _bump_cfg(refl)
    v = _band_limited(cfg, 5)
    m = (-np.arange(cfg["n_z"])) % cfg["n_z"]
    out, cnt = oracle_mod.screen(cfg, q, v)
    out_r, cnt_r = oracle_mod.screen(cfg_r, q, v[m])
    assert rel_l2(out_r, out[m]) < 1e-12
    assert cnt_r == cnt
    wrong, _ = oracle_mod.screen(cfg, q, v[m])
    assert rel_l2(wrong, out[m]) > 1e-2


def test_reflection_mirrors_rays_through_caustics(oracle_mod):
    """Linear medium eps = 1 + 0.02 z and its reflection 1 + 0.02 (2 z_a + L)
    - 0.02 z, with a band-limited field so that rays of every kept slope
    reach turning points.  Mode j (n = j - M/2) of one problem is mode M - j
    of the other; its R rays come in reverse order, with arrival heights
    reflected, slopes q negated and amplitudes equal, and the same dead and
    caustic flags.  The screen's output is the reflected output."""
    cfg = W.linear_caustic(n_screens=4)
    L = cfg["z_b"] - cfg["z_a"]
    H2 = 2.0 * cfg["z_a"] + L
    cfg_r = W.with_overrides(cfg, medium_params=[1.0 + 0.02 * H2, -0.02])
    cfg["caustic_tol"] = cfg_r["caustic_tol"] = 2.0  # report only
    N, M = cfg["n_z"], cfg["n_modes"]
    R = oracle_mod.num_rays(cfg)
    assert (R - 1) * cfg["ray_stride"] == N + 2 * cfg["launch_ext_cells"]  # the launch grid is symmetric
    n_caustic = 0
    for j in range(1, M):
        a = oracle_mod.march_mode(cfg, 1, j)
        b = oracle_mod.march_mode(cfg_r, 1, M - j)
        np.testing.assert_array_equal(b["flag"][::-1], a["flag"])
        live = a["flag"] == 0
        n_caustic += int(np.count_nonzero(a["flag"] == 3))  # caustic: Z_s <= 0
        assert np.abs(b["Z"][::-1][live] - (H2 - a["Z"][live])).max(initial=0.0) < 1e-11
        assert np.abs(b["q"][::-1][live] + a["q"][live]).max(initial=0.0) < 1e-12
        amax = np.abs(a["a"][live]).max(initial=1.0)
        assert np.abs(b["a"][::-1][live] - a["a"][live]).max(initial=0.0) < 1e-12 * max(amax, 1.0)
    assert n_caustic > 500  # the case does reach caustics
    v = _band_limited(cfg, 2)
    m = (-np.arange(N)) % N
    out, cnt = oracle_mod.screen(cfg, 1, v)
    out_r, _ = oracle_mod.screen(cfg_r, 1, v[m])
    assert cnt["caustic_rays"] > 0 and cnt["dead_rays"] > 0
    assert rel_l2(out_r, out[m]) < 1e-12


# ------------------------------------- accuracy against the paper's reference

@pytest.mark.parametrize("name", ["linear", "expgauss"])
def test_error_against_separation_of_variables_is_order_one_over_k(oracle_mod, name):
    """x-invariant eps: the exact separation-of-variables solution (the
    paper's reference, Sec. 3.1) as a Fourier-spectral eigensolve.  S-WKB is
    leading-order WKB, so its error per screen is O(1/k): halving the
    wavelength halves it, and more RK4 steps do not change it."""
    if name == "linear":
        kw = dict(absorber_bot=0.0, absorber_top=0.0)
        epsf = lambda z: 1 + 0.02 * z
    else:
        kw = dict(medium_kind=W.MEDIUM_EXPGAUSS, medium_params=[1.0, 0.05, 0.01, 32.0],
                  absorber_bot=0.0, absorber_top=0.0)
        epsf = lambda z: 1 + 0.05 * np.exp(-0.01 * (z - 32) ** 2)
    errs = {}
    for lam, S in ((1.0, 16), (0.5, 16), (1.0, 32)):
        cfg = small_linear(lam=lam, rk4_steps=S, **kw)
        u0 = W.incident_field(cfg)
        hist, _ = oracle_mod.run(cfg, u0, 0, 4)
        z = W.grid(cfg)
        ref = modal_reference(z, 64.0, cfg["k"], epsf(z), u0, cfg["dx"] * np.arange(1, 5))
        errs[(lam, S)] = rel_l2(hist, ref)
    assert errs[(1.0, 16)] < 2e-4
    assert 1.8 < errs[(1.0, 16)] / errs[(0.5, 16)] < 2.2
    assert abs(errs[(1.0, 32)] / errs[(1.0, 16)] - 1) < 0.02
