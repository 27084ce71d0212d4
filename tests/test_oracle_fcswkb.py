"""Pins of the oracle's Fourier-continuation patch step (FC-SWKB, Sec. 2.4
and 2.5), on the CPU:

* the FC-Gram blend data equal a fresh high-precision derivation;
* Fourier continuation: the DFT of a patch's continued period is an accurate
  Fourier series of a smooth non-periodic function (fifth-order convergence
  at points between the samples);
* in a homogeneous medium every ray is straight and keeps its launch
  amplitude, so the paper's representation propagates in closed form:
  sum_p sum_j (w_j / N) S^p(z - xi_j dx / p_j) e^{i k (xi_j (z - o) + p_j dx)}
  over the points of patch p's period window (plus the image term of eq.
  u_refl over a ground); the oracle's rays and interpolation must give this
  within the error bound of its 4-point Lagrange amplitude interpolation of
  S^p;
* agreement with the single-domain step (Sec. 2.1) when the partition of
  unity varies slowly on the Fresnel scale sqrt(lambda dx)."""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def FC():
    import oracle
    oracle.build()
    import oracle.fcswkb as FC
    return FC


def test_blend_data_equal_their_derivation(FC):
    from oracle import fc_gram
    fresh = np.array([[float(v) for v in row] for row in fc_gram.blend_matrix()])
    assert np.array_equal(fresh, fc_gram.load())


def test_fourier_continuation_converges(FC):
    """f(z) = exp(sin(5.3 z + 0.4)) + 0.3 z^2 on n points of [0, 1]: the
    Fourier series of the continued period at the midpoints between samples."""
    f = lambda z: np.exp(np.sin(5.3 * z + 0.4)) + 0.3 * z ** 2
    errs = []
    for n in (100, 200, 400):
        z = np.linspace(0.0, 1.0, n)
        h = z[1] - z[0]
        nz = 1
        while nz < n + 2 * 27:
            nz *= 2
        start = -((nz - n) // 2)
        v = FC.fc_period(f(z).astype(np.complex128), 0, n - 1, start, nz, False)
        c = np.fft.fft(v) / nz
        kk = np.fft.fftfreq(nz, 1.0 / nz)
        zm = 0.5 * (z[:-1] + z[1:])
        idx = zm / h - start  # period index of the midpoints
        val = np.exp(2j * np.pi * np.outer(idx, kk) / nz) @ c
        errs.append(float(np.max(np.abs(val - f(zm)))))
    assert errs[0] < 5e-8 and errs[1] < 2e-9 and errs[2] < 1e-10, errs
    assert errs[0] / errs[2] > 2.0 ** 8, errs  # at least fourth order


def homogeneous(bc, n_z=1024):
    cfg = W.with_overrides(W.linear_caustic(n_screens=1), medium_params=[1.0, 0.0], absorber_bot=0.0,
                           absorber_top=0.0, bc=bc, n_z=n_z, z_b=128.0,
                           n_modes=n_z // 4 if bc == W.BC_PERIODIC else n_z // 2,
                           launch_ext_cells=0 if bc == W.BC_PERIODIC else 96)
    if bc == W.BC_PERIODIC:
        cfg["source"] = dict(z0=60.0, width=4.0, xi0=0.2)
    else:
        cfg["source"] = dict(z0=14.0, width=4.0, xi0=-0.25)  # aimed at the ground
    return cfg


def sigma4_max(width):
    """max |d^4/dz^4 erfc(-(z - c)/w) / 2| = max |(12 x - 8 x^3) e^{-x^2}| / (sqrt(pi) w^4)."""
    x = np.linspace(-4.0, 4.0, 200001)
    return float(np.max(np.abs((12 * x - 8 * x ** 3) * np.exp(-x * x)))) / (math.sqrt(math.pi) * width ** 4)


def closed_form(FC, cfg, u0, P, width, margin):
    """The paper's representation carried over dx in eps = 1, evaluated
    directly, and the interpolation error bound of the oracle's amplitudes."""
    import oracle
    N = cfg["n_z"]
    h = (cfg["z_b"] - cfg["z_a"]) / N
    k, dx = cfg["k"], cfg["dx"]
    ground = cfg["bc"] != W.BC_PERIODIC
    sgn = -1.0 if cfg["bc"] == W.BC_DIRICHLET else 1.0
    z = W.grid(cfg)
    lay = FC.layout(cfg, P, width, margin)
    out = np.zeros(N, dtype=np.complex128)
    coef_sum = 0.0
    for p, L in enumerate(lay):
        sub, a, b = L["sub"], L["a"], L["b"]
        gp = p == 0 and ground
        c = oracle.modes(sub, FC.fc_period(u0, a, b, L["start"], sub["n_z"], gp))
        Pp = 2 * sub["n_z"] if gp else sub["n_z"]
        origin = sub["z_a"] - (sub["n_z"] * h if gp else 0.0)
        Mp = sub["n_modes"]

        def field_at(zz):
            # the patch's sum covers its period window only
            iw = np.rint((zz - sub["z_a"]) / h)
            inwin = (iw >= 0) & (iw < sub["n_z"])
            acc = np.zeros(zz.size, dtype=np.complex128)
            for j in range(Mp):
                xi = 2.0 * math.pi * (j - Mp // 2) / (k * Pp * h)
                if not (1.0 - xi * xi > cfg["p2_floor"]):
                    continue
                pz = math.sqrt(1.0 - xi * xi)
                s = zz - xi * dx / pz
                gi = (s - cfg["z_a"]) / h
                gm = np.abs(gi) if gp else gi
                ok = (gm >= a) & (gm <= b) & inwin
                S = np.zeros(zz.size)
                S[ok] = FC._partition(cfg, P, width, cfg["z_a"] + gm[ok] * h)[p]
                acc += c[j] * S * np.exp(1j * k * (xi * (zz - origin) + pz * dx))
            return acc

        out += field_at(z)
        reflect = ground and not gp
        if reflect:
            out += sgn * field_at(2.0 * cfg["z_a"] - z)
        coef_sum += float(np.sum(np.abs(c))) * (2.0 if reflect else 1.0)
    # 4-point Lagrange on rays one cell apart: |error| <= (9/16) h^4 / 24 max|S''''|
    bound = coef_sum * (9.0 / 16.0) * h ** 4 / 24.0 * 2.0 * sigma4_max(width)
    return out, bound


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET, W.BC_NEUMANN])
def test_homogeneous_medium_closed_form(FC, bc):
    cfg = homogeneous(bc)
    u0 = W.incident_field(cfg)
    if bc == W.BC_DIRICHLET:
        u0[0] = 0.0
    P, width, margin = 4, 2.0, 12.0
    got = FC.screen(cfg, 0, u0, P, width, margin)
    want, bound = closed_form(FC, cfg, u0, P, width, margin)
    err = float(np.max(np.abs(got - want)))
    assert err <= bound + 1e-12 * float(np.max(np.abs(want))), (err, bound)
    assert bound < 1e-3 * float(np.max(np.abs(want)))  # the pin is tight enough to catch a misplaced window


@pytest.mark.parametrize("case", ["linear_caustic", "duct_dirichlet"])
def test_agrees_with_single_domain(FC, case):
    import oracle
    if case == "linear_caustic":
        cfg, P, width, margin = W.linear_caustic(n_screens=2), 4, 3.0, 16.0
    else:
        cfg, P, width, margin = (W.surface_duct(n_screens=2, n_z=2048, n_modes=512, height=60.0, ext_m=4.0),
                                 4, 2.0, 4.0)
    u0 = W.incident_field(cfg)
    got = FC.run(cfg, u0, P, width, margin)
    ref, _ = oracle.run(cfg, u0)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-3
