"""Pins of the oracle's overlapping-patch screen step (Sec. 2.4): the
partition of unity, exact propagation in a homogeneous medium (free and over
a ground mirror) against the angular spectrum on a large zero-padded domain,
linearity, and agreement with the single-domain step away from the edges."""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def OP():
    import oracle
    oracle.build()
    import oracle.patches as OP
    return OP


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def homogeneous(bc=W.BC_PERIODIC, n_z=512):
    """eps = 1 on z in [0, 64], no absorbers, a tilted Gaussian beam; the
    modes reach the evanescent cutoff (|xi| up to 1) with or without the
    ground mirror."""
    cfg = W.with_overrides(W.linear_caustic(n_screens=2), medium_params=[1.0, 0.0], absorber_bot=0.0,
                           absorber_top=0.0, bc=bc, n_z=n_z,
                           n_modes=n_z // 4 if bc == W.BC_PERIODIC else n_z // 2)
    cfg["source"] = dict(z0=30.0, width=3.0, xi0=0.3)
    return cfg


def angular_spectrum(cfg, u, dx, pad=16):
    """Exact propagation over dx of the field u (zero outside the grid, or odd
    about z_a for a Dirichlet ground) on a domain pad times as tall."""
    N = cfg["n_z"]
    h = (cfg["z_b"] - cfg["z_a"]) / N
    L = pad * N
    big = np.zeros(L, dtype=np.complex128)
    off = L // 2
    big[off:off + N] = u
    if cfg["bc"] == W.BC_DIRICHLET:
        big[off - np.arange(1, N)] = -u[1:]
    xi = np.fft.fftfreq(L, d=h) * cfg["lam"]
    kz = np.where(xi ** 2 < 1.0 - cfg["p2_floor"], np.sqrt(np.maximum(1.0 - xi ** 2, 0.0)), 0.0)
    spec = np.fft.fft(big) * np.where(xi ** 2 < 1.0 - cfg["p2_floor"], np.exp(1j * cfg["k"] * kz * dx), 0.0)
    return np.fft.ifft(spec)[off:off + N]


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_partition_of_unity(OP, P):
    cfg = W.with_overrides(W.linear_caustic(), n_z=480)  # 480 = 4 * 120 = 3 * 160
    z = W.grid(cfg)
    w = 2.0
    S = OP.partition(cfg, P, w, z)
    assert S.shape == (P, z.size)
    assert np.max(np.abs(S.sum(axis=0) - 1.0)) < 2e-15
    assert S.min() >= 0.0 and S.max() <= 1.0
    h = (cfg["z_b"] - cfg["z_a"]) / cfg["n_z"]
    K = cfg["n_z"] // P
    for p in range(P):
        lo = cfg["z_a"] + p * K * h - 6 * w
        hi = cfg["z_a"] + (p + 1) * K * h + 6 * w
        outside = (z < lo) | (z > hi)
        assert np.all(S[p][outside] < 1e-16)


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET])
def test_homogeneous_medium_is_exact(OP, bc):
    """n = 1: every sub-domain step is an exact plane-wave propagation, so the
    patch step equals the exact angular spectrum of the whole field, provided
    the windows are wide enough (3 wavelengths: their spectra fall as
    exp(-(pi w xi / lambda)^2), 1e-39 at the evanescent cutoff) that no
    windowed piece reaches the modes a sub-domain drops."""
    cfg = homogeneous(bc=bc)
    u0 = W.incident_field(cfg)
    got = OP.screen(cfg, 0, u0, 4, 3.0, 16.0)
    ref = angular_spectrum(cfg, u0, cfg["dx"])
    err = rel(got, ref)
    print(f"patch vs angular spectrum (bc={bc}): {err:.2e}")
    assert err < 1e-11


def test_linearity(OP):
    cfg = W.linear_caustic(n_screens=2)
    rng = np.random.default_rng(3)
    z = W.grid(cfg)
    u = W.incident_field(cfg)
    v = np.exp(-((z - 40.0) / 5.0) ** 2) * np.exp(1j * rng.uniform(0, 2 * math.pi))
    a, b = 0.7 - 0.2j, -1.3 + 0.4j
    lhs = OP.screen(cfg, 1, a * u + b * v, 2, 1.5, 12.0)
    rhs = a * OP.screen(cfg, 1, u, 2, 1.5, 12.0) + b * OP.screen(cfg, 1, v, 2, 1.5, 12.0)
    assert rel(lhs, rhs) < 1e-13


def test_close_to_single_domain_step(OP):
    """Away from the edges the patch step and the single-domain step of
    Sec. 2.1 approximate the same field (linear caustic, beam mid-domain)."""
    import oracle
    cfg = W.linear_caustic(n_screens=3)
    cfg["source"] = dict(z0=32.0, width=4.0, xi0=0.1)
    u0 = W.incident_field(cfg)
    full, _ = oracle.run(cfg, u0)
    patch = OP.run(cfg, u0, 4, 3.0, 16.0)
    err = rel(patch, full)
    print(f"patch vs single-domain, 3 screens: {err:.2e}")
    assert err < 1e-6
