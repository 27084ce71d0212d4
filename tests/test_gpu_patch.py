"""The screen step on overlapping patches (swkb_patch_*) through the C ABI
against the oracle's patch steps, for the paper's Fourier-continuation
patches (oracle.fcswkb) and the library's windowed pieces (oracle.patches):
the sub-domain layout bit for bit, FP64 fields to 1e-10, mixed fields to
1e-3 (regression bound 5e-5)."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-3
MIXED_REGRESSION = 5e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import oracle
    oracle.build()
    import oracle.fcswkb as FC
    import oracle.patches as OP
    import paper_2301_03814_amd as pkg
    pkg.load()
    return torch, pkg, {"fc": FC, "windowed": OP}


# (config, patches, window width, margin): periodic linear caustic, a
# Dirichlet and a Neumann duct over a ground (bottom patch mirrored), and an
# x-varying random medium.  Windowed pieces:
WINDOWED_CASES = {
    "linear_caustic_P4": lambda: (W.linear_caustic(n_screens=3), 4, 3.0, 16.0),
    "duct_dirichlet_P2": lambda: (W.surface_duct(n_screens=3, n_z=2048, n_modes=512, height=60.0, ext_m=4.0),
                                  2, 0.15, 4.0),
    "duct_neumann_P4": lambda: (W.surface_duct(n_screens=2, n_z=2048, n_modes=512, height=60.0, ext_m=4.0,
                                               bc=W.BC_NEUMANN), 4, 0.15, 4.0),
    "random_medium_P2": lambda: (W.random_medium(n_screens=3, n_z=1024, n_modes=256, height=125.0, seed=7,
                                                 n_gauss=12, x_len=30.0), 2, 3.0, 20.0),
}


# Fourier-continuation patches: partitions of unity that vary slowly on the
# Fresnel scale sqrt(lambda dx), which the method needs (it carries S^p
# along the rays)
FC_CASES = {
    "linear_caustic_P4": lambda: (W.linear_caustic(n_screens=3), 4, 3.0, 16.0),
    "duct_dirichlet_P4": lambda: (W.surface_duct(n_screens=3, n_z=2048, n_modes=512, height=60.0, ext_m=4.0),
                                  4, 2.0, 4.0),
    "duct_neumann_P2": lambda: (W.surface_duct(n_screens=2, n_z=2048, n_modes=512, height=60.0, ext_m=4.0,
                                               bc=W.BC_NEUMANN), 2, 2.0, 4.0),
    "random_medium_P2": lambda: (W.random_medium(n_screens=3, n_z=1024, n_modes=256, height=125.0, seed=7,
                                                 n_gauss=12, x_len=30.0), 2, 3.0, 20.0),
}
CASES = {"windowed": WINDOWED_CASES, "fc": FC_CASES}
_REF = {}


def reference(oracles, method, name):
    if (method, name) not in _REF:
        cfg, P, width, margin = CASES[method][name]()
        _REF[(method, name)] = oracles[method].run(cfg, W.incident_field(cfg), P, width, margin)
    return _REF[(method, name)]


def layout_info(oracles, method, cfg, P, width, margin):
    if method == "fc":
        return [(L["start"], L["sub"]["n_z"], L["sub"]["n_modes"]) for L in oracles["fc"].layout(cfg, P, width, margin)]
    return [(s, sub["n_z"], sub["n_modes"]) for s, sub in oracles["windowed"].layout(cfg, P, width, margin)]


@pytest.mark.parametrize("method,name", [(m, n) for m in ("fc", "windowed") for n in sorted(CASES[m])])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_patch_step_matches_oracle(env, method, name, prec):
    torch, pkg, oracles = env
    cfg, P, width, margin = CASES[method][name]()
    say(f"[patch] {method} {name} {prec} N={cfg['n_z']} P={P}")
    pp = pkg.PatchPlan(cfg, P, width, margin, precision=pkg.FP64 if prec == "fp64" else pkg.MIXED,
                       method=pkg.PATCH_FC if method == "fc" else pkg.PATCH_WINDOWED)
    assert pp.info() == layout_info(oracles, method, cfg, P, width, margin)
    u0 = W.incident_field(cfg)
    hist = pp.propagate(torch.from_numpy(u0).cuda(), 0, cfg["n_screens"]).cpu().numpy()
    ref = reference(oracles, method, name)
    err = rel(hist, ref)
    mx = float(np.max(np.abs(hist - ref)) / np.max(np.abs(ref)))
    say(f"[patch] {method} {name} {prec} rel_l2={err:.3e} max-norm={mx:.3e}")
    if prec == "fp64":
        assert err <= FP64_TOL
    else:
        assert err <= MIXED_TOL and err <= MIXED_REGRESSION
    assert torch.equal(pp.field().cpu(), torch.from_numpy(hist[-1]))
    pp.close()


@pytest.mark.parametrize("method", ["fc", "windowed"])
def test_resume_and_state(env, method):
    """Screens in two calls equal one call; continuing without a field on the
    right screen is refused."""
    torch, pkg, _ = env
    cfg, P, width, margin = CASES[method]["linear_caustic_P4"]()
    m = pkg.PATCH_FC if method == "fc" else pkg.PATCH_WINDOWED
    u0 = torch.from_numpy(W.incident_field(cfg)).cuda()
    pp = pkg.PatchPlan(cfg, P, width, margin, method=m)
    h_all = pp.propagate(u0, 0, 3)
    pp2 = pkg.PatchPlan(cfg, P, width, margin, method=m)
    h1 = pp2.propagate(u0, 0, 1)
    h2 = pp2.propagate(None, 1, 3)
    assert torch.equal(torch.cat([h1, h2]), h_all)
    with pytest.raises(pkg.SwkbError):
        pp2.propagate(None, 1, 2)
    pp.close()
    pp2.close()


@pytest.mark.parametrize("method", ["fc", "windowed"])
def test_graph_replays_equal_eager(env, method):
    """The grouped patch step (x-invariant medium, mixed) captured and replayed
    three times, with eager work between the replays, equals the eager run of
    the same plan (a second plan runs its own autotuner, whose timing-based
    choice of launch shapes may differ and change the rounding)."""
    torch, pkg, _ = env
    name = "duct_neumann_P2" if method == "fc" else "duct_neumann_P4"
    cfg, P, width, margin = CASES[method][name]()
    u0 = torch.from_numpy(W.incident_field(cfg)).cuda()
    pp = pkg.PatchPlan(cfg, P, width, margin, precision=pkg.MIXED,
                       method=pkg.PATCH_FC if method == "fc" else pkg.PATCH_WINDOWED)
    ref = pp.propagate(u0, 0, cfg["n_screens"]).cpu()
    pp.graphs(True)
    out = torch.empty((cfg["n_screens"], cfg["n_z"]), dtype=torch.complex128, device="cuda")
    for r in range(3):
        say(f"[patch] graph replay {r}")
        out.zero_()
        pp.propagate(u0, 0, cfg["n_screens"], out=out)  # the same arguments: one capture, then replays
        junk = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(out.cpu(), ref), r
    pp.graphs(False)
    pp.close()
