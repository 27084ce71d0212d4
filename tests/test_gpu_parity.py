"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

FP64 runs must match the oracle to a relative L2 error of 1e-10 over all
screens, mixed-precision runs to 1e-3.  Stage entry points are checked on
their own (modes, ray arrivals) so that a failure names its step.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-3
# Regression bound for the mixed path on the small cases below, whose
# measured errors against the oracle are 6e-7 .. 6e-6: FP32 rounding of the
# ray state, interpolation and phase.  A mistake in an FP32-only code path
# (an interpolation variable not advanced, a wrong coefficient) shows up here
# long before it reaches the 1e-3 bar.
MIXED_REGRESSION = 5e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def swkb():
    import paper_2301_03814_amd as pkg
    pkg.load()
    return pkg


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def small_random(n_screens=12, n_z=1024, n_modes=256, seed=7):
    cfg = W.random_medium(n_screens=n_screens, n_z=n_z, n_modes=n_modes, height=125.0, seed=seed,
                          n_gauss=12, x_len=n_screens * 10.0)
    return cfg


def small_duct(bc=W.BC_DIRICHLET, n_screens=4):
    return W.surface_duct(n_screens=n_screens, n_z=2048, n_modes=512, height=60.0, bc=bc, ext_m=4.0)


CASES = {
    "linear_caustic_N512": lambda: W.linear_caustic(),
    "random_medium_N1024": lambda: small_random(),
    "duct_dirichlet_N2048": lambda: small_duct(),
    "duct_neumann_N2048": lambda: small_duct(bc=W.BC_NEUMANN),
    "expgauss_N64_M2": lambda: W.with_overrides(
        W.linear_caustic(n_screens=3), n_z=64, n_modes=2, medium_kind=W.MEDIUM_EXPGAUSS,
        medium_params=[1.0, 0.05, 0.01, 32.0], launch_ext_cells=8, ray_stride=3),
    "expgauss_N64_allmodes": lambda: W.with_overrides(
        W.linear_caustic(n_screens=3), n_z=64, n_modes=64, medium_kind=W.MEDIUM_EXPGAUSS,
        medium_params=[1.0, 0.05, 0.01, 32.0], launch_ext_cells=8, ray_stride=1),
    "linear_M6_ragged": lambda: W.with_overrides(W.linear_caustic(n_screens=5), n_z=256, n_modes=6,
                                                 ray_stride=5, launch_ext_cells=37),
}


@pytest.fixture(scope="module")
def oracle_runs():
    import oracle
    oracle.build()
    cache = {}

    def get(name):
        if name not in cache:
            cfg = CASES[name]()
            u0 = W.incident_field(cfg)
            hist, cnt = oracle.run(cfg, u0)
            cache[name] = (cfg, u0, hist, cnt)
        return cache[name]
    return get


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("prop", ["auto", "recompute"])
def test_propagation_matches_oracle(torch_dev, swkb, oracle_runs, name, prec, prop):
    """auto = mode-function matrix for media that do not depend on x."""
    torch, dev = torch_dev
    cfg, u0, ref, cnt = oracle_runs(name)
    if prop == "recompute":
        if cfg["medium_kind"] == W.MEDIUM_GAUSSSUM:
            pytest.skip("x-varying medium: always recomputed")
        cfg = W.with_overrides(cfg, propagator=2)
    say(f"[parity] {name} {prec} {prop} N={cfg['n_z']} M={cfg['n_modes']} Q={cfg['n_screens']}")
    plan = swkb.Plan(cfg, precision=swkb.FP64 if prec == "fp64" else swkb.MIXED, device=dev)
    assert plan.uses_matrix == (prop == "auto" and cfg["medium_kind"] != W.MEDIUM_GAUSSSUM)
    hist = plan.propagate(torch.from_numpy(u0).to(dev), 0, cfg["n_screens"])
    got = hist.cpu().numpy()
    diag = plan.diagnostics()
    err = rel(got, ref)
    # screen by screen: max |difference| / max |oracle field| of that screen
    # (at least 1e-3 of the run's largest value: the beam may leave the domain)
    peak = np.abs(ref).max(axis=1)
    mx = float((np.abs(got - ref).max(axis=1) / np.maximum(peak, 1e-3 * peak.max())).max())
    say(f"[parity] {name} {prec} rel_l2={err:.3e} per-screen max-norm={mx:.3e} diag={diag} oracle={cnt}")
    assert err <= (FP64_TOL if prec == "fp64" else MIXED_TOL)
    assert mx <= (FP64_TOL if prec == "fp64" else MIXED_TOL)
    if prec == "mixed":
        assert err <= MIXED_REGRESSION
    assert diag["screens"] == cfg["n_screens"]
    if prec == "fp64":
        # discrete decisions (dead / caustic rays, folded modes) agree with the oracle
        assert diag["caustic_rays"] == cnt["caustic_rays"]
        assert diag["dead_rays"] == cnt["dead_rays"]
        assert diag["folded_modes"] == cnt["folded_modes"]
        assert diag["significant"] == cnt["significant"]
    # the last field equals the last history row
    assert torch.equal(plan.field(), hist[-1])
    plan.close()


@pytest.mark.parametrize("bc", [W.BC_PERIODIC, W.BC_DIRICHLET, W.BC_NEUMANN])
def test_stage_modes_match_oracle(torch_dev, swkb, bc):
    import oracle
    torch, dev = torch_dev
    for n_z, n_modes in ((64, 2), (512, 128), (4096, 1024), (16384, 4096)):
        cfg = W.with_overrides(W.linear_caustic(), n_z=n_z, n_modes=n_modes, bc=bc)
        rng = np.random.default_rng(n_z)
        u = rng.normal(size=n_z) + 1j * rng.normal(size=n_z)
        plan = swkb.Plan(cfg, device=dev)
        c = plan.stage_modes(torch.from_numpy(u).to(dev)).cpu().numpy()
        ref = oracle.modes(cfg, u)
        err = rel(c, ref)
        say(f"[modes] bc={bc} N={n_z} M={n_modes} rel={err:.2e}")
        assert err < 1e-13
        plan.close()


@pytest.mark.parametrize("name", ["linear_caustic_N512", "random_medium_N1024", "duct_dirichlet_N2048"])
def test_stage_rays_match_oracle(torch_dev, swkb, name):
    import oracle
    torch, dev = torch_dev
    cfg = CASES[name]()
    plan = swkb.Plan(cfg, device=dev)
    q = 1
    rays = {k: v.cpu().numpy() for k, v in plan.stage_rays(q).items()}
    M = cfg["n_modes"]
    for j in sorted({0, 1, M // 4, M // 2 - 1, M // 2, M // 2 + 3, 3 * M // 4, M - 1}):
        ref = oracle.march_mode(cfg, q, j)
        # liveness and caustics agree exactly; "dead at launch" and "dead on the
        # way" may trade places for a ray launched exactly at p^2 = p2_floor
        assert np.array_equal(rays["flag"][j] == 0, ref["flag"] == 0), f"liveness differs in mode {j}"
        assert np.array_equal(rays["flag"][j] == 3, ref["flag"] == 3), f"caustics differ in mode {j}"
        live = ref["flag"] == 0
        scale = max(1.0, abs(cfg["z_b"]))
        assert np.abs(rays["Z"][j][live] - ref["Z"][live]).max(initial=0) < 1e-12 * scale
        assert np.abs(rays["q"][j][live] - ref["q"][live]).max(initial=0) < 1e-12
        psi_scale = max(1.0, np.abs(ref["psi"][live]).max(initial=1.0))
        assert np.abs(rays["psi"][j][live] - ref["psi"][live]).max(initial=0) < 1e-12 * psi_scale
        assert np.abs(rays["a"][j][live] - ref["a"][live]).max(initial=0) < 1e-11
    say(f"[rays] {name} ok R={plan.num_rays}")
    plan.close()


# (launch extension, ray stride) -> rays per mode R on the 1024-point random
# medium: the FP32 Gaussian-sum march fills a mode's first R // 64 wavefronts
# and packs the last R mod 64 rays of several modes into shared wavefronts
# (64 // (R mod 64) modes each).  R = 192: no tail; 33: tails only, one mode
# per wavefront; 100: one full wavefront and a 36-ray tail; 70: ten 6-ray
# tails per wavefront, the last wavefront part-filled (256 modes); 129: one
# ray of each of 64 modes per wavefront.
RAY_LAYOUTS = {192: (250, 8), 33: (0, 32), 100: (280, 16), 70: (40, 16), 129: (0, 8)}


@pytest.mark.parametrize("R", sorted(RAY_LAYOUTS))
def test_mixed_march_ray_layouts(torch_dev, swkb, R):
    import oracle
    torch, dev = torch_dev
    ext, stride = RAY_LAYOUTS[R]
    cfg = W.with_overrides(small_random(n_screens=3), launch_ext_cells=ext, ray_stride=stride)
    say(f"[layout] R={R} ext={ext} stride={stride}")
    plan = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    assert plan.num_rays == R
    u0 = W.incident_field(cfg)
    # one screen: the diagnostics' ray counts (per-wavefront sums, per-mode
    # totals) equal the flags of that screen's rays
    plan.propagate(torch.from_numpy(u0).to(dev), 0, 1)
    d = plan.diagnostics()
    flag = plan.stage_rays(0)["flag"].cpu().numpy()
    assert d["caustic_rays"] == int((flag == 3).sum())
    assert d["dead_rays"] == int(((flag != 0) & (flag != 3)).sum())
    # the whole run against the oracle
    oracle.build()
    ref, cnt = oracle.run(cfg, u0)
    got = plan.propagate(torch.from_numpy(u0).to(dev), 0, cfg["n_screens"]).cpu().numpy()
    err = rel(got, ref)
    peak = np.abs(ref).max(axis=1)
    mx = float((np.abs(got - ref).max(axis=1) / np.maximum(peak, 1e-3 * peak.max())).max())
    say(f"[layout] R={R} rel_l2={err:.3e} per-screen max-norm={mx:.3e} caustic={d['caustic_rays']} "
        f"dead={d['dead_rays']}")
    assert err <= MIXED_REGRESSION
    assert mx <= MIXED_TOL
    plan.close()


def test_resume_and_determinism(torch_dev, swkb):
    """Resuming from screen q equals an uninterrupted run bit for bit, and
    two runs are bitwise identical (fixed-order reductions, no atomics on
    the field)."""
    torch, dev = torch_dev
    cfg = small_random()
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    Q = cfg["n_screens"]
    a = swkb.Plan(cfg, device=dev)
    full = a.propagate(u0, 0, Q)
    b = swkb.Plan(cfg, device=dev)
    h1 = b.propagate(u0, 0, 5)
    h2 = b.propagate(None, 5, Q)
    assert torch.equal(torch.cat([h1, h2]), full)
    again = a.propagate(u0, 0, Q)
    assert torch.equal(again, full)
    # restart from a stored screen through u_in
    c = swkb.Plan(cfg, device=dev)
    h3 = c.propagate(full[6].contiguous(), 7, Q)
    assert torch.equal(h3, full[7:])
    for p in (a, b, c):
        p.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_overlapped_march_equals_serial(torch_dev, swkb, prec):
    """For a medium that changes with x the march of screen q + 1 runs on a
    second stream while screen q is summed (two record slots).  With
    profiling on, every kernel runs on the caller's stream one after
    another; both orders give the same field bit for bit, also when single
    screens are stepped one call at a time and the same screen is
    propagated twice."""
    torch, dev = torch_dev
    cfg = small_random()
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    Q = cfg["n_screens"]
    p = swkb.Plan(cfg, precision=swkb.FP64 if prec == "fp64" else swkb.MIXED, device=dev)
    fast = p.propagate(u0, 0, Q)
    p.profile(True)
    slow = p.propagate(u0, 0, Q)
    t = p.profile_read()
    p.profile(False)
    assert t["march_launches"] == Q and t["superpose_launches"] == Q
    assert torch.equal(fast, slow)
    steps = [p.propagate(u0 if q == 0 else None, q, q + 1) for q in range(Q)]
    assert torch.equal(torch.cat(steps), fast)
    again = p.propagate(fast[2].contiguous(), 3, 4)  # screen 3 again: its rays are reused
    assert torch.equal(again[0], fast[3])
    p.close()


@pytest.mark.parametrize("name,prop", [("random_medium_N1024", "auto"), ("duct_dirichlet_N2048", "auto"),
                                       ("linear_caustic_N512", "recompute")])
def test_graph_replay_equals_eager(torch_dev, swkb, name, prop):
    """Screen ranges captured into HIP graphs: every replay (with eager work
    and synchronisations in between) gives the eager fields bit for bit, for
    an x-varying medium (two streams), the mode-function matrix and rays
    marched once; chained ranges continue from the plan's field."""
    torch, dev = torch_dev
    cfg = CASES[name]()
    if prop == "recompute":
        cfg = W.with_overrides(cfg, propagator=2)
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    Q = cfg["n_screens"]
    p = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    other = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    eager = p.propagate(u0, 0, Q).clone()
    p.graphs(True)
    out = torch.empty_like(eager)
    for rep in range(3):
        out.zero_()
        p.propagate(u0, 0, Q, out=out)
        assert torch.equal(out, eager), f"replay {rep} differs"
        assert p.current_screen == Q
        other.propagate(u0, 0, 3)  # eager work of another plan between replays
        torch.cuda.synchronize()
    # two chained ranges, each captured once and replayed once
    qs = Q // 2
    h1, h2 = torch.empty_like(eager[:qs]), torch.empty_like(eager[qs:])
    for rep in range(2):
        p.propagate(u0, 0, qs, out=h1)
        p.propagate(None, qs, Q, out=h2)
        torch.cuda.synchronize()
        assert torch.equal(torch.cat([h1, h2]), eager)
    p.graphs(False)
    assert torch.equal(p.propagate(u0, 0, Q), eager)
    p.close()
    other.close()


def test_zero_screens_and_state_errors(torch_dev, swkb):
    torch, dev = torch_dev
    cfg = W.linear_caustic()
    plan = swkb.Plan(cfg, device=dev)
    with pytest.raises(swkb.SwkbError):
        plan.field()
    with pytest.raises(swkb.SwkbError):
        plan.propagate(None, 0, 2)  # no field yet
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    h = plan.propagate(u0, 3, 3)
    assert h.shape == (0, cfg["n_z"])
    assert torch.equal(plan.field(), u0) and plan.current_screen == 3
    with pytest.raises(swkb.SwkbError):
        plan.propagate(u0, 0, cfg["n_screens"] + 1)
    plan.close()


def test_caustic_is_reported(torch_dev, swkb):
    """A screen much wider than the caustic-free spacing makes significant
    modes cross; the library drops those rays and reports SWKB_ERR_CAUSTIC."""
    torch, dev = torch_dev
    cfg = W.with_overrides(W.linear_caustic(n_screens=1), dx=300.0, rk4_steps=64, absorber_top=0.0,
                           absorber_bot=0.0, caustic_tol=1e-3)
    plan = swkb.Plan(cfg, device=dev)
    plan.propagate(torch.from_numpy(W.incident_field(cfg)).to(dev), 0, 1)
    d = plan.diagnostics()
    assert d["significant"] > 0
    with pytest.raises(swkb.SwkbError) as ei:
        plan.diagnostics(raise_on_caustic=True)
    assert ei.value.status == swkb.swkb.SWKB_ERR_CAUSTIC
    plan.close()


def test_mixed_medium_table_and_fallback(torch_dev, swkb, oracle_runs):
    """The mixed Gaussian-sum march reads eps and its z-derivatives from a
    per-screen FP64-built table (cubic Hermite in z) and evaluates the bump
    sum directly for heights outside it.  In this case steep rays leave the
    table, so both paths run; the result stays within the FP32 rounding
    level of the FP64 run and within the mixed bar of the oracle."""
    torch, dev = torch_dev
    cfg, u0, ref, _ = oracle_runs("random_medium_N1024")
    u0_d = torch.from_numpy(u0).to(dev)
    res = {}
    for prec in (swkb.FP64, swkb.MIXED):
        plan = swkb.Plan(cfg, precision=prec, device=dev)
        res[prec] = (plan.propagate(u0_d, 0, cfg["n_screens"]).cpu().numpy(), plan.diagnostics())
        plan.close()
    (h64, d64), (h32, d32) = res[swkb.FP64], res[swkb.MIXED]
    say(f"[table] fp64 diag={d64}")
    say(f"[table] mixed diag={d32}")
    assert d64["table_evals"] == 0
    assert d32["table_evals"] > 0 and d32["medium_evals"] > 0
    err = rel(h32, h64)
    say(f"[table] mixed vs fp64 rel_l2={err:.3e}, mixed vs oracle {rel(h32, ref):.3e}")
    assert err <= 1e-4
    assert rel(h32, ref) <= MIXED_TOL


def test_mixed_direct_evaluation_when_table_too_fine(torch_dev, swkb, oracle_runs):
    """A bump much narrower than the others would make the table too fine;
    the mixed march then evaluates the bump sum directly at every stage."""
    torch, dev = torch_dev
    cfg, u0, _, _ = oracle_runs("random_medium_N1024")
    mp = np.concatenate([cfg["medium_params"], [0.0, 1e-4, 60.0, 60.0]])  # zero amplitude, width 1e-4
    mp[0] += 1
    cfg = W.with_overrides(cfg, medium_params=mp)
    u0_d = torch.from_numpy(u0).to(dev)
    res = {}
    for prec in (swkb.FP64, swkb.MIXED):
        plan = swkb.Plan(cfg, precision=prec, device=dev)
        res[prec] = (plan.propagate(u0_d, 0, cfg["n_screens"]).cpu().numpy(), plan.diagnostics())
        plan.close()
    (h64, _), (h32, d32) = res[swkb.FP64], res[swkb.MIXED]
    err = rel(h32, h64)
    say(f"[table] direct mixed diag={d32} vs fp64 rel_l2={err:.3e}")
    assert d32["table_evals"] == 0 and d32["medium_evals"] > 0
    assert err <= 1e-4


@pytest.mark.slow
def test_random_medium_full_size_sampled_screens(torch_dev, swkb):
    """Full random-medium workload (N = 8192, M = 2048, 400 screens) in the
    launch configuration the benchmark times: sampled screens, each started
    from the workload's seeded incident beam, by the GPU and by the oracle;
    the mixed run is held against the FP64 run over all 400 screens."""
    import oracle
    torch, dev = torch_dev
    cfg = W.random_medium()
    u0 = W.incident_field(cfg)
    u0_d = torch.from_numpy(u0).to(dev)
    Q = cfg["n_screens"]
    p64 = swkb.Plan(cfg, precision=swkb.FP64, device=dev)
    h64 = p64.propagate(u0_d, 0, Q)
    d64 = p64.diagnostics()
    say(f"[full] fp64 done diag={d64}")
    hist = h64.cpu().numpy()
    for q in (0, 211):
        got = hist[q] if q == 0 else p64.propagate(u0_d, q, q + 1)[0].cpu().numpy()
        ref, cnt = oracle.screen(cfg, q, u0)
        err = rel(got, ref)
        say(f"[full] screen {q} fp64 vs oracle rel={err:.3e}")
        assert err <= FP64_TOL
    p32 = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    h32 = p32.propagate(u0_d, 0, Q).cpu().numpy()
    d32 = p32.diagnostics()
    err = rel(h32, hist)
    say(f"[full] mixed vs fp64 over {Q} screens rel={err:.3e} diag={d32}")
    assert d32["table_evals"] > 0
    assert err <= MIXED_TOL
    assert d64["significant"] == 0
    p64.close()
    p32.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_random_medium_full_size_reflection(torch_dev, swkb, prec):
    """Full-size random medium (N = 8192, M = 2048, 200 bumps over the whole
    height, absorbers of equal thickness at both ends): the bumps reflected
    about the middle of the domain and a band-limited field (modes -M/2 + 1
    .. M/2 - 1) reflected with them give, screen by screen, the reflected
    output.  This holds at any size, so it checks the full-size launch
    configuration everywhere, not only on the screens the oracle samples."""
    import oracle
    torch, dev = torch_dev
    cfg = W.random_medium()
    N, M = cfg["n_z"], cfg["n_modes"]
    H2 = 2.0 * cfg["z_a"] + (cfg["z_b"] - cfg["z_a"])
    assert (oracle.num_rays(cfg) - 1) * cfg["ray_stride"] == N + 2 * cfg["launch_ext_cells"]
    assert cfg["absorber_bot"] == cfg["absorber_top"]
    refl = W.with_overrides(cfg, medium_params=cfg["medium_params"].copy())
    refl["medium_params"][4::4] = H2 - refl["medium_params"][4::4]
    rng = np.random.default_rng(17)
    spec = np.zeros(N, complex)
    n = np.arange(-M // 2 + 1, M // 2)
    spec[n % N] = rng.normal(size=n.size) + 1j * rng.normal(size=n.size)
    v = np.fft.ifft(spec) * N
    m = (-np.arange(N)) % N
    P = swkb.FP64 if prec == "fp64" else swkb.MIXED
    pa = swkb.Plan(cfg, precision=P, device=dev)
    pb = swkb.Plan(refl, precision=P, device=dev)
    # measured: FP64 1.6e-14 and 7.3e-15; mixed 2.4e-6 and 4.8e-7 (its medium
    # table's nodes do not reflect onto each other, so its errors differ)
    bound = FP64_TOL if prec == "fp64" else MIXED_REGRESSION
    for q in (0, 211):
        say(f"[reflect] {prec} screen {q}")
        out = pa.propagate(torch.from_numpy(v).to(dev), q, q + 1)[0].cpu().numpy()
        out_r = pb.propagate(torch.from_numpy(v[m].copy()).to(dev), q, q + 1)[0].cpu().numpy()
        err = rel(out_r, out[m])
        say(f"[reflect] {prec} screen {q} rel={err:.3e}")
        assert err <= bound
    pa.close()
    pb.close()


def test_random_medium_full_size_batch(torch_dev, swkb):
    """Four sources (heights 350-650) through the full-size random medium in
    one batched propagation, the launch configuration the benchmark times
    (one march per screen, the several-field sum): over the first 40 screens
    each field equals its own single-field run, and field 0 stays within
    the mixed bound of the FP64 run."""
    torch, dev = torch_dev
    cfg = W.random_medium()
    Q, B = 40, 4
    srcs = []
    for b in range(B):
        c = W.with_overrides(cfg)
        c["source"] = dict(cfg["source"], z0=350.0 + 100.0 * b)
        srcs.append(W.incident_field(c))
    U0 = np.stack(srcs)
    say(f"[full-batch] {B} fields, {Q} screens")
    pb = swkb.Plan(W.with_overrides(cfg, max_batch=B), precision=swkb.MIXED, device=dev)
    hist, _ = pb.propagate_batch(torch.from_numpy(U0).to(dev), 0, Q)
    hist = hist.cpu().numpy()
    pb.close()
    ps = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    for b in range(B):
        ref = ps.propagate(torch.from_numpy(U0[b]).to(dev), 0, Q).cpu().numpy()
        err = rel(hist[:, b, :], ref)
        say(f"[full-batch] field {b} batch vs single rel={err:.2e}")
        assert err <= 2e-5  # measured 3.0e-6 .. 4.0e-6 (FP32 rounding of two sum kernels)
    ps.close()
    p64 = swkb.Plan(cfg, precision=swkb.FP64, device=dev)
    ref64 = p64.propagate(torch.from_numpy(U0[0]).to(dev), 0, Q).cpu().numpy()
    err = rel(hist[:, 0, :], ref64)
    say(f"[full-batch] field 0 batch vs fp64 rel={err:.2e}")
    assert err <= MIXED_REGRESSION
    p64.close()


def test_maximum_grid_stages_match_oracle(torch_dev, swkb):
    """The largest grid one plan takes (N = 32768, M = 8192; the 0-600 m
    duct over its Dirichlet ground, FFT length 65536): mode amplitudes of a
    random field against the oracle's direct DFT, and the ray arrivals of
    sampled modes (the evanescent edges, the middle, a quarter) against the
    oracle's march of those modes."""
    import oracle
    torch, dev = torch_dev
    cfg = W.surface_duct(n_screens=2, n_z=32768, n_modes=8192, height=600.0)
    N, M = cfg["n_z"], cfg["n_modes"]
    say(f"[max] stages N={N} M={M}")
    rng = np.random.default_rng(32768)
    u = rng.normal(size=N) + 1j * rng.normal(size=N)
    plan = swkb.Plan(cfg, precision=swkb.FP64, device=dev)
    c = plan.stage_modes(torch.from_numpy(u).to(dev)).cpu().numpy()
    err = rel(c, oracle.modes(cfg, u))
    say(f"[max] modes rel={err:.2e}")
    assert err < 1e-13
    q = 1
    rays = plan.stage_rays(q)
    for j in (0, 1, M // 4, M // 2 - 1, M // 2, 3 * M // 4, M - 1):
        got = {k: v[j].cpu().numpy() for k, v in rays.items()}
        ref = oracle.march_mode(cfg, q, j)
        assert np.array_equal(got["flag"] == 0, ref["flag"] == 0), f"liveness differs in mode {j}"
        assert np.array_equal(got["flag"] == 3, ref["flag"] == 3), f"caustics differ in mode {j}"
        live = ref["flag"] == 0
        assert np.abs(got["Z"][live] - ref["Z"][live]).max(initial=0) < 1e-12 * cfg["z_b"]
        assert np.abs(got["q"][live] - ref["q"][live]).max(initial=0) < 1e-12
        psi_scale = max(1.0, np.abs(ref["psi"][live]).max(initial=1.0))
        assert np.abs(got["psi"][live] - ref["psi"][live]).max(initial=0) < 1e-12 * psi_scale
        assert np.abs(got["a"][live] - ref["a"][live]).max(initial=0) < 1e-11
    say(f"[max] rays ok R={plan.num_rays}")
    del rays
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_maximum_grid_homogeneous_is_exact(torch_dev, swkb, prec):
    """eps = 1 on the largest grid (N = 32768, M = 8192, periodic): rays are
    straight and the amplitude is 1, so one screen of 100 m at 6 GHz is the
    exact propagator of the kept plane waves; the input is a random field
    over every kept mode except -M/2.  The launch extension (40 m) exceeds
    the steepest kept mode's drift over the screen (36 m), so every grid
    point has rays of every mode on both sides."""
    torch, dev = torch_dev
    cfg = W.with_overrides(W.surface_duct(n_screens=2, n_z=32768, n_modes=8192, height=600.0, ext_m=40.0),
                           bc=W.BC_PERIODIC, medium_kind=W.MEDIUM_LINEAR, medium_params=[1.0, 0.0],
                           eps_ref=1.0, absorber_bot=0.0, absorber_top=0.0)
    N, M = cfg["n_z"], cfg["n_modes"]
    say(f"[max] homogeneous {prec} N={N} M={M}")
    n = np.arange(-M // 2 + 1, M // 2)
    rng = np.random.default_rng(6)
    spec = np.zeros(N, complex)
    spec[n % N] = rng.normal(size=n.size) + 1j * rng.normal(size=n.size)
    v = np.fft.ifft(spec) * N
    xi = 2 * np.pi * n / (cfg["k"] * (cfg["z_b"] - cfg["z_a"]))
    assert (1.0 - xi ** 2).min() > cfg["p2_floor"]  # every kept mode propagates
    h = (cfg["z_b"] - cfg["z_a"]) / N
    assert cfg["dx"] * xi.max() / np.sqrt(1.0 - xi.max() ** 2) < cfg["launch_ext_cells"] * h
    out_spec = np.zeros(N, complex)
    out_spec[n % N] = spec[n % N] * np.exp(1j * cfg["k"] * np.sqrt(1.0 - xi ** 2) * cfg["dx"])
    exact = np.fft.ifft(out_spec) * N
    plan = swkb.Plan(cfg, precision=swkb.FP64 if prec == "fp64" else swkb.MIXED, device=dev)
    out = plan.propagate(torch.from_numpy(v).to(dev), 0, 1)[0].cpu().numpy()
    err = rel(out, exact)
    say(f"[max] homogeneous {prec} rel={err:.3e}")
    # measured: FP64 6.5e-13 (phases of ~1.2e4 rad), mixed 3.6e-7
    assert err <= (FP64_TOL if prec == "fp64" else MIXED_REGRESSION)
    plan.close()


@pytest.mark.slow
def test_surface_duct_full_size_sampled_screen(torch_dev, swkb):
    """Full surface duct (N = 16384, M = 4096, 1000 screens, Dirichlet ground)
    through the mode-function matrix: screen 500, started from the
    workload's seeded incident beam, by the GPU and by the oracle; the mixed
    run held against FP64."""
    import oracle
    torch, dev = torch_dev
    cfg = W.surface_duct()
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    Q = cfg["n_screens"]
    p64 = swkb.Plan(cfg, precision=swkb.FP64, device=dev)
    assert p64.uses_matrix
    h64 = p64.propagate(u0, 0, Q)
    sel = h64[::25].cpu().numpy()
    q = 500
    uin = W.incident_field(cfg)
    del h64
    got = p64.propagate(torch.from_numpy(uin).to(dev), q, q + 1)[0].cpu().numpy()
    p64.close()
    ref, _ = oracle.screen(cfg, q, uin)
    err = rel(got, ref)
    say(f"[duct] screen {q} fp64 vs oracle rel={err:.3e}")
    assert err <= FP64_TOL
    p32 = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    h32 = p32.propagate(u0, 0, Q)[::25].cpu().numpy()
    err = rel(h32, sel)
    say(f"[duct] mixed vs fp64 every 25th screen rel={err:.3e}")
    assert err <= MIXED_TOL
    p32.close()


def _sources(cfg, B):
    """B different incident beams on the same screen grid (heights, tilts)."""
    out = []
    L = cfg["z_b"] - cfg["z_a"]
    for b in range(B):
        c = W.with_overrides(cfg)
        c["source"] = dict(z0=cfg["z_a"] + L * (0.3 + 0.4 * b / max(1, B - 1)),
                           width=cfg["source"]["width"] * (1.0 + 0.25 * b),
                           xi0=cfg["source"]["xi0"] + 0.01 * b)
        out.append(W.incident_field(c))
    return np.stack(out)


@pytest.mark.parametrize("name,prop", [("random_medium_N1024", "auto"), ("linear_caustic_N512", "auto"),
                                       ("linear_caustic_N512", "recompute"), ("duct_dirichlet_N2048", "auto")])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_equals_separate_runs(torch_dev, swkb, name, prop, prec):
    """Several sources through one plan at once (shared rays; for x-invariant
    media one complex GEMM per screen) equal separate single-field runs."""
    torch, dev = torch_dev
    B = 3
    cfg = W.with_overrides(CASES[name](), max_batch=4, propagator=2 if prop == "recompute" else 0)
    P = swkb.FP64 if prec == "fp64" else swkb.MIXED
    U0 = _sources(cfg, B)
    plan = swkb.Plan(cfg, precision=P, device=dev)
    u_keep = torch.from_numpy(U0[0]).to(dev)
    plan.propagate(u_keep, 0, 2)
    f_before = plan.field()
    Q = cfg["n_screens"]
    hist, last = plan.propagate_batch(torch.from_numpy(U0).to(dev), 0, Q)
    assert torch.equal(plan.field(), f_before) and plan.current_screen == 2  # single-field state untouched
    hist = hist.cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 2e-5
    for b in range(B):
        single = swkb.Plan(cfg, precision=P, device=dev)
        ref = single.propagate(torch.from_numpy(U0[b]).to(dev), 0, Q).cpu().numpy()
        err = rel(hist[:, b, :], ref)
        say(f"[batch] {name} {prop} {prec} field {b} rel={err:.2e} matrix={plan.uses_matrix}")
        assert err <= tol
        single.close()
    assert torch.equal(last, torch.from_numpy(hist[-1]).to(dev))
    # one field through the batch entry point
    h1, _ = plan.propagate_batch(torch.from_numpy(U0[1:2]).to(dev), 0, Q)
    assert rel(h1.cpu().numpy()[:, 0, :], hist[:, 1, :]) <= tol
    plan.close()


@pytest.mark.parametrize("name", ["random_medium_N1024", "linear_caustic_N512", "duct_dirichlet_N2048"])
def test_fields_between_screens_match_oracle(torch_dev, swkb, name):
    """Stations x_q + i dx/S: the oracle runs the screen step with width
    i dx/S and i RK4 steps from the same field (the seeded incident beam
    handed to screen q)."""
    import oracle
    torch, dev = torch_dev
    cfg = CASES[name]()
    S = cfg["rk4_steps"]
    q = 2
    plan = swkb.Plan(cfg, device=dev)
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    hist = plan.propagate(u0, 0, q + 1)
    uq = u0  # the seeded incident beam, handed to screen q
    st = [1, S // 2, S]
    got = plan.stations(uq, q, st).cpu().numpy()
    for k, i in enumerate(st):
        c_i = W.with_overrides(cfg, dx=i * (cfg["dx"] / S), rk4_steps=i)
        c_i["x0"] = cfg["x0"] + q * cfg["dx"] - q * c_i["dx"]  # screen q of c_i sits at x_q
        ref, _ = oracle.screen(c_i, q, uq.cpu().numpy())
        err = rel(got[k], ref)
        say(f"[stations] {name} i={i} rel={err:.2e}")
        assert err <= FP64_TOL
    # the last station is the next screen
    assert rel(got[-1], plan.propagate(uq, q, q + 1)[0].cpu().numpy()) <= 1e-12
    # the plan's own propagation is unaffected afterwards
    again = plan.propagate(u0, 0, q + 1)
    assert torch.equal(again, hist)
    plan.close()


@pytest.mark.parametrize("name", ["random_medium_N1024", "linear_caustic_N512", "duct_dirichlet_N2048"])
def test_fields_between_screens_mixed(torch_dev, swkb, name):
    """Stations in the mixed path: the one-field FP32 sum takes each mode's
    coefficient in polar form and adds the station's own range phase (not the
    screen's); held against the FP64 stations and the oracle.  The
    x-invariant duct runs its stations through the recomputing sum although
    the plan itself uses the mode-function matrix."""
    import oracle
    torch, dev = torch_dev
    cfg = CASES[name]()
    S = cfg["rk4_steps"]
    q = 2
    p64 = swkb.Plan(cfg, precision=swkb.FP64, device=dev)
    p32 = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    hist = p64.propagate(u0, 0, q + 1)
    own32 = p32.propagate(u0, 0, q + 1)
    uq = u0  # the seeded incident beam, handed to screen q
    st = [1, S // 2, S]
    g64 = p64.stations(uq, q, st).cpu().numpy()
    g32 = p32.stations(uq, q, st).cpu().numpy()
    for k, i in enumerate(st):
        c_i = W.with_overrides(cfg, dx=i * (cfg["dx"] / S), rk4_steps=i)
        c_i["x0"] = cfg["x0"] + q * cfg["dx"] - q * c_i["dx"]
        ref, _ = oracle.screen(c_i, q, uq.cpu().numpy())
        e64, eor = rel(g32[k], g64[k]), rel(g32[k], ref)
        say(f"[stations] {name} mixed i={i} vs fp64 {e64:.2e} vs oracle {eor:.2e}")
        assert e64 <= 1e-4 and eor <= 1e-4
    # the mixed plan's own propagation is unaffected afterwards
    assert torch.equal(p32.propagate(u0, 0, q + 1), own32)
    p64.close()
    p32.close()


def _np_modal(cfg, u0, xs):
    """numpy separation of variables on the same grid (mirror: doubled grid,
    reflected eps, odd/even extension) -- independent of the GPU solver."""
    import oracle
    from refs import modal_reference
    N, L = cfg["n_z"], cfg["z_b"] - cfg["z_a"]
    if cfg["bc"] == W.BC_PERIODIC:
        z = W.grid(cfg)
        e, _, _ = oracle.medium(cfg, 0.0, z)
        return modal_reference(z, L, cfg["k"], e, u0, xs)
    h = L / N
    z = cfg["z_a"] - L + h * np.arange(2 * N)
    e, _, _ = oracle.medium(cfg, 0.0, z)  # the oracle reflects eps below z_a
    sgn = -1.0 if cfg["bc"] == W.BC_DIRICHLET else 1.0
    v = np.zeros(2 * N, complex)
    v[N:] = u0
    v[N - np.arange(1, N)] = sgn * u0[1:]
    if cfg["bc"] == W.BC_DIRICHLET:
        v[N] = 0.0
    return modal_reference(z, 2 * L, cfg["k"], e, v, xs)[:, N:]


@pytest.mark.parametrize("name", ["linear_caustic_N512", "duct_dirichlet_N1024", "duct_neumann_N1024"])
def test_gpu_modal_reference_matches_numpy(torch_dev, swkb, name):
    """The GPU separation-of-variables solver (rocSOLVER) against numpy eigh."""
    torch, dev = torch_dev
    if name == "linear_caustic_N512":
        cfg = W.linear_caustic()
    else:
        bc = W.BC_DIRICHLET if "dirichlet" in name else W.BC_NEUMANN
        cfg = W.surface_duct(n_screens=4, n_z=1024, n_modes=256, height=60.0, bc=bc, ext_m=4.0)
    u0 = W.incident_field(cfg)
    xs = [cfg["dx"], 3 * cfg["dx"]]
    got = swkb.modal_reference(cfg, torch.from_numpy(u0).to(dev), xs).cpu().numpy()
    ref = _np_modal(cfg, u0, xs)
    err = rel(got, ref)
    say(f"[modal] {name} rel={err:.2e}")
    assert err < 1e-9


def test_swkb_accuracy_against_gpu_modal_reference(torch_dev, swkb):
    """Method accuracy (not parity): S-WKB through a 2 km surface duct at 6 GHz
    (N = 4096, M = 1024, 20 screens of 100 m, Dirichlet ground, no absorber)
    against the exact separation-of-variables solution on the GPU."""
    torch, dev = torch_dev
    cfg = W.surface_duct(n_screens=20, n_z=4096, n_modes=1024, height=75.0, ext_m=10.0)
    cfg = W.with_overrides(cfg, absorber_top=0.0)
    u0 = W.incident_field(cfg)
    u0d = torch.from_numpy(u0).to(dev)
    plan = swkb.Plan(cfg, device=dev)
    hist = plan.propagate(u0d, 0, cfg["n_screens"]).cpu().numpy()
    xs = cfg["dx"] * np.arange(1, cfg["n_screens"] + 1)
    ref = swkb.modal_reference(cfg, u0d, xs).cpu().numpy()
    errs = [rel(hist[i], ref[i]) for i in range(len(xs))]
    say(f"[accuracy] duct 2 km: per-screen rel err first {errs[0]:.2e} last {errs[-1]:.2e} all {rel(hist, ref):.2e}")
    # measured 8.9e-5 (4e-7 after one screen, 2.2e-4 after twenty)
    assert rel(hist, ref) < 4e-4
    assert errs[0] < 1e-5
    plan.close()


def test_mixed_amplitude_near_turning_points(torch_dev, swkb):
    """The mixed path accumulates the ray tube (Z_s, Q_s) in FP64 from FP32
    RK4 increments and forms the amplitude sqrt(p0 / (p Z_s)) with its Z_s
    factor in FP64 (stored in FP32).  On the linear caustic, rays whose
    vertical slowness changes sign within the screen (they pass a turning
    point) and all live rays keep amplitudes close to the oracle's FP64
    march; the bounds hold the FP32-ray-state level."""
    import oracle
    torch, dev = torch_dev
    cfg = CASES["linear_caustic_N512"]()
    plan = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    q = 1
    rays = {k: v.cpu().numpy() for k, v in plan.stage_rays(q).items()}
    worst_turn, worst_all, n_turn = 0.0, 0.0, 0
    for j in range(cfg["n_modes"]):
        ref = oracle.march_mode(cfg, q, j)
        live = (ref["flag"] == 0) & (rays["flag"][j] == 0)
        if not live.any():
            continue
        err = np.abs(rays["a"][j][live] - ref["a"][live]) / np.abs(ref["a"][live])
        worst_all = max(worst_all, float(err.max()))
        # launched with q = xi_n; turned when the arrival slowness has the other sign
        xi_n = 2.0 * math.pi * (j - cfg["n_modes"] // 2) / (cfg["k"] * (cfg["z_b"] - cfg["z_a"]))  # P h = L
        turned = live & (ref["q"] * xi_n < 0.0)
        if turned.any():
            n_turn += int(turned.sum())
            e = np.abs(rays["a"][j][turned] - ref["a"][turned]) / np.abs(ref["a"][turned])
            worst_turn = max(worst_turn, float(e.max()))
    say(f"[rays] mixed amplitude: {n_turn} turning rays, max rel err {worst_turn:.2e}; all live rays {worst_all:.2e}")
    assert n_turn > 0
    assert worst_turn <= 1e-4
    assert worst_all <= 1e-4
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name,B", [("linear_caustic_N512", 9), ("linear_caustic_N512", 33),
                                    ("linear_caustic_N512", 70), ("expgauss_N64_M2", 5)])
def test_batch_product_shapes_equal_separate_runs(torch_dev, swkb, name, B, prec):
    """The batched product on the matrix cores in every launch shape: one or
    several column tiles (16 fields each in FP32, 8 in FP64), several passes
    over T (more than 64 resp. 32 fields), a two-mode problem (one mode group
    of one mode pair).  Every field equals its own single-field run."""
    torch, dev = torch_dev
    cfg = W.with_overrides(CASES[name](), max_batch=B)
    assert cfg["medium_kind"] != W.MEDIUM_GAUSSSUM
    P = swkb.FP64 if prec == "fp64" else swkb.MIXED
    Q = min(cfg["n_screens"], 6)
    rng = np.random.default_rng(B)
    base = _sources(cfg, 3)
    U0 = np.stack([base[b % 3] * np.exp(2j * np.pi * rng.uniform()) * rng.uniform(0.5, 2.0) for b in range(B)])
    plan = swkb.Plan(cfg, precision=P, device=dev)
    assert plan.uses_matrix
    hist, last = plan.propagate_batch(torch.from_numpy(U0).to(dev), 0, Q)
    hist = hist.cpu().numpy()
    single = swkb.Plan(W.with_overrides(cfg, max_batch=1), precision=P, device=dev)
    tol = 1e-12 if prec == "fp64" else 2e-5
    worst = 0.0
    for b in range(B):
        ref = single.propagate(torch.from_numpy(U0[b]).to(dev), 0, Q).cpu().numpy()
        worst = max(worst, rel(hist[:, b, :], ref))
    say(f"[batch-shapes] {name} B={B} {prec}: worst field vs single run {worst:.2e}")
    assert worst <= tol
    assert torch.equal(last, torch.from_numpy(hist[-1]).to(dev))
    plan.close()
    single.close()
