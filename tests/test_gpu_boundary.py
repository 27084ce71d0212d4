"""GPU tests of the C ABI's contract beyond the numerics: a batch of one field
on a plan without a batch buffer, HIP-graph replays after calls that change
the plan's rays or field buffer, the single-stream rule (SWKB_ERR_BUSY), the
field of any screen (swkb_field with keep_history), the report of a
significant evanescent mode (SWKB_ERR_EVANESCENT) and the diagnostics of a
batch against those of one field."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


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


def duct(bc=W.BC_DIRICHLET, n_screens=6, **kw):
    return W.with_overrides(W.surface_duct(n_screens=n_screens, n_z=2048, n_modes=512, height=60.0, bc=bc,
                                           ext_m=4.0), **kw)


@pytest.mark.parametrize("bc", [W.BC_DIRICHLET, W.BC_NEUMANN, W.BC_PERIODIC])
@pytest.mark.parametrize("prop", [0, 2])
def test_batch_of_one_on_default_plan_equals_propagate(torch_dev, swkb, bc, prop):
    """max_batch = 1 (no batch buffer): a batch of one field uses the plan's
    own field buffer, so the mirror extension of the next screen's FFT reads
    a field no other kernel is writing; the result equals swkb_propagate bit
    for bit over several screens."""
    torch, dev = torch_dev
    cfg = duct(bc=bc, propagator=prop)
    Q = cfg["n_screens"]
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    say(f"[batch1] bc={bc} prop={prop} Q={Q}")
    for prec in (swkb.FP64, swkb.MIXED):
        ref = swkb.Plan(cfg, precision=prec, device=dev)
        want = ref.propagate(u0, 0, Q)
        plan = swkb.Plan(cfg, precision=prec, device=dev)
        for rep in range(2):
            hist, last = plan.propagate_batch(u0.reshape(1, -1).contiguous(), 0, Q)
            assert torch.equal(hist[:, 0, :], want), f"batch of one differs (prec {prec}, rep {rep})"
            assert torch.equal(last[0], want[-1])
        # the single-field state was consumed: no current field
        assert plan.current_screen == -1
        ref.close()
        plan.close()


@pytest.mark.parametrize("name", ["linear_recompute", "duct_matrix", "random"])
def test_graph_replay_after_stations_and_batch(torch_dev, swkb, name):
    """With graphs on: propagate (captured), fields between screens (which
    march station rays into the plan's ray slot), propagate again (replayed),
    a batch of one field (which swaps the plan's field buffer), propagate
    again: every propagate equals the eager result bit for bit."""
    torch, dev = torch_dev
    if name == "linear_recompute":
        cfg = W.with_overrides(W.linear_caustic(n_screens=6), propagator=2, max_batch=2)
    elif name == "duct_matrix":
        cfg = duct(max_batch=2)
    else:
        cfg = W.with_overrides(W.random_medium(n_screens=6, n_z=1024, n_modes=256, height=125.0, seed=7,
                                               n_gauss=12, x_len=60.0), max_batch=2)
    Q = cfg["n_screens"]
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    eager_plan = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    eager = eager_plan.propagate(u0, 0, Q).clone()
    eager_plan.close()
    plan = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    plan.graphs(True)
    out = torch.empty_like(eager)
    say(f"[graph] {name}")
    for rep in range(3):
        out.zero_()
        plan.propagate(u0, 0, Q, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep} differs"
        if rep == 0:
            plan.stations(u0, 1, [1, cfg["rk4_steps"] // 2])
        elif rep == 1:
            plan.propagate_batch(u0.reshape(1, -1).contiguous(), 0, Q)
        torch.cuda.synchronize()
    assert torch.equal(plan.field(), eager[-1])
    plan.close()


def test_busy_while_work_runs_on_another_stream(torch_dev, swkb):
    """A plan is single-stream: while the work of a call on stream A is still
    running, a call on stream B returns SWKB_ERR_BUSY and does nothing; once
    A is done, stream B may take the plan."""
    torch, dev = torch_dev
    cfg = W.random_medium(n_screens=200)  # about 30 ms of GPU work, microseconds of host time
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    plan = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    sa, sb = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    hist = torch.empty((cfg["n_screens"], cfg["n_z"]), dtype=torch.complex128, device=dev)
    with torch.cuda.stream(sa):
        u0a = u0.clone()
    sa.synchronize()
    say("[busy] long propagation on stream A")
    plan.propagate(u0a, 0, cfg["n_screens"], out=hist, stream=sa)
    with pytest.raises(swkb.SwkbError) as ei:
        plan.field(stream=sb)
    assert ei.value.status == swkb.swkb.SWKB_ERR_BUSY
    assert "another stream" in plan.last_error
    sa.synchronize()
    f = plan.field(stream=sb)
    sb.synchronize()
    assert torch.equal(f, hist[-1])
    # the same stream never waits on itself
    plan.propagate(None, cfg["n_screens"], cfg["n_screens"], stream=sb)
    plan.field(stream=sb)
    sb.synchronize()
    plan.close()


def test_field_of_any_screen_with_kept_history(torch_dev, swkb):
    """keep_history = 1: swkb_field(q) returns the field of every screen a
    propagation reached, whether the caller asked for a history or not."""
    torch, dev = torch_dev
    base = W.linear_caustic(n_screens=10)
    u0 = torch.from_numpy(W.incident_field(base)).to(dev)
    ref = swkb.Plan(base, device=dev)
    want = ref.propagate(u0, 0, 10)
    ref.close()
    plan = swkb.Plan(W.with_overrides(base, keep_history=1), device=dev)
    with pytest.raises(swkb.SwkbError) as ei:
        plan.field(0)
    assert ei.value.status == swkb.swkb.SWKB_ERR_STATE
    plan.propagate(u0, 0, 4, history=False)       # kernels write the kept rows
    plan.propagate(None, 4, 7)                    # caller's history, copied into the kept rows
    plan.propagate(None, 7, 10, history=False)
    assert torch.equal(plan.field(0), u0)
    for q in range(1, 11):
        assert torch.equal(plan.field(q), want[q - 1]), f"screen {q}"
    assert torch.equal(plan.field(-1), want[-1])
    with pytest.raises(swkb.SwkbError) as ei:
        plan.field(11)
    assert ei.value.status == swkb.swkb.SWKB_ERR_ARG
    plan.close()
    # without kept history only the current screen is held
    plain = swkb.Plan(base, device=dev)
    plain.propagate(u0, 0, 3, history=False)
    assert torch.equal(plain.field(3), want[2])
    with pytest.raises(swkb.SwkbError) as ei:
        plain.field(2)
    assert ei.value.status == swkb.swkb.SWKB_ERR_STATE
    plain.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_evanescent_mode_is_reported(torch_dev, swkb, prec):
    """A beam aimed at grazing incidence in free space puts weight on the
    mode xi = -1, whose rays all have p^2 = 0 <= p2_floor: the mode carries
    nothing across, the counters equal the oracle's and the diagnostics
    return SWKB_ERR_EVANESCENT."""
    import oracle
    torch, dev = torch_dev
    # the launch extension covers the drift of the steepest live mode, so the
    # first screen's output holds no weight on the dead mode (a clear
    # decision on the second screen for both sides)
    cfg = W.with_overrides(W.linear_caustic(n_screens=2), medium_params=[1.0, 0.0], eps_ref=1.0,
                           absorber_top=0.0, absorber_bot=0.0, launch_ext_cells=400)
    cfg["source"] = dict(cfg["source"], xi0=-0.999, z0=32.0)
    u0 = W.incident_field(cfg)
    ref, cnt = oracle.run(cfg, u0)
    say(f"[evanescent] oracle {cnt}")
    assert cnt["evanescent_modes"] == 2 and cnt["significant_evanescent"] == 1
    plan = swkb.Plan(cfg, precision=swkb.FP64 if prec == "fp64" else swkb.MIXED, device=dev)
    hist = plan.propagate(torch.from_numpy(u0).to(dev), 0, cfg["n_screens"]).cpu().numpy()
    d = plan.diagnostics()
    say(f"[evanescent] {prec} {d}")
    assert d["evanescent_modes"] == cnt["evanescent_modes"]
    assert d["significant_evanescent"] == cnt["significant_evanescent"]
    assert d["significant"] == cnt["significant"] == 0
    with pytest.raises(swkb.SwkbError) as ei:
        plan.diagnostics(raise_on_caustic=True)
    assert ei.value.status == swkb.swkb.SWKB_ERR_EVANESCENT
    err = float(np.linalg.norm(hist - ref) / np.linalg.norm(ref))
    assert err <= (1e-10 if prec == "fp64" else 1e-3)
    plan.close()


@pytest.mark.parametrize("prop", [0, 2])
@pytest.mark.parametrize("n_z,n_modes,stride", [(512, 128, 1), (16384, 8192, 8)])
def test_batch_diagnostics_equal_one_field(torch_dev, swkb, n_z, n_modes, stride, prop):
    """The epilogue's diagnostics have a one-field path (each thread holds
    its modes' energies in registers while M <= 4096, and makes a second
    pass over the modes above that) and a several-field path (energies summed
    over the batch).  Two copies of one field double every mode energy and
    the largest one (to within rounding, which could move only a mode lying
    at the threshold itself), so every count of the batch equals the
    one-field count; the wide screen makes caustic modes significant."""
    torch, dev = torch_dev
    cfg = W.with_overrides(W.linear_caustic(n_screens=2), n_z=n_z, n_modes=n_modes, ray_stride=stride, dx=300.0,
                           rk4_steps=64, absorber_top=0.0, absorber_bot=0.0, caustic_tol=1e-3, propagator=prop)
    u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
    say(f"[diag] N={n_z} M={n_modes} prop={prop}: one field")
    one = swkb.Plan(cfg, precision=swkb.MIXED, device=dev)
    one.propagate(u0, 0, 2)
    d1 = one.diagnostics()
    one.close()
    say(f"[diag] N={n_z} M={n_modes} prop={prop}: batch of two, one-field counts {d1}")
    two = swkb.Plan(W.with_overrides(cfg, max_batch=2), precision=swkb.MIXED, device=dev)
    two.propagate_batch(torch.stack([u0, u0]).contiguous(), 0, 2)
    d2 = two.diagnostics()
    two.close()
    say(f"[diag] batch counts {d2}")
    assert d1["screens"] == 2 and d1["significant"] > 0
    assert d1 == d2
