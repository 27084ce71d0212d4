"""Many problems in media that do not depend on x carried together, one
launch per stage per screen step (swkb_multi_*).  With the single-problem
launch shapes every field equals a separate swkb_propagate bit for bit;
with autotuned shapes (another split of the sums over modes) it agrees to
FP32 rounding; small problems are also held against the oracle."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-3
RESPLIT_TOL = 1e-5  # same terms, FP32 partial sums split over other workgroups


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
    import paper_2301_03814_amd as pkg
    pkg.load()
    return torch, torch.device("cuda:0"), pkg


def uneven():
    """Ducts of two grid sizes, two frequencies, both ground conditions and
    uneven ranges (one of a single screen, two of equal length)."""
    out = []
    spec = [(2048, 60.0, 0.05, W.BC_DIRICHLET, 7), (4096, 90.0, 0.05, W.BC_NEUMANN, 3),
            (2048, 80.0, 0.1, W.BC_NEUMANN, 7), (4096, 120.0, 0.1, W.BC_DIRICHLET, 5),
            (2048, 60.0, 0.05, W.BC_DIRICHLET, 1)]
    for i, (nz, H, lam, bc, q) in enumerate(spec):
        c = W.surface_duct(n_screens=q, n_z=nz, n_modes=nz // 4, lam=lam, height=H, bc=bc, ext_m=4.0,
                           source_z=10.0 + 3.0 * i, slope_in=-0.3 + 0.05 * i)
        c["name"] = f"uneven_{i}"
        out.append(c)
    return out


def standalone(torch, dev, pkg, cfg, prec=None):
    p = pkg.Plan(cfg, precision=pkg.MIXED if prec is None else prec, device=dev)
    h = p.propagate(torch.from_numpy(W.incident_field(cfg)).to(dev), 0, cfg["n_screens"])
    d = p.diagnostics()
    p.close()
    return h.cpu().numpy(), d


def group(torch, dev, pkg, cfgs):
    plans = [pkg.Plan(c, precision=pkg.MIXED, device=dev) for c in cfgs]
    assert all(p.uses_matrix for p in plans)
    u0s = [torch.from_numpy(W.incident_field(c)).to(dev) for c in cfgs]
    return plans, u0s, pkg.Multi(plans)


def close(plans, m):
    m.close()
    for p in plans:
        p.close()


def test_default_shapes_equal_separate_runs(env):
    torch, dev, pkg = env
    cfgs = uneven()
    say(f"[multi] default shapes: N {[c['n_z'] for c in cfgs]} Q {[c['n_screens'] for c in cfgs]}")
    ref = [standalone(torch, dev, pkg, c) for c in cfgs]
    plans, u0s, m = group(torch, dev, pkg, cfgs)
    t = m.tuning()
    assert t["n_z"] == [2048, 4096] and not t["graphs"]
    hists = m.propagate(u0s, history=True)
    torch.cuda.synchronize()
    for i, (c, p) in enumerate(zip(cfgs, plans)):
        got = hists[i].cpu().numpy()
        assert np.array_equal(got, ref[i][0]), c["name"]
        assert torch.equal(p.field(), hists[i][-1])
        assert p.current_screen == c["n_screens"]
        assert p.diagnostics() == ref[i][1], c["name"]
    close(plans, m)


def test_graph_replays_equal_eager(env):
    """The captured step sequence replayed three times, with eager work and
    synchronisations between the replays, every replay checked."""
    torch, dev, pkg = env
    cfgs = uneven()
    ref = [standalone(torch, dev, pkg, c)[0] for c in cfgs]
    plans, u0s, m = group(torch, dev, pkg, cfgs)
    m.set_tuning(graphs=True)
    for r in range(3):
        say(f"[multi] graph replay {r}")
        hists = m.propagate(u0s, history=True)
        junk = torch.randn(1 << 16, device=dev).sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i in range(len(cfgs)):
            assert np.array_equal(hists[i].cpu().numpy(), ref[i]), (r, i)
    close(plans, m)


def test_persistent_launch_equals_separate_runs(env):
    """One cooperative launch for every step of every problem (grid-wide
    barriers between the stages) gives each problem's history and
    diagnostics of a separate swkb_propagate bit for bit, on two calls in a
    row."""
    torch, dev, pkg = env
    cfgs = uneven()
    ref = [standalone(torch, dev, pkg, c) for c in cfgs]
    plans, u0s, m = group(torch, dev, pkg, cfgs)
    m.set_tuning(persistent=True)
    assert m.tuning()["persistent"]
    for r in range(2):
        say(f"[multi] persistent launch, call {r}")
        before = [p.diagnostics() for p in plans]
        hists = m.propagate(u0s, history=True)
        torch.cuda.synchronize()
        for i, (c, p) in enumerate(zip(cfgs, plans)):
            assert np.array_equal(hists[i].cpu().numpy(), ref[i][0]), (r, c["name"])
            assert torch.equal(p.field(), hists[i][-1])
            if r == 0:
                assert p.diagnostics() == ref[i][1], c["name"]
            else:  # counters accumulate over calls
                d = p.diagnostics()
                assert d["screens"] == before[i]["screens"] + c["n_screens"], c["name"]
    close(plans, m)


def test_persistent_launch_equals_stage_launches_tuned(env):
    """With autotuned shapes the persistent launch equals the per-stage
    launches of the same tuning bit for bit."""
    torch, dev, pkg = env
    cfgs = uneven()
    plans, u0s, m = group(torch, dev, pkg, cfgs)
    t = m.tune(reps=2)
    say(f"[multi] tuned {t['fft_elems']} {t['apply_groups']}")
    m.set_tuning(graphs=False, persistent=False)
    want = [h.cpu().numpy() for h in m.propagate(u0s, history=True)]
    m.set_tuning(persistent=True)
    got = m.propagate(u0s, history=True)
    torch.cuda.synchronize()
    for i in range(len(cfgs)):
        assert np.array_equal(got[i].cpu().numpy(), want[i]), i
    close(plans, m)


@pytest.mark.parametrize("persistent", [False, True])
def test_fp64_and_mixed_problems_in_one_group(env, persistent):
    """FP64 and mixed plans share a group: with the default shapes, by
    per-stage launches and by the persistent launch, each history equals its
    separate swkb_propagate bit for bit (FP64 products keep their blocking)."""
    torch, dev, pkg = env
    cfgs = uneven()
    precs = [pkg.FP64 if i % 2 == 0 else pkg.MIXED for i in range(len(cfgs))]
    ref = [standalone(torch, dev, pkg, c, pr)[0] for c, pr in zip(cfgs, precs)]
    plans = [pkg.Plan(c, precision=pr, device=dev) for c, pr in zip(cfgs, precs)]
    u0s = [torch.from_numpy(W.incident_field(c)).to(dev) for c in cfgs]
    m = pkg.Multi(plans)
    if persistent:
        m.set_tuning(persistent=True)
    say(f"[multi] FP64 and mixed, persistent={persistent}")
    hists = m.propagate(u0s, history=True)
    torch.cuda.synchronize()
    for i, c in enumerate(cfgs):
        assert np.array_equal(hists[i].cpu().numpy(), ref[i]), (c["name"], precs[i])
    close(plans, m)


def test_autotuned_shapes(env):
    torch, dev, pkg = env
    cfgs = uneven()
    ref = [standalone(torch, dev, pkg, c)[0] for c in cfgs]
    plans, u0s, m = group(torch, dev, pkg, cfgs)
    before = m.tuning()
    t = m.tune(reps=3)
    say(f"[multi] tuned {t}")
    assert t["n_z"] == before["n_z"]
    for c, (nz, fe, gr) in enumerate(zip(t["n_z"], t["fft_elems"], t["apply_groups"])):
        M = nz // 4
        assert fe in (256, 512, 1024)
        assert gr == before["apply_groups"][c] or gr in (M // 32, M // 64, M // 128, M // 256)
        assert t["fft_us"][c] > 0.0 and t["apply_us"][c] > 0.0
    assert all(p.current_screen == -1 for p in plans)
    h1 = m.propagate(u0s, history=True)
    m.set_tuning(graphs=True)
    h2 = m.propagate(u0s, history=True)
    torch.cuda.synchronize()
    for i in range(len(cfgs)):
        a = h1[i].cpu().numpy()
        assert np.array_equal(a, h2[i].cpu().numpy())
        err = rel(a, ref[i])
        say(f"[multi] tuned vs separate {cfgs[i]['name']}: rel={err:.2e}")
        assert err <= RESPLIT_TOL
    # explicit shapes: every candidate value is accepted and agrees
    m.set_tuning(fft_elems=[1024, 256], apply_groups=[1, 3], graphs=False)
    h3 = m.propagate(u0s, history=True)
    torch.cuda.synchronize()
    for i in range(len(cfgs)):
        assert rel(h3[i].cpu().numpy(), ref[i]) <= RESPLIT_TOL
    close(plans, m)


def test_small_problems_match_oracle(env):
    import oracle
    torch, dev, pkg = env
    oracle.build()
    cfgs = [uneven()[k] for k in (1, 2)]
    cfgs = [W.with_overrides(c, n_screens=3) for c in cfgs]
    plans, u0s, m = group(torch, dev, pkg, cfgs)
    m.tune(reps=2)
    hists = m.propagate(u0s, history=True)
    torch.cuda.synchronize()
    for c, h in zip(cfgs, hists):
        ref, _ = oracle.run(c, W.incident_field(c))
        err = rel(h.cpu().numpy(), ref)
        say(f"[multi] {c['name']} vs oracle rel={err:.2e}")
        assert err <= MIXED_TOL
    close(plans, m)


def test_rejects_plans_it_cannot_carry(env):
    torch, dev, pkg = env
    c = uneven()[0]
    rec = pkg.Plan(W.with_overrides(c, propagator=2), precision=pkg.MIXED, device=dev)
    small = pkg.Plan(W.with_overrides(W.linear_caustic(n_screens=2), n_z=256, n_modes=64), precision=pkg.MIXED,
                     device=dev)
    ok = pkg.Plan(c, precision=pkg.MIXED, device=dev)
    for bad in ([rec], [small], [ok, ok]):
        with pytest.raises(pkg.SwkbError) as ei:
            pkg.Multi(bad)
        assert ei.value.status == 1
    m = pkg.Multi([ok])
    for kw in (dict(fft_elems=[300]), dict(apply_groups=[0])):
        with pytest.raises(pkg.SwkbError):
            m.set_tuning(**kw)
    with pytest.raises(ValueError):
        m.set_tuning(fft_elems=[512, 512])
    m.close()
    for p in (rec, small, ok):
        p.close()


@pytest.mark.slow
def test_uneven_duct_batch_full_size(env):
    """The 64 seeded duct problems (1-10 GHz, 200-500 m, N_z 2048-16384, 10-100
    km) at full range in one group, autotuned, graphs on, as the benchmark
    runs them: the problems of extreme size and range equal their separate
    runs to FP32 re-split rounding, and the group's first screen of the
    smallest one (from its seeded incident beam) equals the oracle's."""
    import oracle
    torch, dev, pkg = env
    cfgs = W.duct_batch(seed=4, n_problems=64)
    Q = [c["n_screens"] for c in cfgs]
    N = [c["n_z"] for c in cfgs]
    picks = sorted({int(np.argmax(N)), int(np.argmin(N)), int(np.argmax(Q)), int(np.argmin(Q))})
    say(f"[multi] full batch: sum Q={sum(Q)}, sampled problems {picks}")
    plans, u0s, m = group(torch, dev, pkg, cfgs)
    t = m.tune(reps=3)
    m.set_tuning(graphs=True)
    say(f"[multi] tuned {t}")
    hists = m.propagate(u0s, history=picks)
    torch.cuda.synchronize()
    fields = [p.field() for p in plans]
    for i, f in enumerate(fields):
        assert bool(torch.isfinite(torch.view_as_real(f)).all()), i
        assert plans[i].diagnostics()["screens"] == Q[i]
    for i in picks:
        ref, _ = standalone(torch, dev, pkg, cfgs[i])
        err = rel(hists[i].cpu().numpy(), ref)
        say(f"[multi] problem {i} (N={N[i]}, Q={Q[i]}) vs separate rel={err:.2e}")
        assert err <= RESPLIT_TOL
        assert torch.equal(fields[i], hists[i][-1])
    i = int(np.argmin(N))
    q = 0
    h = hists[i].cpu().numpy()
    ref, _ = oracle.screen(cfgs[i], q, W.incident_field(cfgs[i]))
    err = rel(h[q], ref)
    say(f"[multi] problem {i} screen {q} vs oracle rel={err:.2e}")
    assert err <= MIXED_TOL
    close(plans, m)
