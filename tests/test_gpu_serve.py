"""Serving loop (swkb_server_*): requests admitted by device footprint and
advanced together on their own streams give, for every request, the field
a standalone run gives — bit for bit, alone or in the mix."""
import sys
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def swkb():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2301_03814_amd as pkg
    pkg.load()
    return pkg


def requests():
    """Uneven mix: random media, ducts (mode-function matrix), a caustic case."""
    out = []
    for i, (nz, q) in enumerate(((1024, 7), (1024, 12), (2048, 5))):
        out.append(W.random_medium(n_screens=q, n_z=nz, n_modes=nz // 4, height=nz * (125.0 / 1024.0),
                                   seed=100 + i, n_gauss=8, x_len=q * 10.0))
    for i, bc in enumerate((W.BC_DIRICHLET, W.BC_NEUMANN)):
        out.append(W.surface_duct(n_screens=6 + i, n_z=2048, n_modes=512, height=60.0, bc=bc, ext_m=4.0,
                                  source_z=10.0 + 5.0 * i))
    out.append(W.linear_caustic(n_screens=9))
    return out


def standalone(swkb, cfg, prec):
    import torch
    dev = torch.device("cuda:0")
    p = swkb.Plan(cfg, precision=prec, device=dev)
    h = p.propagate(torch.from_numpy(W.incident_field(cfg)).to(dev), 0, cfg["n_screens"])
    out = h[-1].cpu().numpy()
    p.close()
    return out


def serve(swkb, cfgs, precs, budget, max_active, spr, late=(), quantum=0.0):
    """Submit all but the `late` indices at once, the late ones after a few rounds."""
    srv = swkb.Server(budget, max_active=max_active, screens_per_round=spr, mode_points_per_round=quantum)
    ids = {}
    for i, (c, pr) in enumerate(zip(cfgs, precs)):
        if i not in late:
            ids[i] = srv.submit(c, W.incident_field(c), precision=pr)
    results, most_active, rounds = {}, 0, 0
    t_end = time.time() + 60.0
    while len(results) < len(cfgs):
        assert time.time() < t_end, "serving did not finish"
        a, _ = srv.step()
        most_active = max(most_active, a)
        rounds += 1
        if rounds == 3:
            for i in late:
                ids[i] = srv.submit(cfgs[i], W.incident_field(cfgs[i]), precision=precs[i])
        for i, rid in ids.items():
            if i in results:
                continue
            state, info, field = srv.poll(rid)
            if field is not None:
                results[i] = (field, info)
        time.sleep(0.0005)
    st = srv.stats()
    srv.close()
    return results, most_active, st


@pytest.mark.parametrize("spr,quantum", [(3, 0.0), (1, 4e6)])
def test_served_equals_standalone(swkb, spr, quantum):
    """Chunks of 3 screens, or chunks of about 4e6 mode-points (processor
    sharing: small requests take many screens per chunk, large ones few)."""
    cfgs = requests()
    precs = [swkb.MIXED, swkb.FP64] * 3
    ref = [standalone(swkb, c, p) for c, p in zip(cfgs, precs)]
    results, most_active, st = serve(swkb, cfgs, precs, budget=64 << 30, max_active=4, spr=spr, late=(1, 4),
                                     quantum=quantum)
    say(f"[serve] most admitted at once {most_active}, stats {st}")
    assert most_active >= 2  # work of several requests in flight together
    assert st["completed"] == len(cfgs)
    assert st["device_bytes_in_use"] == 0
    for i, (field, info) in results.items():
        assert np.array_equal(field, ref[i]), f"request {i} differs from its standalone run"
        assert info["latency_us"] > 0


def test_admission_by_footprint(swkb):
    """A budget that holds only the largest request: one request at a time,
    same results."""
    cfgs = [requests()[k] for k in (0, 1, 5)]  # footprints within 2 % of each other
    precs = [swkb.MIXED] * 3
    need = max(swkb.workspace_bytes(c, swkb.MIXED) for c in cfgs) + (1 << 20)
    assert need < 2 * min(swkb.workspace_bytes(c, swkb.MIXED) for c in cfgs)
    ref = [standalone(swkb, c, p) for c, p in zip(cfgs, precs)]
    results, most_active, st = serve(swkb, cfgs, precs, budget=need, max_active=8, spr=2)
    say(f"[serve] budget {need} B: most admitted at once {most_active}")
    assert most_active == 1
    for i, (field, _) in results.items():
        assert np.array_equal(field, ref[i])


def test_uneven_duct_batch_served(swkb):
    """The first problems of the seeded uneven duct batch (1-10 GHz, duct
    depth 10-100 m, 200-500 m high, N_z 2048-16384), ranges cut to 6 screens:
    served together they equal their standalone runs bit for bit."""
    cfgs = [W.with_overrides(c, n_screens=6) for c in W.duct_batch(seed=4, n_problems=4)]
    precs = [swkb.MIXED] * len(cfgs)
    ref = [standalone(swkb, c, p) for c, p in zip(cfgs, precs)]
    results, most_active, st = serve(swkb, cfgs, precs, budget=64 << 30, max_active=4, spr=1, quantum=2e8)
    say(f"[serve] duct batch N_z {[c['n_z'] for c in cfgs]}: most admitted at once {most_active}")
    for i, (field, _) in results.items():
        assert np.array_equal(field, ref[i])
