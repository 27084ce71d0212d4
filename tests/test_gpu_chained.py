"""Chained full-size parity: the library carries the workloads' seeded
incident beams through an uninterrupted chain of screens (Algorithm 1, each
screen's output the next one's input) and the fields on sampled screens are
held against the oracle's own uninterrupted chain, stored by
tests/golden/make_chained.py (which calls only the oracle):

* the random medium (N = 8192, M = 2048), all 400 screens, every 25th;
* the surface duct (N = 16384, M = 4096, Dirichlet ground), the first 20
  screens (2 km), every 4th, through the mode-function matrix and through
  the plain per-screen step (interpolation and sum every screen).

FP64 runs must stay within 1e-10 of the oracle, mixed runs within 1e-3, both
as a relative L2 over the sampled screens and screen by screen as
max |difference| / max |oracle field| (a localized error in a low-amplitude
band cannot hide under the L2 of the whole history)."""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return torch, torch.device("cuda:0")


def load_chain(name):
    d = np.load(os.path.join(HERE, "golden", f"{name}_chain.npz"))
    return d["screens"], d["fields"], dict(zip((str(n) for n in d["counter_names"]), d["counters"]))


def screen_max_rel(got, ref):
    """max |got - ref| / max |ref| per screen (rows)."""
    return np.abs(got - ref).max(axis=1) / np.abs(ref).max(axis=1)


CASES = {
    "random_medium": (lambda: W.random_medium(), 400),
    "surface_duct": (lambda: W.surface_duct(), 20),
    "surface_duct_plain": (lambda: W.with_overrides(W.surface_duct(), propagator=2), 20),
}
TOL = {"fp64": 1e-10, "mixed": 1e-3}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_chain_matches_oracle_chain(torch_dev, name, prec):
    torch, dev = torch_dev
    import paper_2301_03814_amd as pkg
    build, n_screens = CASES[name]
    cfg = build()
    screens, ref, cnt = load_chain(name.replace("_plain", ""))
    say(f"[chain] {name} {prec}: {n_screens} screens on the GPU")
    plan = pkg.Plan(cfg, precision=pkg.FP64 if prec == "fp64" else pkg.MIXED, device=dev)
    assert plan.uses_matrix == (name == "surface_duct")
    hist = plan.propagate(torch.from_numpy(W.incident_field(cfg)).to(dev), 0, n_screens)
    got = hist[torch.from_numpy(screens.astype(np.int64) - 1).to(dev)].cpu().numpy()
    diag = plan.diagnostics()
    plan.close()
    del hist
    l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    mx = screen_max_rel(got, ref)
    say(f"[chain] {name} {prec}: rel L2 {l2:.3e}, per-screen max-norm {mx.max():.3e} "
        f"(screens {list(screens)}: {' '.join(f'{v:.1e}' for v in mx)})")
    say(f"[chain] {name} {prec}: diag {diag} oracle {cnt}")
    assert l2 <= TOL[prec]
    assert mx.max() <= TOL[prec]
    if prec == "fp64":
        # the discrete decisions of the whole chain agree with the oracle's
        for k in ("caustic_rays", "dead_rays", "folded_modes", "significant", "evanescent_modes",
                  "significant_evanescent"):
            assert diag[k] == cnt[k], k
