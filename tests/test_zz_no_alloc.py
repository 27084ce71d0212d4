"""The entry point that allocates nothing (swkb_propagate_static) against the
plan-based entry point (swkb_propagate) on the same inputs: two calls in a
row on one stream, the second on a smaller problem, so the second call runs
in an array that still holds the first call's tables and records."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return torch, torch.device("cuda:0")


def _case(name):
    if name == "linear":
        return W.linear_caustic()
    if name == "linear_small":
        return W.with_overrides(W.linear_caustic(n_screens=5), n_z=256, n_modes=64, ray_stride=3,
                                launch_ext_cells=37)
    if name == "random":
        return W.random_medium(n_screens=12, n_z=1024, n_modes=256, height=125.0, seed=7, n_gauss=12,
                               x_len=120.0)
    if name == "random_small":
        return W.random_medium(n_screens=4, n_z=512, n_modes=128, height=125.0, seed=3, n_gauss=6, x_len=40.0)
    if name == "duct":
        return W.surface_duct(n_screens=4, n_z=2048, n_modes=512, height=60.0, ext_m=4.0)
    if name == "duct_small":
        return W.surface_duct(n_screens=3, n_z=1024, n_modes=256, height=30.0, ext_m=4.0)
    raise KeyError(name)


@pytest.mark.parametrize("first,second", [("linear", "linear_small"), ("random", "random_small"),
                                          ("duct", "duct_small")])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_static_entry_equals_plan(torch_dev, first, second, prec):
    torch, dev = torch_dev
    import paper_2301_03814_amd as pkg
    from paper_2301_03814_amd import swkb
    P = pkg.FP64 if prec == "fp64" else pkg.MIXED
    for name in (first, second):
        cfg = _case(name)
        assert pkg.workspace_bytes(cfg, P) <= swkb.STATIC_WORKSPACE_BYTES
        Q = cfg["n_screens"]
        u0 = torch.from_numpy(W.incident_field(cfg)).to(dev)
        say(f"[static] {name} {prec} N={cfg['n_z']} M={cfg['n_modes']} Q={Q}")
        hist, last = swkb.propagate_static(cfg, u0, 0, Q, precision=P)
        plan = pkg.Plan(cfg, precision=P, device=dev)
        ref = plan.propagate(u0, 0, Q)
        torch.cuda.synchronize()
        # same kernels and launch shapes on the same inputs; FP64 also within
        # the oracle bar of each other, mixed within its regression bound
        err = float(torch.linalg.vector_norm(hist - ref) / torch.linalg.vector_norm(ref))
        say(f"[static] {name} {prec} rel={err:.3e} equal={bool(torch.equal(hist, ref))}")
        assert err <= (1e-10 if prec == "fp64" else 5e-5)
        assert torch.equal(hist, ref)
        assert torch.equal(last, ref[-1])
        # a range that starts later, without history
        h2, last2 = swkb.propagate_static(cfg, ref[0].contiguous(), 1, Q, precision=P, history=False)
        assert h2 is None and torch.equal(last2, ref[-1])
        plan.close()


def test_static_entry_rejects_large_and_bad_problems(torch_dev):
    torch, dev = torch_dev
    import paper_2301_03814_amd as pkg
    from paper_2301_03814_amd import swkb
    lib = pkg.load()
    big = W.random_medium()
    assert pkg.workspace_bytes(big) > swkb.STATIC_WORKSPACE_BYTES
    u0 = torch.from_numpy(W.incident_field(big)).to(dev)
    p = swkb.make_params(big)
    st = lib.swkb_propagate_static(C.byref(p), C.c_void_p(u0.data_ptr()), 0, 1, None, None, None)
    assert st == swkb.SWKB_ERR_NOMEM and b"static workspace" in lib.swkb_last_error()
    bad = swkb.make_params(W.with_overrides(W.linear_caustic(), n_z=100))
    st = lib.swkb_propagate_static(C.byref(bad), C.c_void_p(u0.data_ptr()), 0, 1, None, None, None)
    assert st == swkb.SWKB_ERR_ARG and b"power of two" in lib.swkb_last_error()
    small = swkb.make_params(W.linear_caustic())
    st = lib.swkb_propagate_static(C.byref(small), C.c_void_p(u0.data_ptr()), 3, 3, None, None, None)
    assert st == swkb.SWKB_ERR_ARG
