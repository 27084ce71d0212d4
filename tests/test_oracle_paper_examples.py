"""The paper's worked example with a printed accuracy, checked on the oracle."""
import json
import os

import numpy as np

import workloads as W
from refs import modal_reference, rel_l2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_example1.json")


def test_example1_single_cusp_error_magnitude(oracle_mod):
    """Single cusp caustic, 40 km at k = 125 (Sec. 3.2): relative error of the
    order of 1e-5 against separation of variables over all 40 screens."""
    g = json.load(open(GOLDEN))
    pr, rd = g["printed"], g["reading"]
    k = pr["k"]
    cfg = W._base(lam=2 * np.pi / k, z_a=rd["z_a"], z_b=rd["z_b"], n_z=rd["n_z"], n_modes=pr["n_modes"],
                  x0=0.0, dx=pr["range_m"] / pr["n_screens"], n_screens=pr["n_screens"],
                  rk4_steps=rd["rk4_steps"], ray_stride=rd["ray_stride"],
                  launch_ext_cells=rd["launch_ext_cells"], bc=W.BC_PERIODIC, absorber_bot=0.0,
                  absorber_top=0.0, medium_kind=W.MEDIUM_EXPGAUSS,
                  medium_params=[1.0, pr["a"], pr["b"], 0.0], eps_ref=1.0,
                  source=dict(z0=rd["beam_centre_m"], width=rd["beam_width_m"], xi0=0.0))
    u0 = W.incident_field(cfg)
    hist, cnt = oracle_mod.run(cfg, u0)
    z = W.grid(cfg)
    ref = modal_reference(z, rd["z_b"] - rd["z_a"], k, 1 + pr["a"] * np.exp(-pr["b"] * z ** 2), u0,
                          cfg["dx"] * np.arange(1, pr["n_screens"] + 1))
    err = rel_l2(hist, ref)
    assert err < g["assert_rel_l2_below"]
    assert err > 1e-7  # an asymptotic method: the error is not at rounding level
    assert cnt["caustic_rays"] == 0 and cnt["significant"] == 0
