"""Screened-WKB (S-WKB) propagation on AMD MI355X.

The product is the C-ABI library libswkb.so (include/swkb.h), built from the
HIP sources in csrc/ by ``paper_2301_03814_amd.build``; ``swkb`` is its thin
Python binding.
"""
from .swkb import (BC_DIRICHLET, BC_NEUMANN, BC_PERIODIC, FP64, MIXED, PATCH_FC, PATCH_WINDOWED, Multi, PatchPlan,  # noqa: F401
                   Plan, Server, SwkbError,
                   footprint, load, make_params, modal_reference, workspace_bytes)
