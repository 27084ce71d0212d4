"""Overlapping-patch Fourier-continuation screened WKB (FC-SWKB), Sec. 2.4
(eq. ifft_eq_phi_patches) with the boundary treatment of Sec. 2.5, plain
FP64 CPU.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: it composes the
oracle's own mode, ray and interpolation steps and shares no code with the
GPU library.

Patches.  With K = N / P grid cells per core and e_w = ceil(6 w / h), patch p
is the index range [a_p, b_p] = [p K - e_w, (p + 1) K + e_w] clipped to the
grid [0, N - 1].  The partition of unity S^p is the erfc one of
``patches.partition`` (sum_p S^p = 1; S^p < 1e-17 beyond the patch).

One screen (the paper's representation, read literally):

1. Fourier continuation of u on each patch (FC-Gram blend of ``fc_gram``):
   the n_p samples, C = 27 values blending the last d = 5 samples to zero
   after b_p, zeros, and the mirrored blend of the first 5 samples before
   a_p, one period of length P_p (a power of two) placed so that the patch
   sits in its middle; the DFT of that period gives the patch's modes
   w_j / P_p (the amplitude normalisation of eq. ifft_eq_phi_patches).
2. Each mode of each patch is carried across the screen by the rays of the
   periodic method (Sec. 2.1.2) launched at the grid points of the patch
   only, with initial amplitude S^p(z) w_j / P_p: the launch amplitude of ray
   r is multiplied by S^p(s_r); rays launched outside [a_p, b_p] are not
   launched at all.
3. Each patch's modes are interpolated and summed (eq. ray_bundle_q_plus_1)
   on the grid points of its period window (patch plus the continuation
   cells around it), and the patches' sums are added on the global grid.

Boundaries (Sec. 2.5).  Open ends (bc = periodic here means no wall): the
sums outside the grid are dropped and the exit taper W applies once.  A
ground at z_a (Dirichlet or Neumann): the boundary patch p = 0 is continued
only at its top, and its period is the odd (even) extension about z_a with
the medium reflected (the mirror of Sec. 2.3, launch amplitude S^0(|z - z_a|
+ z_a)), so it is never reflected afterwards; every other patch's sum is
reflected on each screen, u_p(z) -/+ u_p(2 z_a - z) (eq. u_refl).

Mode counts keep the global largest vertical slowness: M_p = 2 round(M P_p /
(2 P_g)), P_g the global FFT length.  Each period window has room for
ceil(margin / h) cells of ray drift beyond the continuation cells.
"""
from __future__ import annotations

import math

import numpy as np

from . import march_mode as _march_mode
from . import modes as _modes
from . import interp as _interp
from . import num_rays as _num_rays
from . import taper as _taper
from . import RAY_DEAD_LAUNCH
from .fc_gram import C_CONT, D_MATCH, load as _load_blend
from .patches import partition as _partition

BC_PERIODIC = 0
_BLEND = None


def blend():
    global _BLEND
    if _BLEND is None:
        _BLEND = _load_blend()
    return _BLEND


def _pow2_at_least(n):
    p = 1
    while p < n:
        p *= 2
    return p


def layout(cfg, n_patches, width, margin):
    """Per patch: dict(a, b, start, sub) with the support [a, b] (global
    indices), the global index of the period window's first point and the
    sub-problem configuration of that window."""
    N, M = cfg["n_z"], cfg["n_modes"]
    if n_patches < 1 or N % n_patches:
        raise ValueError("n_patches must divide n_z")
    h = (cfg["z_b"] - cfg["z_a"]) / N
    K = N // n_patches
    e_w = int(math.ceil(6.0 * width / h))
    e_m = int(math.ceil(margin / h))
    ground = cfg["bc"] != BC_PERIODIC
    P_g = N if not ground else 2 * N
    out = []
    for p in range(n_patches):
        a = max(0, p * K - e_w)
        b = min(N - 1, (p + 1) * K + e_w)
        n = b - a + 1
        if n < 2 * D_MATCH:
            raise ValueError("patch shorter than two matching stencils")
        sub = dict(cfg)
        sub["absorber_bot"] = 0.0
        sub["absorber_top"] = 0.0
        if p == 0 and ground:
            nz = _pow2_at_least(b + 1 + C_CONT + e_m)
            start = 0
            sub["launch_ext_cells"] = e_m
            P_p = 2 * nz
        else:
            nz = _pow2_at_least(n + 2 * C_CONT + 2 * e_m)
            start = a - (nz - n) // 2
            sub["bc"] = BC_PERIODIC
            sub["launch_ext_cells"] = 0
            P_p = nz
        sub["n_z"] = nz
        sub["n_modes"] = max(2, 2 * int(math.floor(M * P_p / (2.0 * P_g) + 0.5)))
        sub["z_a"] = cfg["z_a"] + start * h
        sub["z_b"] = cfg["z_a"] + (start + nz) * h
        out.append(dict(a=a, b=b, start=start, sub=sub))
    return out


def fc_period(u, a, b, start, nz, ground_patch):
    """The sub-problem's input vector (nz values at global indices start ..
    start + nz - 1): the samples on [a, b] and their Fourier continuation."""
    B = blend()
    d = D_MATCH
    v = np.zeros(nz, dtype=np.complex128)
    right = B @ u[b - d + 1:b + 1]            # values at b + 1 .. b + C
    left = B @ u[a:a + d][::-1]               # values at a - 1 .. a - C
    for i in range(nz):
        g = start + i
        if a <= g <= b:
            v[i] = u[g]
        elif b < g <= b + C_CONT:
            v[i] = right[g - b - 1]
        elif not ground_patch and a - C_CONT <= g < a:
            v[i] = left[a - g - 1]
    return v


def patch_screen(cfg, q, u, lay, p, n_patches, width):
    """Sum of patch p's modes on its period window (nz values)."""
    L = lay[p]
    sub, a, b, start = L["sub"], L["a"], L["b"], L["start"]
    nz = sub["n_z"]
    ground_patch = p == 0 and cfg["bc"] != BC_PERIODIC
    h = (cfg["z_b"] - cfg["z_a"]) / cfg["n_z"]
    c = _modes(sub, fc_period(u, a, b, start, nz, ground_patch))
    # launch heights of the sub-problem's rays and their amplitude factors
    R = _num_rays(sub)
    gi = start + np.arange(R) * sub["ray_stride"] - sub["launch_ext_cells"]  # global launch index
    gm = np.abs(gi) if ground_patch else gi
    inside = (gm >= a) & (gm <= b)
    S = np.zeros(R)
    S[inside] = _partition(cfg, n_patches, width, cfg["z_a"] + gm[inside] * h)[p]
    z_out = sub["z_a"] + np.arange(nz) * h
    out = np.zeros(nz, dtype=np.complex128)
    k = cfg["k"]
    for j in range(sub["n_modes"]):
        rec = _march_mode(sub, q, j)
        rec["a"] = rec["a"] * S
        rec["flag"] = np.where(inside, rec["flag"], RAY_DEAD_LAUNCH).astype(np.int32)
        ps, amp, has, fold = _interp(rec, z_out)
        if fold:
            continue
        out[has] += c[j] * (amp[has] * np.exp(1j * k * ps[has]))
    return out


def screen(cfg, q, u_in, n_patches, width, margin):
    """Field on screen q+1 from the field on screen q by FC-SWKB."""
    N = cfg["n_z"]
    u = np.asarray(u_in, dtype=np.complex128)
    lay = layout(cfg, n_patches, width, margin)
    ground = cfg["bc"] != BC_PERIODIC
    sgn = -1.0 if cfg["bc"] == 1 else 1.0
    total = np.zeros(N, dtype=np.complex128)
    for p in range(n_patches):
        part = patch_screen(cfg, q, u, lay, p, n_patches, width)
        start, nz = lay[p]["start"], lay[p]["sub"]["n_z"]
        g = np.arange(N)
        i = g - start
        ok = (i >= 0) & (i < nz)
        total[g[ok]] += part[i[ok]]
        if ground and p > 0:  # eq. u_refl on every patch but the boundary one
            im = -g - start
            okm = (im >= 0) & (im < nz)
            total[g[okm]] += sgn * part[im[okm]]
    return _taper(cfg, total)


def run(cfg, u0, n_patches, width, margin, q_begin=0, q_end=None):
    """Screens q_begin..q_end-1 by FC-SWKB; history [q_end-q_begin, N]."""
    if q_end is None:
        q_end = cfg["n_screens"]
    hist = np.zeros((q_end - q_begin, cfg["n_z"]), dtype=np.complex128)
    cur = np.asarray(u0, dtype=np.complex128)
    for q in range(q_begin, q_end):
        cur = screen(cfg, q, cur, n_patches, width, margin)
        hist[q - q_begin] = cur
    return hist
