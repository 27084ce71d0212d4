"""Overlapping-patch screened WKB (Sec. 2.4 of the paper), plain FP64 CPU.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: it composes the
oracle's own screen step and shares no code with the GPU library.

The vertical interval is covered by P patches with cores
[c_p, c_{p+1}], c_p = z_a + p K h (K = N / P grid cells), blended by the
smooth partition of unity

    sigma_p(z) = erfc(-(z - c_p) / w) / 2,
    S^0 = 1 - sigma_1,  S^p = sigma_p - sigma_{p+1},  S^{P-1} = sigma_{P-1},

so that sum_p S^p = 1 exactly in real arithmetic, and each S^p falls below
1e-17 more than 6 w outside its core (the paper asks for a smooth partition
of unity vanishing at the patch ends).  A screen step is

    u'(z_m) = W(z_m) sum_p [ screen step of S^p u on sub-domain p ](z_m):

each windowed piece S^p u is smooth and vanishes near the ends of its
sub-domain, so the periodic method of Sec. 2.1 applies to it on that
sub-domain (the ground patch keeps the mirror of Sec. 2.3); the pieces'
outputs are added on the global grid and the global exit taper W is applied
once.  Sub-domain p holds n_p = 2^j >= K + 2 e points (K + e for the ground
patch), e = ceil((6 w + margin) / h), placed symmetrically around the core;
points outside [0, N) carry no field and their outputs are dropped.  Its mode
count keeps the global largest vertical slowness: M_p = 2 round(M P_p / (2 P_g))
with P_p, P_g the sub-domain's and the global FFT lengths.  Sub-domains run
without absorbers.  This composition stands in for the paper's
Fourier-continuation expansion of u on each patch, whose continuation
matrices the paper does not give: the windowed piece needs no continuation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from . import screen as _screen
from . import taper as _taper

BC_PERIODIC = 0


def _pow2_at_least(n):
    p = 1
    while p < n:
        p *= 2
    return p


def layout(cfg, n_patches, width, margin):
    """[(start index, sub-domain config)] of the P patches."""
    N, M = cfg["n_z"], cfg["n_modes"]
    if n_patches < 1 or N % n_patches:
        raise ValueError("n_patches must divide n_z")
    h = (cfg["z_b"] - cfg["z_a"]) / N
    K = N // n_patches
    e = int(math.ceil((6.0 * width + margin) / h))
    P_g = N if cfg["bc"] == BC_PERIODIC else 2 * N
    out = []
    for p in range(n_patches):
        sub = dict(cfg)
        if p == 0 and cfg["bc"] != BC_PERIODIC:
            n = _pow2_at_least(K + e)
            start = 0
        else:
            need = K + 2 * e
            n = _pow2_at_least(need)
            start = p * K - e - (n - need) // 2
            sub["bc"] = BC_PERIODIC
        P_p = n if sub["bc"] == BC_PERIODIC else 2 * n
        sub["n_z"] = n
        sub["n_modes"] = max(2, 2 * int(math.floor(M * P_p / (2.0 * P_g) + 0.5)))
        sub["z_a"] = cfg["z_a"] + start * h
        sub["z_b"] = cfg["z_a"] + (start + n) * h
        sub["absorber_bot"] = 0.0
        sub["absorber_top"] = 0.0
        out.append((start, sub))
    return out


def partition(cfg, n_patches, width, z):
    """S^p(z) for p = 0..P-1 as an array [P, len(z)]."""
    N = cfg["n_z"]
    h = (cfg["z_b"] - cfg["z_a"]) / N
    K = N // n_patches
    z = np.asarray(z, dtype=np.float64)
    if n_patches == 1:
        return np.ones((1, z.size))
    sig = [0.5 * erfc(-(z - (cfg["z_a"] + p * K * h)) / width) for p in range(n_patches + 1)]
    S = np.empty((n_patches, z.size))
    S[0] = 1.0 - sig[1]
    for p in range(1, n_patches - 1):
        S[p] = sig[p] - sig[p + 1]
    S[n_patches - 1] = sig[n_patches - 1]
    return S


def screen(cfg, q, u_in, n_patches, width, margin):
    """Field on screen q+1 from the field on screen q by the patch method."""
    N = cfg["n_z"]
    h = (cfg["z_b"] - cfg["z_a"]) / N
    u_in = np.asarray(u_in, dtype=np.complex128)
    out = np.zeros(N, dtype=np.complex128)
    for p, (start, sub) in enumerate(layout(cfg, n_patches, width, margin)):
        n = sub["n_z"]
        m = start + np.arange(n)
        ok = (m >= 0) & (m < N)
        zg = cfg["z_a"] + m[ok] * h
        v = np.zeros(n, dtype=np.complex128)
        v[ok] = partition(cfg, n_patches, width, zg)[p] * u_in[m[ok]]
        w, _ = _screen(sub, q, v)
        out[m[ok]] += w[ok]
    return _taper(cfg, out)


def run(cfg, u0, n_patches, width, margin, q_begin=0, q_end=None):
    """Screens q_begin..q_end-1 by the patch method; history [q_end-q_begin, N]."""
    if q_end is None:
        q_end = cfg["n_screens"]
    hist = np.zeros((q_end - q_begin, cfg["n_z"]), dtype=np.complex128)
    cur = np.asarray(u0, dtype=np.complex128)
    for q in range(q_begin, q_end):
        cur = screen(cfg, q, cur, n_patches, width, margin)
        hist[q - q_begin] = cur
    return hist
