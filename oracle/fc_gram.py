"""Fourier-continuation (FC-Gram) blending data for the overlapping-patch
method, derived from its definition in high precision.  Writes
``fc_gram_d5_c27.txt`` beside this file.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``.

Sec. 2.4 expands the field on each patch by Fourier continuation (the
FC-Gram method of the cited FC papers): the samples of a non-periodic
function on a patch are extended by C values beyond its last point so that
the extended sequence is the restriction of a smooth periodic function,
whose DFT then gives an accurate Fourier series of the function on the
patch.  The data are built here as follows (grid spacing 1, d = 5 matching
points t = 0..d-1 at an end of the patch, C = 27 continuation points
t = d-1+c, c = 1..C):

* Gram basis: the polynomials of degree < d orthonormal for the discrete
  inner product sum_{i<d} f(t_i) g(t_i), by Gram-Schmidt on 1, t, .., t^{d-1};
* blend to zero: for each basis polynomial phi_k, the trigonometric
  polynomial g_k of period 72 = 2 (2d + C - 1) with harmonics 0..16 that is
  the exact least-squares fit (no regularisation) of phi_k on [0, d-1] and
  of zero on [d+C, 2d+C-1], both sampled 20 times per grid cell;
* blend matrix B[c][i] = sum_k g_k(d-1+c) phi_k(t_i): the continuation
  values beyond the last matching point are B f_end (f_end the last d
  samples in increasing t).

The least-squares problem is solved through the singular value
decomposition in 60-digit arithmetic (its smallest singular value is about
1e-18 of the largest) and B is rounded to binary64 at the end.
"""
from __future__ import annotations

import os

import mpmath as mp

D_MATCH = 5
C_CONT = 27
OVERSAMPLE = 20
HARMONICS = 16
PERIOD = 2 * (2 * D_MATCH + C_CONT - 1)
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"fc_gram_d{D_MATCH}_c{C_CONT}.txt")


def gram_basis(d):
    """Coefficients (lowest degree first) of the orthonormal polynomials."""
    t = [mp.mpf(i) for i in range(d)]
    out = []
    for k in range(d):
        vals = [ti ** k for ti in t]
        coef = [mp.mpf(0)] * d
        coef[k] = mp.mpf(1)
        for bvals, bcoef in out:  # modified Gram-Schmidt against the earlier ones
            pr = mp.fsum(vals[i] * bvals[i] for i in range(d))
            vals = [vals[i] - pr * bvals[i] for i in range(d)]
            coef = [coef[j] - pr * bcoef[j] for j in range(d)]
        nrm = mp.sqrt(mp.fsum(v * v for v in vals))
        out.append(([v / nrm for v in vals], [c / nrm for c in coef]))
    return out


def poly(coef, t):
    return mp.fsum(c * t ** j for j, c in enumerate(coef))


def trig_row(t):
    row = [mp.mpf(1)]
    for m in range(1, HARMONICS + 1):
        a = 2 * mp.pi * m * t / PERIOD
        row += [mp.cos(a), mp.sin(a)]
    return row


def blend_matrix(dps=60):
    """B as a list of C rows of d mpf values."""
    with mp.workdps(dps):
        d, C = D_MATCH, C_CONT
        basis = gram_basis(d)
        t_match = [mp.mpf(j) / OVERSAMPLE for j in range(OVERSAMPLE * (d - 1) + 1)]
        t_zero = [d + C + mp.mpf(j) / OVERSAMPLE for j in range(OVERSAMPLE * (d - 1) + 1)]
        A = mp.matrix([trig_row(t) for t in t_match + t_zero])
        U, S, V = mp.svd_r(A)
        cont_rows = [mp.matrix([trig_row(mp.mpf(d - 1 + c))]) for c in range(1, C + 1)]
        g = []  # g[k][c-1]: continuation of phi_k
        for k in range(d):
            rhs = mp.matrix([poly(basis[k][1], t) for t in t_match] + [0] * len(t_zero))
            x = mp.matrix(A.cols, 1)
            for i in range(len(S)):
                x += ((U[:, i].T * rhs)[0] / S[i]) * V[i, :].T
            g.append([(r * x)[0] for r in cont_rows])
        return [[mp.fsum(g[k][c] * basis[k][0][i] for k in range(d)) for i in range(d)] for c in range(C)]


def write(path=DATA):
    B = blend_matrix()
    with open(path, "w") as f:
        f.write(f"# FC-Gram blend matrix B[c][i], c = 1..{C_CONT} rows, i = 0..{D_MATCH - 1} columns "
                f"(written by oracle/fc_gram.py)\n")
        for row in B:
            f.write(" ".join(repr(float(v)) for v in row) + "\n")
    return path


def load(path=DATA):
    import numpy as np
    return np.loadtxt(path, comments="#", dtype=np.float64).reshape(C_CONT, D_MATCH)


if __name__ == "__main__":
    print(write())
