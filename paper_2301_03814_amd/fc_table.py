"""Build step: writes csrc/fc_gram.h, the Fourier-continuation blend matrix
that the overlapping-patch kernels use (run it after changing the
continuation parameters; the header is committed).

Fourier continuation of a patch (Sec. 2.4; the FC-Gram method of the cited
FC papers): C values appended after the last of n samples make the sequence
one period of a smooth function.  Near an end of the patch the samples are
a polynomial of degree < d (d = 5 points, spacing 1, t = 0..4); each such
polynomial is continued by the trigonometric polynomial of period
72 = 2 (2d + C - 1) with harmonics 0..16 that best fits it, in least
squares on 20 samples per cell, on [0, 4] and fits zero on [d + C,
2d + C - 1] = [32, 36].  The blend is linear in the data, so it is computed
here for the monomials 1, t, .., t^4 and mapped to sample values through the
inverse Vandermonde matrix: B = G V^-1, G[c][k] the continuation of t^k at
t = 4 + c, V[i][k] = i^k.  Householder least squares in 80-digit arithmetic
(the fit matrix has a condition number near 1e18), rounded to binary64.
"""
import os

import mpmath as mp

D, C, OVER, HARM = 5, 27, 20, 16
LAM = 2 * (2 * D + C - 1)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "fc_gram.h")


def build():
    with mp.workdps(80):
        ts = [mp.mpf(j) / OVER for j in range(OVER * (D - 1) + 1)]
        ts += [D + C + mp.mpf(j) / OVER for j in range(OVER * (D - 1) + 1)]
        nfit = OVER * (D - 1) + 1

        def basis(t):
            r = [mp.mpf(1)]
            for m in range(1, HARM + 1):
                r.append(mp.cos(2 * mp.pi * m * t / LAM))
                r.append(mp.sin(2 * mp.pi * m * t / LAM))
            return r

        F = mp.matrix([basis(t) for t in ts])
        G = mp.matrix(C, D)
        for k in range(D):
            y = mp.matrix([ts[i] ** k if i < nfit else mp.mpf(0) for i in range(len(ts))])
            coef, _ = mp.qr_solve(F, y)
            for c in range(C):
                G[c, k] = mp.fdot(basis(mp.mpf(D - 1 + c + 1)), coef)
        V = mp.matrix([[mp.mpf(i) ** k for k in range(D)] for i in range(D)])
        B = G * mp.inverse(V)
        return [[float(B[c, i]) for i in range(D)] for c in range(C)]


def write(path=OUT):
    B = build()
    lines = [
        "// Fourier-continuation blend matrix, written by paper_2301_03814_amd/fc_table.py (do not edit).",
        "// Row c, column i: weight of the i-th of the last kFcMatch samples (increasing z) in the",
        "// continuation value c + 1 cells beyond the last sample.",
        "#pragma once",
        "",
        "namespace swkb {",
        "",
        f"constexpr int kFcMatch = {D};",
        f"constexpr int kFcCont = {C};",
        "",
        "}  // namespace swkb",
        "",
        "#define SWKB_FC_BLEND_INIT \\",
        "  { \\",
    ]
    for row in B:
        lines.append("    {" + ", ".join(f"{v!r}" for v in row) + "}, \\")
    lines += ["  }", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))
    return path


if __name__ == "__main__":
    print(write())
