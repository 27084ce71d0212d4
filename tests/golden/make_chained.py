"""Writes the chained full-size fixtures: the oracle's fields on sampled
screens of an uninterrupted screen chain (Algorithm 1 repeated from the
seeded incident beam), for the GPU tests that hold the library's own chain
against them.

Calls only the CPU oracle (``oracle``) and the seeded inputs (``workloads``).

    python tests/golden/make_chained.py [random_medium|surface_duct] [--threads T]

random_medium_chain.npz: the random medium (N = 8192, M = 2048, 400 screens
of 10 wavelengths), every 25th screen and the last.
surface_duct_chain.npz: the surface duct (N = 16384, M = 4096, Dirichlet
ground), its first 20 screens (2 km), every 4th screen.
Each file: screens (int32, 1-based screen index q of the field on x_q),
fields (complex128 [len(screens), N]), counters of the whole chain.
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

CASES = {
    "random_medium": (lambda: W.random_medium(), 400, 25),
    "surface_duct": (lambda: W.surface_duct(), 20, 4),
}


def make(name, threads):
    build, n_screens, every = CASES[name]
    cfg = build()
    oracle.set_threads(threads)
    u = W.incident_field(cfg)
    keep = sorted(set(list(range(every, n_screens + 1, every)) + [n_screens]))
    fields, cnt_all = [], {}
    t0 = time.time()
    for q in range(n_screens):
        u, cnt = oracle.screen(cfg, q, u)
        for key, val in cnt.items():
            cnt_all[key] = cnt_all.get(key, 0) + val
        if q + 1 in keep:
            fields.append(u.copy())
        print(f"[{name}] screen {q + 1}/{n_screens} {time.time() - t0:.0f}s", flush=True)
    out = os.path.join(HERE, f"{name}_chain.npz")
    np.savez(out, screens=np.array(keep, dtype=np.int32), fields=np.array(fields),
             counters=np.array([cnt_all[k] for k in sorted(cnt_all)], dtype=np.int64),
             counter_names=np.array(sorted(cnt_all)))
    print(f"[{name}] wrote {out}: screens {keep}", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=sorted(CASES))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for c in a.cases:
        make(c, a.threads)
