"""Plain FP64 CPU screened-WKB oracle (ctypes wrapper around swkb_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the GPU library.  It shares no
code with the GPU path; the two meet only in the seeded inputs of the
``workloads`` module.

Functions take a workload dict (see ``workloads``) and numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "swkb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RAY_LIVE, RAY_DEAD_LAUNCH, RAY_DEAD, RAY_CAUSTIC = 0, 1, 2, 3


class _Params(C.Structure):
    _fields_ = [
        ("k", C.c_double), ("z_a", C.c_double), ("z_b", C.c_double),
        ("n_z", C.c_int32), ("n_modes", C.c_int32),
        ("x0", C.c_double), ("dx", C.c_double),
        ("n_screens", C.c_int32), ("rk4_steps", C.c_int32), ("ray_stride", C.c_int32),
        ("launch_ext_cells", C.c_int32),
        ("p2_floor", C.c_double),
        ("bc", C.c_int32),
        ("absorber_bot", C.c_double), ("absorber_top", C.c_double),
        ("medium_kind", C.c_int32), ("n_medium_params", C.c_int32),
        ("medium_params", C.POINTER(C.c_double)),
        ("caustic_tol", C.c_double),
    ]


class Counters(C.Structure):
    _fields_ = [("caustic_rays", C.c_int64), ("dead_rays", C.c_int64),
                ("folded_modes", C.c_int64), ("significant", C.c_int64),
                ("evanescent_modes", C.c_int64), ("significant_evanescent", C.c_int64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        pp = C.POINTER(_Params)
        lib.or_num_rays.argtypes = [pp]
        lib.or_modes.argtypes = [pp, dp, dp]
        lib.or_march_mode.argtypes = [pp, C.c_double, C.c_int, dp, dp, dp, dp, ip]
        lib.or_interp.argtypes = [C.c_int, dp, dp, dp, dp, ip, C.c_int, dp, dp, dp, ip]
        lib.or_screen.argtypes = [pp, C.c_int, dp, dp, C.POINTER(Counters)]
        lib.or_run.argtypes = [pp, dp, C.c_int, C.c_int, dp, C.POINTER(Counters)]
        lib.or_medium.argtypes = [pp, C.c_int, dp, dp, dp, dp, dp]
        lib.or_taper.argtypes = [pp, dp]
        lib.or_set_threads.argtypes = [C.c_int]
        lib.or_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _params(cfg):
    mp = np.ascontiguousarray(cfg["medium_params"], dtype=np.float64)
    p = _Params(cfg["k"], cfg["z_a"], cfg["z_b"], cfg["n_z"], cfg["n_modes"], cfg["x0"], cfg["dx"],
                cfg["n_screens"], cfg["rk4_steps"], cfg["ray_stride"], cfg["launch_ext_cells"],
                cfg["p2_floor"], cfg["bc"], cfg["absorber_bot"], cfg["absorber_top"],
                cfg["medium_kind"], mp.size, _dp(mp), cfg["caustic_tol"])
    p._keep = mp  # keep the parameter array alive with the struct
    return p


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def max_threads() -> int:
    return int(_load().or_max_threads())


def num_rays(cfg) -> int:
    return int(_load().or_num_rays(C.byref(_params(cfg))))


def modes(cfg, u):
    """Mode amplitudes c_j (j = n + M/2) of the field u on a screen."""
    u = np.ascontiguousarray(u, dtype=np.complex128)
    c = np.zeros(cfg["n_modes"], dtype=np.complex128)
    _check(_load().or_modes(C.byref(_params(cfg)), _dp(u.view(np.float64)), _dp(c.view(np.float64))))
    return c


def march_mode(cfg, q, j):
    """Arrival records (Z, psi, q, a, flag) of the R rays of mode j on screen q."""
    R = num_rays(cfg)
    Z, psi, qq, a = (np.zeros(R) for _ in range(4))
    flag = np.zeros(R, dtype=np.int32)
    x_q = cfg["x0"] + q * cfg["dx"]
    _check(_load().or_march_mode(C.byref(_params(cfg)), x_q, int(j), _dp(Z), _dp(psi), _dp(qq),
                                 _dp(a), _ip(flag)))
    return dict(Z=Z, psi=psi, q=qq, a=a, flag=flag)


def interp(rec, z):
    """Interpolate one mode's records at heights z: (psi, a, has, folded)."""
    R = rec["Z"].size
    z = np.ascontiguousarray(z, dtype=np.float64)
    ps, a = np.zeros(z.size), np.zeros(z.size)
    has = np.zeros(z.size, dtype=np.int32)
    arrs = [np.ascontiguousarray(rec[k], dtype=np.float64) for k in ("Z", "psi", "q", "a")]
    fl = np.ascontiguousarray(rec["flag"], dtype=np.int32)
    fold = _load().or_interp(R, *(_dp(x) for x in arrs), _ip(fl), z.size, _dp(z), _dp(ps), _dp(a), _ip(has))
    return ps, a, has.astype(bool), bool(fold)


def screen(cfg, q, u_in):
    """Field on screen q+1 from the field on screen q; returns (u_out, counters)."""
    u_in = np.ascontiguousarray(u_in, dtype=np.complex128)
    out = np.zeros(cfg["n_z"], dtype=np.complex128)
    cnt = Counters()
    _check(_load().or_screen(C.byref(_params(cfg)), int(q), _dp(u_in.view(np.float64)),
                             _dp(out.view(np.float64)), C.byref(cnt)))
    return out, cnt.as_dict()


def taper(cfg, u):
    """The exit taper W(z_m) of cfg applied to a copy of u (complex128[N])."""
    out = np.array(u, dtype=np.complex128, copy=True)
    _check(_load().or_taper(C.byref(_params(cfg)), _dp(out.view(np.float64))))
    return out


def run(cfg, u0, q_begin=0, q_end=None):
    """Screens q_begin..q_end-1; returns (history[q_end-q_begin, N], counters)."""
    if q_end is None:
        q_end = cfg["n_screens"]
    u0 = np.ascontiguousarray(u0, dtype=np.complex128)
    hist = np.zeros((q_end - q_begin, cfg["n_z"]), dtype=np.complex128)
    cnt = Counters()
    _check(_load().or_run(C.byref(_params(cfg)), _dp(u0.view(np.float64)), int(q_begin), int(q_end),
                          _dp(hist.view(np.float64)), C.byref(cnt)))
    return hist, cnt.as_dict()


def medium(cfg, x, z):
    """(eps, eps_z, eps_zz) at points (x, z) as the rays see the medium."""
    x = np.ascontiguousarray(np.broadcast_to(x, np.shape(z)), dtype=np.float64).ravel()
    z = np.ascontiguousarray(z, dtype=np.float64).ravel()
    e, ez, ezz = np.zeros(z.size), np.zeros(z.size), np.zeros(z.size)
    _check(_load().or_medium(C.byref(_params(cfg)), z.size, _dp(x), _dp(z), _dp(e), _dp(ez), _dp(ezz)))
    return e, ez, ezz
