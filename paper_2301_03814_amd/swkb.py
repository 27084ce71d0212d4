"""Python binding of libswkb (include/swkb.h): argument marshalling only.

Every step of the propagation runs in the library's HIP kernels; PyTorch
provides device memory (the plan workspace, fields, history) and the
stream.  There is no CPU fallback: without the built library, or without a
GPU, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswkb.so")

(SWKB_OK, SWKB_ERR_ARG, SWKB_ERR_NOMEM, SWKB_ERR_DEVICE, SWKB_ERR_CAUSTIC, SWKB_ERR_STATE, SWKB_ERR_EVANESCENT,
 SWKB_ERR_BUSY) = range(8)
FP64, MIXED = 0, 1
BC_PERIODIC, BC_DIRICHLET, BC_NEUMANN = 0, 1, 2
MEDIUM_LINEAR, MEDIUM_EXPGAUSS, MEDIUM_GAUSSSUM, MEDIUM_MPROFILE = 0, 1, 2, 3
PROP_AUTO, PROP_MATRIX, PROP_RECOMPUTE = 0, 1, 2

EXPORTS = ["swkb_workspace_bytes", "swkb_plan", "swkb_propagate", "swkb_field", "swkb_current_screen",
           "swkb_diagnostics", "swkb_destroy", "swkb_status_string", "swkb_last_error",
           "swkb_stage_modes", "swkb_stage_rays", "swkb_num_rays", "swkb_profile", "swkb_profile_read",
           "swkb_uses_matrix", "swkb_propagate_batch", "swkb_propagate_stations", "swkb_modal_reference",
           "swkb_server_create", "swkb_server_submit", "swkb_server_step", "swkb_server_poll",
           "swkb_server_stats", "swkb_server_destroy", "swkb_graphs", "swkb_multi_create",
           "swkb_multi_get_tuning", "swkb_multi_set_tuning", "swkb_multi_tune", "swkb_multi_propagate",
           "swkb_multi_destroy", "swkb_patch_plan", "swkb_patch_info", "swkb_patch_propagate",
           "swkb_patch_field", "swkb_patch_destroy", "swkb_patch_graphs", "swkb_footprint", "swkb_plan_error",
           "swkb_propagate_static"]

MULTI_MAX_CLASSES = 16
MULTI_PERSISTENT = 2  # swkb_multi_tuning.graphs: one persistent launch


class Params(C.Structure):
    """Mirror of swkb_params (include/swkb.h), field for field."""
    _fields_ = [
        ("k", C.c_double), ("z_a", C.c_double), ("z_b", C.c_double),
        ("n_z", C.c_int32), ("n_modes", C.c_int32),
        ("x0", C.c_double), ("dx", C.c_double),
        ("n_screens", C.c_int32), ("rk4_steps", C.c_int32), ("ray_stride", C.c_int32),
        ("launch_ext_cells", C.c_int32),
        ("p2_floor", C.c_double),
        ("bc", C.c_int32), ("medium_kind", C.c_int32),
        ("absorber_bot", C.c_double), ("absorber_top", C.c_double),
        ("medium_params", C.POINTER(C.c_double)),
        ("n_medium_params", C.c_int32), ("precision", C.c_int32),
        ("eps_ref", C.c_double), ("caustic_tol", C.c_double),
        ("propagator", C.c_int32), ("max_batch", C.c_int32), ("keep_history", C.c_int32),
    ]


class Counters(C.Structure):
    _fields_ = [("caustic_rays", C.c_int64), ("dead_rays", C.c_int64), ("folded_modes", C.c_int64),
                ("significant", C.c_int64), ("screens", C.c_int64), ("rhs_evals", C.c_int64),
                ("medium_evals", C.c_int64), ("medium_terms", C.c_int64),
                ("table_evals", C.c_int64), ("evanescent_modes", C.c_int64),
                ("significant_evanescent", C.c_int64)]


class Timing(C.Structure):
    _fields_ = [("march_ms", C.c_double), ("scan_ms", C.c_double), ("fft_ms", C.c_double),
                ("superpose_ms", C.c_double), ("march_launches", C.c_int64), ("scan_launches", C.c_int64),
                ("fft_launches", C.c_int64), ("superpose_launches", C.c_int64),
                ("table_ms", C.c_double), ("table_launches", C.c_int64)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_active", C.c_int32), ("screens_per_round", C.c_int32),
                ("mode_points_per_round", C.c_double)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("n_z", C.c_int32), ("queue_us", C.c_double), ("latency_us", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("completed", C.c_int64), ("screens", C.c_int64), ("mode_points", C.c_int64),
                ("device_bytes_in_use", C.c_size_t), ("active", C.c_int32), ("pending", C.c_int32),
                ("seconds", C.c_double)]


class MultiTuning(C.Structure):
    _fields_ = [("n_classes", C.c_int32), ("class_n_z", C.c_int32 * MULTI_MAX_CLASSES),
                ("fft_elems", C.c_int32 * MULTI_MAX_CLASSES), ("apply_groups", C.c_int32 * MULTI_MAX_CLASSES),
                ("graphs", C.c_int32), ("fft_us", C.c_double * MULTI_MAX_CLASSES),
                ("apply_us", C.c_double * MULTI_MAX_CLASSES)]


PATCH_FC, PATCH_WINDOWED = 0, 1


class PatchConfig(C.Structure):
    _fields_ = [("n_patches", C.c_int32), ("width", C.c_double), ("margin", C.c_double),
                ("method", C.c_int32)]


REQ_PENDING, REQ_ACTIVE, REQ_DONE, REQ_FAILED = range(4)


class SwkbError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"swkb error {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libswkb.so (built by paper_2301_03814_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libswkb.so not built ({path}); run paper_2301_03814_amd.build.build()")
    lib = C.CDLL(path)
    vp, i32, pp = C.c_void_p, C.c_int32, C.POINTER(Params)
    lib.swkb_workspace_bytes.argtypes = [pp]
    lib.swkb_workspace_bytes.restype = C.c_size_t
    lib.swkb_footprint.argtypes = [pp]
    lib.swkb_footprint.restype = C.c_size_t
    lib.swkb_plan_error.argtypes = [vp]
    lib.swkb_plan_error.restype = C.c_char_p
    lib.swkb_propagate_static.argtypes = [pp, vp, i32, i32, vp, vp, vp]
    lib.swkb_propagate_static.restype = C.c_int
    lib.swkb_plan.argtypes = [pp, vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.swkb_propagate.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.swkb_field.argtypes = [vp, i32, vp, vp]
    lib.swkb_propagate_batch.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp]
    lib.swkb_propagate_batch.restype = C.c_int
    lib.swkb_propagate_stations.argtypes = [vp, vp, i32, C.POINTER(C.c_int32), i32, vp, vp]
    lib.swkb_propagate_stations.restype = C.c_int
    lib.swkb_modal_reference.argtypes = [pp, vp, C.POINTER(C.c_double), i32, vp, vp]
    lib.swkb_modal_reference.restype = C.c_int
    lib.swkb_current_screen.argtypes = [vp]
    lib.swkb_current_screen.restype = i32
    lib.swkb_diagnostics.argtypes = [vp, vp, C.POINTER(Counters)]
    lib.swkb_destroy.argtypes = [vp]
    lib.swkb_destroy.restype = None
    lib.swkb_status_string.argtypes = [C.c_int]
    lib.swkb_status_string.restype = C.c_char_p
    lib.swkb_last_error.restype = C.c_char_p
    lib.swkb_stage_modes.argtypes = [vp, vp, vp, vp]
    lib.swkb_stage_rays.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
    lib.swkb_num_rays.argtypes = [vp]
    lib.swkb_num_rays.restype = i32
    lib.swkb_profile.argtypes = [vp, i32]
    lib.swkb_graphs.argtypes = [vp, i32]
    lib.swkb_graphs.restype = C.c_int
    lib.swkb_uses_matrix.argtypes = [vp]
    lib.swkb_uses_matrix.restype = i32
    lib.swkb_profile_read.argtypes = [vp, vp, C.POINTER(Timing)]
    lib.swkb_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(vp)]
    lib.swkb_server_submit.argtypes = [vp, pp, vp, C.POINTER(C.c_int64)]
    lib.swkb_server_step.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    lib.swkb_server_poll.argtypes = [vp, C.c_int64, vp, C.POINTER(RequestInfo)]
    lib.swkb_server_stats.argtypes = [vp, C.POINTER(ServerStats)]
    lib.swkb_server_destroy.argtypes = [vp]
    lib.swkb_server_destroy.restype = None
    lib.swkb_multi_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp)]
    lib.swkb_multi_get_tuning.argtypes = [vp, C.POINTER(MultiTuning)]
    lib.swkb_multi_set_tuning.argtypes = [vp, C.POINTER(MultiTuning)]
    lib.swkb_multi_tune.argtypes = [vp, i32, vp, C.POINTER(MultiTuning)]
    lib.swkb_multi_propagate.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), vp]
    lib.swkb_multi_destroy.argtypes = [vp]
    lib.swkb_multi_destroy.restype = None
    lib.swkb_patch_plan.argtypes = [pp, C.POINTER(PatchConfig), vp, C.POINTER(vp)]
    lib.swkb_patch_info.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.swkb_patch_propagate.argtypes = [vp, vp, i32, i32, vp, vp]
    lib.swkb_patch_field.argtypes = [vp, vp, vp]
    lib.swkb_patch_graphs.argtypes = [vp, i32]
    lib.swkb_patch_graphs.restype = C.c_int
    lib.swkb_patch_destroy.argtypes = [vp]
    lib.swkb_patch_destroy.restype = None
    for name in ("swkb_patch_plan", "swkb_patch_info", "swkb_patch_propagate", "swkb_patch_field"):
        getattr(lib, name).restype = C.c_int
    for name in ("swkb_multi_create", "swkb_multi_get_tuning", "swkb_multi_set_tuning", "swkb_multi_tune",
                 "swkb_multi_propagate"):
        getattr(lib, name).restype = C.c_int
    for name in ("swkb_plan", "swkb_propagate", "swkb_field", "swkb_diagnostics", "swkb_stage_modes",
                 "swkb_stage_rays", "swkb_profile", "swkb_profile_read", "swkb_server_create",
                 "swkb_server_submit", "swkb_server_step", "swkb_server_poll", "swkb_server_stats"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(status):
    if status != SWKB_OK:
        raise SwkbError(status, _lib.swkb_last_error().decode())


def make_params(cfg, precision=FP64):
    """swkb_params from a workload dict (keys as in the workloads module)."""
    mp = np.ascontiguousarray(cfg["medium_params"], dtype=np.float64)
    p = Params(
        k=cfg["k"], z_a=cfg["z_a"], z_b=cfg["z_b"], n_z=cfg["n_z"], n_modes=cfg["n_modes"],
        x0=cfg["x0"], dx=cfg["dx"], n_screens=cfg["n_screens"], rk4_steps=cfg["rk4_steps"],
        ray_stride=cfg["ray_stride"], launch_ext_cells=cfg["launch_ext_cells"], p2_floor=cfg["p2_floor"],
        bc=cfg["bc"], medium_kind=cfg["medium_kind"], absorber_bot=cfg["absorber_bot"],
        absorber_top=cfg["absorber_top"], medium_params=mp.ctypes.data_as(C.POINTER(C.c_double)),
        n_medium_params=mp.size, precision=int(precision), eps_ref=cfg["eps_ref"],
        caustic_tol=cfg["caustic_tol"], propagator=int(cfg.get("propagator", PROP_AUTO)),
        max_batch=int(cfg.get("max_batch", 1)), keep_history=int(cfg.get("keep_history", 0)))
    p._keep = mp
    return p


def workspace_bytes(cfg, precision=FP64) -> int:
    return int(load().swkb_workspace_bytes(C.byref(make_params(cfg, precision))))


def footprint(cfg, precision=FP64) -> int:
    """Device bytes one propagation request holds while it runs (swkb_footprint)."""
    return int(load().swkb_footprint(C.byref(make_params(cfg, precision))))


STATIC_WORKSPACE_BYTES = 64 << 20  # SWKB_STATIC_WORKSPACE_BYTES


def propagate_static(cfg, u0, q_begin=0, q_end=None, precision=FP64, history=True, stream=None):
    """One propagation through swkb_propagate_static (no device allocation
    inside the library): returns (history [q_end-q_begin, N] or None, field
    on screen q_end [N]), complex128 on u0's device."""
    import torch
    if q_end is None:
        q_end = cfg["n_screens"]
    p = make_params(cfg, precision)
    n = cfg["n_z"]
    hist = torch.empty((q_end - q_begin, n), dtype=torch.complex128, device=u0.device) if history else None
    out = torch.empty(n, dtype=torch.complex128, device=u0.device)
    _check(load().swkb_propagate_static(C.byref(p), _dev_ptr(u0, torch.complex128, n, "u0"), int(q_begin),
                                        int(q_end), C.c_void_p(hist.data_ptr()) if hist is not None else None,
                                        C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return hist, out


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name} must be a contiguous {dtype} tensor with {numel} elements")
    return C.c_void_p(t.data_ptr())


def modal_reference(cfg, u0, xs, stream=None):
    """Separation-of-variables reference (x-invariant media) on the GPU:
    fields at ranges xs (from the screen of u0), complex128 [len(xs), N]."""
    import torch
    lib = load()
    p = make_params(cfg)
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.float64))
    out = torch.empty((xs.size, cfg["n_z"]), dtype=torch.complex128, device=u0.device)
    _check(lib.swkb_modal_reference(C.byref(p), _dev_ptr(u0, torch.complex128, cfg["n_z"], "u0"),
                                    xs.ctypes.data_as(C.POINTER(C.c_double)), int(xs.size),
                                    C.c_void_p(out.data_ptr()), _stream_handle(stream)))
    return out


class Plan:
    """One propagation problem resident on the GPU (workspace owned here)."""

    def __init__(self, cfg, precision=FP64, device="cuda", stream=None):
        import torch
        lib = load()
        self.cfg = cfg
        self.precision = precision
        self._params = make_params(cfg, precision)
        nbytes = lib.swkb_workspace_bytes(C.byref(self._params))
        if nbytes == 0:
            raise SwkbError(SWKB_ERR_ARG, "invalid parameters")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.device = self.workspace.device
        h = C.c_void_p()
        _check(lib.swkb_plan(C.byref(self._params), C.c_void_p(self.workspace.data_ptr()), nbytes,
                             _stream_handle(stream), C.byref(h)))
        self._h = h
        self.n_z = cfg["n_z"]
        self.n_modes = cfg["n_modes"]
        self.num_rays = int(lib.swkb_num_rays(h))
        self.uses_matrix = bool(lib.swkb_uses_matrix(h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.swkb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def current_screen(self) -> int:
        return int(_lib.swkb_current_screen(self._h))

    def propagate(self, u0=None, q_begin=0, q_end=None, history=True, out=None, stream=None):
        """Screens q_begin..q_end-1.  Returns the history [q_end-q_begin, N]
        (complex128, device) when history is True, else None."""
        import torch
        if q_end is None:
            q_end = self.cfg["n_screens"]
        up = C.c_void_p(0) if u0 is None else _dev_ptr(u0, torch.complex128, self.n_z, "u0")
        hist = None
        hp = C.c_void_p(0)
        if out is not None:
            hist = out
            hp = _dev_ptr(out, torch.complex128, (q_end - q_begin) * self.n_z, "out")
        elif history:
            hist = torch.empty((q_end - q_begin, self.n_z), dtype=torch.complex128, device=self.device)
            hp = C.c_void_p(hist.data_ptr())
        _check(_lib.swkb_propagate(self._h, up, int(q_begin), int(q_end), hp, _stream_handle(stream)))
        return hist

    def propagate_batch(self, u0, q_begin=0, q_end=None, history=True, stream=None):
        """Carry B fields (u0: complex128 [B, N] on the device) across screens
        q_begin..q_end-1 together.  Returns (history [q_end-q_begin, B, N] or
        None, fields on screen q_end [B, N])."""
        import torch
        if q_end is None:
            q_end = self.cfg["n_screens"]
        if u0.dim() != 2:
            raise ValueError("u0 must be [B, N]")
        B = int(u0.shape[0])
        up = _dev_ptr(u0, torch.complex128, B * self.n_z, "u0")
        hist = None
        hp = C.c_void_p(0)
        if history:
            hist = torch.empty((q_end - q_begin, B, self.n_z), dtype=torch.complex128, device=self.device)
            hp = C.c_void_p(hist.data_ptr())
        out = torch.empty((B, self.n_z), dtype=torch.complex128, device=self.device)
        _check(_lib.swkb_propagate_batch(self._h, up, B, int(q_begin), int(q_end), hp, C.c_void_p(out.data_ptr()),
                                         _stream_handle(stream)))
        return hist, out

    def stations(self, u, q, stations, stream=None):
        """Fields at x_q + i dx/S for i in stations, from the field u on screen q.
        Returns complex128 [len(stations), N] on the device."""
        import torch
        st = np.ascontiguousarray(np.asarray(stations, dtype=np.int32))
        out = torch.empty((st.size, self.n_z), dtype=torch.complex128, device=self.device)
        _check(_lib.swkb_propagate_stations(self._h, _dev_ptr(u, torch.complex128, self.n_z, "u"), int(q),
                                            st.ctypes.data_as(C.POINTER(C.c_int32)), int(st.size),
                                            C.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def field(self, q=-1, stream=None):
        """The field on screen q (complex128 [N], device); q = -1: the current one."""
        import torch
        out = torch.empty(self.n_z, dtype=torch.complex128, device=self.device)
        _check(_lib.swkb_field(self._h, int(q), C.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    @property
    def last_error(self) -> str:
        return _lib.swkb_plan_error(self._h).decode()

    def diagnostics(self, stream=None, raise_on_caustic=False):
        """Counters summed over the screens so far.  raise_on_caustic: raise on
        SWKB_ERR_CAUSTIC or SWKB_ERR_EVANESCENT instead of returning them."""
        cnt = Counters()
        st = _lib.swkb_diagnostics(self._h, _stream_handle(stream), C.byref(cnt))
        if st not in (SWKB_OK, SWKB_ERR_CAUSTIC, SWKB_ERR_EVANESCENT) or (raise_on_caustic and st != SWKB_OK):
            _check(st)
        return {f: int(getattr(cnt, f)) for f, _ in Counters._fields_}

    def graphs(self, enable=True):
        """Capture screen ranges into HIP graphs and replay them (swkb_graphs)."""
        _check(_lib.swkb_graphs(self._h, 1 if enable else 0))

    def profile(self, enable=True):
        """Record HIP events around every kernel launch of this plan."""
        _check(_lib.swkb_profile(self._h, 1 if enable else 0))

    def profile_read(self, stream=None):
        """Device milliseconds and launch counts per kernel class since the last read."""
        t = Timing()
        _check(_lib.swkb_profile_read(self._h, _stream_handle(stream), C.byref(t)))
        return {f: (float(getattr(t, f)) if f.endswith("_ms") else int(getattr(t, f))) for f, _ in Timing._fields_}

    def stage_modes(self, u, stream=None):
        import torch
        c = torch.empty(self.n_modes, dtype=torch.complex128, device=self.device)
        _check(_lib.swkb_stage_modes(self._h, _dev_ptr(u, torch.complex128, self.n_z, "u"),
                                     C.c_void_p(c.data_ptr()), _stream_handle(stream)))
        return c

    def stage_rays(self, q, stream=None):
        import torch
        n = self.n_modes * self.num_rays
        shape = (self.n_modes, self.num_rays)
        arrs = {k: torch.empty(shape, dtype=torch.float64, device=self.device) for k in ("Z", "psi", "q", "a")}
        arrs["flag"] = torch.empty(shape, dtype=torch.int32, device=self.device)
        _check(_lib.swkb_stage_rays(self._h, int(q), *(C.c_void_p(arrs[k].data_ptr())
                                                          for k in ("Z", "psi", "q", "a", "flag")),
                                    _stream_handle(stream)))
        del n
        return arrs


class Multi:
    """Several x-invariant problems (each a mixed-precision matrix Plan) carried
    to their last screens together, one launch per stage per screen step for
    all problems still running (swkb_multi_*).  The plans must outlive it."""

    def __init__(self, plans):
        lib = load()
        self.plans = list(plans)
        arr = (C.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = C.c_void_p()
        _check(lib.swkb_multi_create(arr, len(self.plans), C.byref(h)))
        self._h = h

    @staticmethod
    def _tuning_dict(t):
        n = t.n_classes
        return {"n_z": list(t.class_n_z[:n]), "fft_elems": list(t.fft_elems[:n]),
                "apply_groups": list(t.apply_groups[:n]), "graphs": t.graphs == 1,
                "persistent": t.graphs == MULTI_PERSISTENT,
                "fft_us": list(t.fft_us[:n]), "apply_us": list(t.apply_us[:n])}

    def tuning(self):
        t = MultiTuning()
        _check(_lib.swkb_multi_get_tuning(self._h, C.byref(t)))
        return self._tuning_dict(t)

    def set_tuning(self, fft_elems=None, apply_groups=None, graphs=None, persistent=None):
        """Change launch shapes: per-class lists (ascending n_z) or None to
        keep; graphs: capture and replay the per-stage launches; persistent:
        one cooperative launch for every step instead."""
        t = MultiTuning()
        _check(_lib.swkb_multi_get_tuning(self._h, C.byref(t)))
        for name, vals in (("fft_elems", fft_elems), ("apply_groups", apply_groups)):
            if vals is not None:
                if len(vals) != t.n_classes:
                    raise ValueError(f"{name} needs {t.n_classes} values")
                for i, v in enumerate(vals):
                    getattr(t, name)[i] = int(v)
        if graphs is not None:
            t.graphs = 1 if graphs else 0
        if persistent:
            t.graphs = MULTI_PERSISTENT
        elif persistent is not None and t.graphs == MULTI_PERSISTENT:
            t.graphs = 0
        _check(_lib.swkb_multi_set_tuning(self._h, C.byref(t)))

    def tune(self, reps=10, stream=None):
        """Autotune the launch shapes on the device; returns the chosen tuning."""
        t = MultiTuning()
        _check(_lib.swkb_multi_tune(self._h, int(reps), _stream_handle(stream), C.byref(t)))
        return self._tuning_dict(t)

    def propagate(self, u0s, history=False, stream=None):
        """u0s: one complex128[n_z] device tensor per plan (screen 0).
        history: False, True (every problem) or a collection of plan indices.
        Returns a list with each problem's history (complex128 [n_screens,
        n_z]) or None; the final fields are then available from each plan's
        field()."""
        import torch
        if len(u0s) != len(self.plans):
            raise ValueError("one incident field per plan")
        ptrs = [_dev_ptr(u, torch.complex128, p.n_z, f"u0s[{i}]").value
                for i, (u, p) in enumerate(zip(u0s, self.plans))]
        uin = (C.c_void_p * len(ptrs))(*ptrs)
        hists = None
        hp = None
        if history is not False and history is not None:
            want = set(range(len(self.plans))) if history is True else set(history)
            hists = [torch.empty((p.cfg["n_screens"], p.n_z), dtype=torch.complex128, device=p.device)
                     if i in want else None for i, p in enumerate(self.plans)]
            hp = (C.c_void_p * len(hists))(*[h.data_ptr() if h is not None else None for h in hists])
        _check(_lib.swkb_multi_propagate(self._h, uin, hp, _stream_handle(stream)))
        return hists

    def close(self):
        if getattr(self, "_h", None):
            _lib.swkb_multi_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PatchPlan:
    """The screen step on overlapping patches (swkb_patch_*): by default the
    paper's Fourier-continuation patches (method=PATCH_FC), or the library's
    windowed pieces (method=PATCH_WINDOWED)."""

    def __init__(self, cfg, n_patches, width, margin, precision=FP64, stream=None, method=PATCH_FC):
        lib = load()
        self.cfg = cfg
        self.n_z = cfg["n_z"]
        self._params = make_params(cfg, precision)
        pc = PatchConfig(n_patches=int(n_patches), width=float(width), margin=float(margin), method=int(method))
        h = C.c_void_p()
        _check(lib.swkb_patch_plan(C.byref(self._params), C.byref(pc), _stream_handle(stream), C.byref(h)))
        self._h = h
        self.n_patches = int(n_patches)

    def info(self):
        """[(start index, points, modes)] of the sub-domains."""
        out = []
        for p in range(self.n_patches):
            a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
            _check(_lib.swkb_patch_info(self._h, p, C.byref(a), C.byref(b), C.byref(c)))
            out.append((a.value, b.value, c.value))
        return out

    def propagate(self, u0=None, q_begin=0, q_end=None, history=True, out=None, stream=None):
        """Screens q_begin..q_end-1; returns the history [q_end-q_begin, N]
        (into `out` if given) when history is True, else None."""
        import torch
        if q_end is None:
            q_end = self.cfg["n_screens"]
        up = C.c_void_p(0) if u0 is None else _dev_ptr(u0, torch.complex128, self.n_z, "u0")
        hist = None
        hp = C.c_void_p(0)
        if out is not None:
            hist = out
            hp = _dev_ptr(out, torch.complex128, (q_end - q_begin) * self.n_z, "out")
        elif history:
            hist = torch.empty((q_end - q_begin, self.n_z), dtype=torch.complex128, device="cuda")
            hp = C.c_void_p(hist.data_ptr())
        _check(_lib.swkb_patch_propagate(self._h, up, int(q_begin), int(q_end), hp, _stream_handle(stream)))
        return hist

    def graphs(self, enable=True):
        """Capture screen ranges into HIP graphs and replay them (swkb_patch_graphs)."""
        _check(_lib.swkb_patch_graphs(self._h, 1 if enable else 0))

    def field(self, stream=None):
        import torch
        out = torch.empty(self.n_z, dtype=torch.complex128, device="cuda")
        _check(_lib.swkb_patch_field(self._h, C.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.swkb_patch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop of the library (swkb_server_*): requests are independent
    problems, admitted by device footprint and advanced together in chunks
    of screens on their own streams.  Fields are host numpy complex128."""

    def __init__(self, hbm_budget_bytes, max_active=16, screens_per_round=8, mode_points_per_round=0.0):
        lib = load()
        cfg = ServerConfig(hbm_budget_bytes=int(hbm_budget_bytes), max_active=int(max_active),
                           screens_per_round=int(screens_per_round),
                           mode_points_per_round=float(mode_points_per_round))
        h = C.c_void_p()
        _check(lib.swkb_server_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._n_z = {}

    def submit(self, cfg, u0, precision=MIXED) -> int:
        p = make_params(cfg, precision)
        u0 = np.ascontiguousarray(np.asarray(u0, dtype=np.complex128))
        if u0.shape != (cfg["n_z"],):
            raise ValueError("u0 must be complex128[n_z]")
        rid = C.c_int64()
        _check(_lib.swkb_server_submit(self._h, C.byref(p), C.c_void_p(u0.ctypes.data), C.byref(rid)))
        self._n_z[rid.value] = cfg["n_z"]
        return rid.value

    def step(self):
        """One scheduling round; returns (admitted, pending)."""
        a, b = C.c_int32(), C.c_int32()
        _check(_lib.swkb_server_step(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def poll(self, rid):
        """(state, info dict, field or None); the field is returned once, when done."""
        info = RequestInfo()
        st = _lib.swkb_server_poll(self._h, int(rid), None, C.byref(info))
        d = {"state": info.state, "queue_us": info.queue_us, "latency_us": info.latency_us}
        if st == SWKB_ERR_STATE:
            return info.state, d, None
        if st != SWKB_OK:
            _check(st)
        out = np.empty(self._n_z.pop(rid), dtype=np.complex128)
        _check(_lib.swkb_server_poll(self._h, int(rid), C.c_void_p(out.ctypes.data), None))
        return REQ_DONE, d, out

    def stats(self):
        s = ServerStats()
        _check(_lib.swkb_server_stats(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _lib.swkb_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
