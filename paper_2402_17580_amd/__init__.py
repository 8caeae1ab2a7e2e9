"""Python binding of the mstruct HIP library (gfx950).

Argument marshalling only: every step of the phase update runs in the HIP
kernels of ``libmstruct.so``; PyTorch provides device memory and streams.
The C-ABI is declared in ``include/mstruct.h``.  If the library has not been
built, importing works but every call raises ``MstructError``.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmstruct.so")

CORRECTION_T = {"next": 0, "prev": 1}
MARTENSITE = {"max": 0, "assign": 1}
MODE_PLAIN = 0
MODE_SURROGATE = 1
MODE_IMPLICIT = 2
OPTION_SKIP_COLD_WAVES = 1
OPTION_COUNT_WAVES = 2
OPTION_TILE_WAVES = 3
OPTION_WAVE_TILE_WIDTH = 4
WAVE_COUNT_NAMES = ("points_loaded", "points_stored", "still_waves", "cold_waves", "hot_waves", "flagged_waves",
                    "hot_subblocks", "indicator_subblocks")
F64_LIBRARY = 0
F64_SYNTH = 1
F64_PAPER = 2
MLP_NPARAM = 4803

STATUS = {0: "ok", -1: "invalid argument", -2: "HIP device error", -3: "out of memory",
          -4: "unsupported option", -5: "context not ready"}


class MstructError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"mstruct status {code} ({STATUS.get(code, '?')}): {msg}")
        self.code = code


class PhasesC(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_void_p), ("alpha_s", ctypes.c_void_p), ("alpha_m", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("xbt", ctypes.c_void_p)]


class ParamsC(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in
                ("T_solidus", "T_liquidus", "T_ambient", "T_alpha_s_start", "T_alpha_s_end", "T_alpha_m_start",
                 "k_alpha_eq", "k_alpha_m_eq", "c_alpha_s", "c_beta", "k1", "k2", "k3", "f", "T_alpha_s_reg")] + \
               [("correction_T", ctypes.c_int), ("martensite_mode", ctypes.c_int)]


class PhasesF64C(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_void_p), ("alpha_s", ctypes.c_void_p), ("alpha_m", ctypes.c_void_p),
                ("n", ctypes.c_int64)]


class ScanC(ctypes.Structure):
    _fields_ = [("tracks", ctypes.c_void_p), ("n_tracks", ctypes.c_int64), ("conductivity", ctypes.c_double),
                ("diffusivity", ctypes.c_double), ("T0", ctypes.c_double), ("T_clamp", ctypes.c_double),
                ("window", ctypes.c_int)]


class PointsC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64), ("h", ctypes.c_double),
                ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double),
                ("index", ctypes.c_void_p), ("n", ctypes.c_int64), ("z_top", ctypes.c_double)]


EXPORTS = ("mstruct_default_params", "mstruct_init", "mstruct_destroy", "mstruct_status_string", "mstruct_last_error", "mstruct_step",
           "mstruct_step_implicit", "mstruct_implicit_unconverged", "mstruct_set_option", "mstruct_wave_counts", "mstruct_step_f64", "mstruct_temperature", "mstruct_fused_scan_steps",
           "mstruct_fused_scan_steps_noalloc", "mstruct_gather", "mstruct_check_invariants",
           "mstruct_correct", "mstruct_mlp_set_params", "mstruct_mlp_get_params", "mstruct_mlp_forward",
           "mstruct_mlp_grad", "mstruct_mlp_train_step")

_lib = None


def lib() -> ctypes.CDLL:
    """Load libmstruct.so (raises MstructError if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MstructError(-4, f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        p, i64, d, i = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        sig = {
            "mstruct_default_params": [p], "mstruct_init": [p, i, p], "mstruct_destroy": [p],
            "mstruct_status_string": [i],
            "mstruct_last_error": [p], "mstruct_step": [p, p, p, d, p, p],
            "mstruct_step_implicit": [p, p, p, d, d, i, p, p, p],
            "mstruct_implicit_unconverged": [p, p, i, p], "mstruct_set_option": [p, i, i],
            "mstruct_wave_counts": [p, p, i, p],
            "mstruct_step_f64": [p, p, p, d, p, i, p],
            "mstruct_temperature": [p, p, p, d, p, p],
            "mstruct_fused_scan_steps": [p, p, p, d, d, i64, i, i, p, p],
            "mstruct_fused_scan_steps_noalloc": [p, p, p, d, d, i64, i, i, p, p],
            "mstruct_gather": [p, p, p, i64, p, p], "mstruct_check_invariants": [p, p, p, ctypes.c_float, p, p],
            "mstruct_correct": [p, p, p, p],
            "mstruct_mlp_set_params": [p, p, p, p, p, p], "mstruct_mlp_get_params": [p, p],
            "mstruct_mlp_forward": [p, p, i64, p, p], "mstruct_mlp_grad": [p, p, p, i64, p, p, p],
            "mstruct_mlp_train_step": [p, p, p, i64, ctypes.c_float, p, p],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name in ("mstruct_status_string", "mstruct_last_error") else ctypes.c_int
        _lib = L
    return _lib


def _dev_ptr(t, dtype, n=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise MstructError(-1, f"{name} must be a contiguous CUDA {dtype} tensor")
    if n is not None and t.numel() != n:
        raise MstructError(-1, f"{name} has {t.numel()} entries, expected {n}")
    return t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def scan_struct(scan):
    tr = np.ascontiguousarray(scan.tracks, dtype=np.float64)
    c = ScanC(tr.ctypes.data, tr.shape[0], scan.conductivity, scan.diffusivity, scan.T0, scan.T_clamp,
              int(scan.window))
    c._keep = tr
    return c


def points_struct(grid, n, z_top=math.inf, index=None):
    import torch
    ip = None
    if index is not None:
        ip = _dev_ptr(index, torch.int32, name="index")
    return PointsC(grid.nx, grid.ny, grid.nz, grid.h, grid.ox, grid.oy, grid.oz, ip, n, float(z_top))


def default_params() -> ParamsC:
    """The paper's model constants and the default readings (mstruct_default_params)."""
    p = ParamsC()
    rc = lib().mstruct_default_params(ctypes.byref(p))
    if rc != 0:
        raise MstructError(rc, "mstruct_default_params")
    return p


class Context:
    """A library context on one GPU (one process per GPU).  correction_T
    ("next" | "prev") and martensite ("max" | "assign") select the readings
    of the paper (see mstruct_params in include/mstruct.h)."""

    def __init__(self, device: int = 0, correction_T: str = "next", martensite: str = "max"):
        self._h = ctypes.c_void_p()
        p = default_params()
        p.correction_T = CORRECTION_T[correction_T]
        p.martensite_mode = MARTENSITE[martensite]
        self._check(lib().mstruct_init(ctypes.byref(p), int(device), ctypes.byref(self._h)), "mstruct_init")
        self.device = device

    def close(self):
        if self._h:
            lib().mstruct_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != 0:
            msg = lib().mstruct_last_error(self._h).decode() if self._h else ""
            raise MstructError(rc, f"{what}: {msg}")

    @staticmethod
    def _phases(beta, alpha_s, alpha_m, xbt=None):
        import torch
        n = beta.numel()
        return PhasesC(_dev_ptr(beta, torch.float32, n, "beta"), _dev_ptr(alpha_s, torch.float32, n, "alpha_s"),
                       _dev_ptr(alpha_m, torch.float32, n, "alpha_m"), n, _dev_ptr(xbt, torch.float64, n, "xbt"))

    # -- hot path ----------------------------------------------------------
    def step(self, T_prev, T_next, dt, beta, alpha_s, alpha_m, xbt=None, stream=None):
        """Explicit step in place; xbt: optional CUDA float64 tensor carrying
        the tracked X~beta (NaN-filled before first use, see new_xbt)."""
        import torch
        ph = self._phases(beta, alpha_s, alpha_m, xbt)
        self._check(lib().mstruct_step(self._h, _dev_ptr(T_prev, torch.float32, ph.n, "T_prev"),
                                       _dev_ptr(T_next, torch.float32, ph.n, "T_next"), float(dt),
                                       ctypes.byref(ph), _stream(stream)), "mstruct_step")

    def step_f64(self, T_prev, T_next, dt, beta, alpha_s, alpha_m, math=F64_LIBRARY, stream=None):
        """The explicit step in float64 (all arrays float64 CUDA tensors)."""
        import torch
        n = beta.numel()
        f = torch.float64
        ph = PhasesF64C(_dev_ptr(beta, f, n, "beta"), _dev_ptr(alpha_s, f, n, "alpha_s"),
                        _dev_ptr(alpha_m, f, n, "alpha_m"), n)
        self._check(lib().mstruct_step_f64(self._h, _dev_ptr(T_prev, f, n, "T_prev"), _dev_ptr(T_next, f, n, "T_next"),
                                           float(dt), ctypes.byref(ph), int(math), _stream(stream)),
                    "mstruct_step_f64")

    def step_implicit(self, T_prev, T_next, dt, beta, alpha_s, alpha_m, dt_sub=0.01, max_iter=50,
                      unconverged=None, xbt=None, stream=None):
        """Implicit (Crank-Nicolson, fixed-point) step; unconverged: optional
        CUDA int64 tensor of one element, incremented by the number of
        substeps that hit max_iter; xbt as for step."""
        import torch
        ph = self._phases(beta, alpha_s, alpha_m, xbt)
        up = _dev_ptr(unconverged, torch.int64, 1, "unconverged") if unconverged is not None else None
        self._check(lib().mstruct_step_implicit(self._h, _dev_ptr(T_prev, torch.float32, ph.n, "T_prev"),
                                                _dev_ptr(T_next, torch.float32, ph.n, "T_next"), float(dt),
                                                float(dt_sub), int(max_iter), ctypes.byref(ph), up,
                                                _stream(stream)), "mstruct_step_implicit")

    def set_option(self, option, value):
        self._check(lib().mstruct_set_option(self._h, int(option), int(value)), "mstruct_set_option")

    def implicit_unconverged(self, reset=False, stream=None) -> int:
        """Substeps of fused IMPLICIT runs that hit the iteration cap."""
        c = ctypes.c_int64()
        self._check(lib().mstruct_implicit_unconverged(self._h, ctypes.byref(c), int(bool(reset)), _stream(stream)),
                    "mstruct_implicit_unconverged")
        return c.value

    def wave_counts(self, reset=False, stream=None) -> dict:
        """Counts of MSTRUCT_OPTION_COUNT_WAVES (see mstruct_wave_counts)."""
        c = (ctypes.c_int64 * len(WAVE_COUNT_NAMES))()
        self._check(lib().mstruct_wave_counts(self._h, c, int(bool(reset)), _stream(stream)), "mstruct_wave_counts")
        return dict(zip(WAVE_COUNT_NAMES, list(c)))

    def temperature(self, scan, grid, t, T_out, z_top=math.inf, index=None, stream=None):
        import torch
        n = T_out.numel()
        sc, pts = scan_struct(scan), points_struct(grid, n, z_top, index)
        self._check(lib().mstruct_temperature(self._h, ctypes.byref(sc), ctypes.byref(pts), float(t),
                                              _dev_ptr(T_out, torch.float32, n, "T_out"), _stream(stream)),
                    "mstruct_temperature")

    def fused_scan_steps(self, scan, grid, t0, dt, n_steps, K, beta, alpha_s, alpha_m, z_top=math.inf,
                         mode=MODE_PLAIN, index=None, xbt=None, stream=None):
        ph = self._phases(beta, alpha_s, alpha_m, xbt)
        sc, pts = scan_struct(scan), points_struct(grid, ph.n, z_top, index)
        self._check(lib().mstruct_fused_scan_steps(self._h, ctypes.byref(sc), ctypes.byref(pts), float(t0),
                                                   float(dt), int(n_steps), int(K), int(mode), ctypes.byref(ph),
                                                   _stream(stream)), "mstruct_fused_scan_steps")

    def fused_scan_steps_noalloc(self, scan, grid, t0, dt, n_steps, K, beta, alpha_s, alpha_m, z_top=math.inf,
                                 mode=MODE_PLAIN, index=None, xbt=None, stream=None):
        """fused_scan_steps without device allocations (PLAIN and IMPLICIT
        modes; the library's fixed per-GPU array holds the call's buffers)."""
        ph = self._phases(beta, alpha_s, alpha_m, xbt)
        sc, pts = scan_struct(scan), points_struct(grid, ph.n, z_top, index)
        self._check(lib().mstruct_fused_scan_steps_noalloc(self._h, ctypes.byref(sc), ctypes.byref(pts), float(t0),
                                                           float(dt), int(n_steps), int(K), int(mode),
                                                           ctypes.byref(ph), _stream(stream)),
                    "mstruct_fused_scan_steps_noalloc")

    def gather(self, src, idx, dst, stream=None):
        import torch
        m = idx.numel()
        self._check(lib().mstruct_gather(self._h, _dev_ptr(src, torch.float32, name="src"),
                                         _dev_ptr(idx, torch.int64, m, "idx"), m,
                                         _dev_ptr(dst, torch.float32, m, "dst"), _stream(stream)),
                    "mstruct_gather")

    def check_invariants(self, beta, alpha_s, alpha_m, T=None, tol=1e-5, stream=None):
        import torch
        ph = self._phases(beta, alpha_s, alpha_m)
        out = ctypes.c_int64()
        self._check(lib().mstruct_check_invariants(self._h, ctypes.byref(ph),
                                                   _dev_ptr(T, torch.float32, ph.n, "T") if T is not None else None,
                                                   float(tol), ctypes.byref(out), _stream(stream)),
                    "mstruct_check_invariants")
        return out.value

    # -- learned surrogate ---------------------------------------------------
    def correct(self, T, beta, alpha_s, alpha_m, stream=None):
        import torch
        ph = self._phases(beta, alpha_s, alpha_m)
        self._check(lib().mstruct_correct(self._h, _dev_ptr(T, torch.float32, ph.n, "T"), ctypes.byref(ph),
                                          _stream(stream)), "mstruct_correct")

    def mlp_set_params(self, params, in_mean, in_scale, out_scale, indicator=None):
        f = lambda a, n: np.ascontiguousarray(a, dtype=np.float32).reshape(n)
        p, im, isc, osc = f(params, MLP_NPARAM), f(in_mean, 6), f(in_scale, 6), f(out_scale, 3)
        ind = None if indicator is None else f(indicator, 4)
        self._check(lib().mstruct_mlp_set_params(self._h, p.ctypes.data, im.ctypes.data, isc.ctypes.data,
                                                 osc.ctypes.data, None if ind is None else ind.ctypes.data),
                    "mstruct_mlp_set_params")

    def mlp_get_params(self):
        out = np.zeros(MLP_NPARAM, np.float32)
        self._check(lib().mstruct_mlp_get_params(self._h, out.ctypes.data), "mstruct_mlp_get_params")
        return out

    def mlp_forward(self, X, Y, stream=None):
        import torch
        B = X.shape[0]
        self._check(lib().mstruct_mlp_forward(self._h, _dev_ptr(X, torch.float32, B * 6, "X"), B,
                                              _dev_ptr(Y, torch.float32, B * 3, "Y"), _stream(stream)),
                    "mstruct_mlp_forward")

    def mlp_grad(self, X, Y, grad, loss, stream=None):
        import torch
        B = X.shape[0]
        self._check(lib().mstruct_mlp_grad(self._h, _dev_ptr(X, torch.float32, B * 6, "X"),
                                           _dev_ptr(Y, torch.float32, B * 3, "Y"), B,
                                           _dev_ptr(grad, torch.float32, MLP_NPARAM, "grad"),
                                           _dev_ptr(loss, torch.float32, 1, "loss"), _stream(stream)),
                    "mstruct_mlp_grad")

    def mlp_train_step(self, X, Y, lr, loss=None, stream=None):
        import torch
        B = X.shape[0]
        self._check(lib().mstruct_mlp_train_step(self._h, _dev_ptr(X, torch.float32, B * 6, "X"),
                                                 _dev_ptr(Y, torch.float32, B * 3, "Y"), B, float(lr),
                                                 _dev_ptr(loss, torch.float32, 1, "loss") if loss is not None
                                                 else None, _stream(stream)), "mstruct_mlp_train_step")


def new_xbt(n, device="cuda"):
    """A tracked-X~beta side array for n points, nothing tracked yet."""
    import torch
    return torch.full((n,), float("nan"), dtype=torch.float64, device=device)


def run_layers(ctx: Context, wl, beta, alpha_s, alpha_m, K=16, mode=MODE_PLAIN, index=None, layers=None,
               xbt=None, stream=None):
    """Run the layers of a workload with the fused kernel (one call per layer)."""
    for L in (wl.layers if layers is None else layers):
        ctx.fused_scan_steps(wl.scan, wl.grid, wl.t0(L), wl.dt, L.step_end - L.step_begin, K, beta, alpha_s,
                             alpha_m, z_top=L.z_top, mode=mode, index=index, xbt=xbt, stream=stream)


def run_phases(ctx: Context, pw, beta, alpha_s, alpha_m, K=16, xbt=None, stream=None):
    """Run the phases of a phased workload (scan phases with the explicit
    scheme, cool-down phases with the implicit one), one fused call each."""
    for ph in pw.phases:
        mode = MODE_IMPLICIT if ph.scheme == "implicit" else MODE_PLAIN
        ctx.fused_scan_steps(pw.scan, pw.grid, ph.t0, ph.dt, ph.n_steps, K, beta, alpha_s, alpha_m, z_top=ph.z_top,
                             mode=mode, xbt=xbt, stream=stream)


def run_layers_stepwise(ctx: Context, wl, beta, alpha_s, alpha_m, T_a, T_b, layers=None, stream=None):
    """Run the layers with the temperature-field kernel and the plain step
    kernel (T arrays ping-pong); box grids only, active suffix per layer."""
    n_plane = wl.grid.nx * wl.grid.ny
    for L in (wl.layers if layers is None else layers):
        off = wl.grid.first_active_k(L.z_top) * n_plane
        ctx.temperature(wl.scan, wl.grid, wl.t0(L), T_a, z_top=L.z_top, stream=stream)
        for s in range(L.step_end - L.step_begin):
            t1 = wl.t0(L) + (s + 1) * wl.dt
            ctx.temperature(wl.scan, wl.grid, t1, T_b, z_top=L.z_top, stream=stream)
            ctx.step(T_a[off:], T_b[off:], wl.dt, beta[off:], alpha_s[off:], alpha_m[off:], stream=stream)
            T_a, T_b = T_b, T_a
