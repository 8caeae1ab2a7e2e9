"""FP64 CPU oracle for the Ti-6Al-4V phase update (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the HIP library or its binding.
The arithmetic lives in ``mstruct_oracle.c`` (plain C, double precision,
C-library transcendentals, OpenMP over points) and ``mlp_oracle.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mstruct_oracle.c")
_LIB = os.path.join(_HERE, "liborc_mstruct.so")
_lib = None

CONSTANT_NAMES = ("T_s", "T_l", "T_inf", "T_as_start", "T_as_end", "T_am_start",
                  "k_alpha_eq", "k_am_eq", "c_as", "c_beta", "k1", "k2", "k3", "f",
                  "T_as_reg", "x_alpha_max", "startup_limit")


def build() -> str:
    """Compile the oracle with gcc (IEEE double arithmetic, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        d, i64, p = ctypes.c_double, ctypes.c_int64, ctypes.c_void_p
        for name in ("orc_liquid_fraction", "orc_alpha_eq", "orc_am0_eq", "orc_k_as", "orc_erfcx"):
            getattr(L, name).restype = d
            getattr(L, name).argtypes = [d]
        L.orc_logistic_step.restype = d
        L.orc_logistic_step.argtypes = [d, d, d, d, d]
        L.orc_correct.restype = d
        L.orc_correct.argtypes = [d, p, p]
        L.orc_rates.restype = None
        L.orc_rates.argtypes = [d, d, d, d, p, p, p]
        L.orc_step.restype = None
        L.orc_step.argtypes = [p, p, p, p, d, d, d]
        L.orc_step_n.restype = None
        L.orc_step_n.argtypes = [i64, p, p, p, p, p, p, d]
        L.orc_source_F.restype = d
        L.orc_source_F.argtypes = [p, d, d, d, d, d, d]
        L.orc_temperature.restype = d
        L.orc_temperature.argtypes = [p, i64, p, d, d, d, d]
        L.orc_temperature_n.restype = None
        L.orc_temperature_n.argtypes = [p, i64, p, p, i64, d, p]
        L.orc_scan_run.restype = None
        L.orc_scan_run.argtypes = [p, i64, p, p, i64, d, d, d, d, i64, p, p, p, p, ctypes.c_int]
        L.orc_history_run.restype = None
        L.orc_history_run.argtypes = [i64, i64, p, d, p, p, p, p]
        L.orc_constants.restype = ctypes.c_int
        L.orc_constants.argtypes = [p, ctypes.c_int]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_step_cn.restype = ctypes.c_int
        L.orc_step_cn.argtypes = [p, p, p, p, d, d, d, ctypes.c_int, d, d]
        L.orc_substeps.restype = i64
        L.orc_substeps.argtypes = [d, d]
        L.orc_step_implicit_n.restype = i64
        L.orc_scan_run_implicit.restype = i64
        L.orc_scan_run_implicit.argtypes = [p, i64, p, p, i64, d, d, d, d, i64, d, ctypes.c_int, p, p, p, p,
                                            ctypes.c_int]
        L.orc_step_implicit_n.argtypes = [i64, p, p, p, p, p, p, d, d, ctypes.c_int, d, d, p]
        L.orc_set_readings.restype = None
        L.orc_set_readings.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_get_readings.restype = ctypes.c_int
        L.orc_get_readings.argtypes = []
        _lib = L
    return _lib


CORRECTION_T = {"next": 0, "prev": 1}
MARTENSITE = {"max": 0, "assign": 1}


def set_readings(correction_T="next", martensite="max"):
    """Switch the two readings of the paper that the library exposes: the
    temperature of the explicit correction ("next": T^{n+1} of eq.
    explicit_correction; "prev": the T^n Algorithm 2 passes) and the
    martensite formation law ("max": never lowers alpha_m; "assign": the
    literal "=" of eq. inst_martensite_formation)."""
    lib().orc_set_readings(CORRECTION_T[correction_T], MARTENSITE[martensite])


class readings:
    """Context manager: the given readings inside, the defaults after."""

    def __init__(self, correction_T="next", martensite="max"):
        self.args = (correction_T, martensite)

    def __enter__(self):
        set_readings(*self.args)
        return self

    def __exit__(self, *exc):
        set_readings()
        return False


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def constants() -> dict:
    buf = np.zeros(len(CONSTANT_NAMES), np.float64)
    lib().orc_constants(_ptr(buf), len(buf))
    return dict(zip(CONSTANT_NAMES, buf.tolist()))


def liquid_fraction(T): return lib().orc_liquid_fraction(float(T))
def alpha_eq(T): return lib().orc_alpha_eq(float(T))
def am0_eq(T): return lib().orc_am0_eq(float(T))
def k_as(T): return lib().orc_k_as(float(T))
def erfcx(y): return lib().orc_erfcx(float(y))


def logistic_step(X, D, kt, c, dt):
    return lib().orc_logistic_step(float(X), float(D), float(kt), float(c), float(dt))


def rates(a_s, a_m, xbt, T):
    r = [ctypes.c_double() for _ in range(3)]
    lib().orc_rates(float(a_s), float(a_m), float(xbt), float(T), *[ctypes.byref(x) for x in r])
    return tuple(x.value for x in r)


def correct(T, a_s, a_m):
    a, m = ctypes.c_double(a_s), ctypes.c_double(a_m)
    b = lib().orc_correct(float(T), ctypes.byref(a), ctypes.byref(m))
    return a.value, m.value, b


class State:
    """FP64 point state: alpha_s, alpha_m, beta and the shifted beta X~beta."""

    def __init__(self, beta, alpha_s, alpha_m):
        self.alpha_s = _f64(alpha_s).copy()
        self.alpha_m = _f64(alpha_m).copy()
        self.beta = _f64(beta).copy()
        self.xbt = 0.9 - (self.alpha_s + self.alpha_m)

    @classmethod
    def initial(cls, n):
        return cls(np.full(n, 0.1), np.full(n, 0.9), np.zeros(n))

    def copy(self):
        s = State(self.beta, self.alpha_s, self.alpha_m)
        s.xbt = self.xbt.copy()
        return s

    def arrays(self):
        return self.alpha_s, self.alpha_m, self.beta, self.xbt


def step(state: State, Tn, Tn1, dt):
    Tn, Tn1 = _f64(np.broadcast_to(Tn, state.beta.shape)), _f64(np.broadcast_to(Tn1, state.beta.shape))
    lib().orc_step_n(state.beta.size, *[_ptr(a) for a in state.arrays()], _ptr(Tn), _ptr(Tn1), float(dt))
    return state


CN_EPS_ABS, CN_EPS_REL, CN_MAX_ITER, DT_SUB = 1e-10, 1e-3, 50, 0.01


def step_implicit(state: State, Tn, Tn1, dt, dt_sub=DT_SUB, max_iter=CN_MAX_ITER, eps_abs=CN_EPS_ABS,
                  eps_rel=CN_EPS_REL):
    """Crank-Nicolson step with fixed-point iteration and subcycling, in
    place.  Returns (number of substeps that hit max_iter, iterations per
    point)."""
    Tn, Tn1 = _f64(np.broadcast_to(Tn, state.beta.shape)), _f64(np.broadcast_to(Tn1, state.beta.shape))
    iters = np.zeros(state.beta.size, dtype=np.int64)
    bad = lib().orc_step_implicit_n(state.beta.size, *[_ptr(a) for a in state.arrays()], _ptr(Tn), _ptr(Tn1),
                                    float(dt), float(dt_sub), int(max_iter), float(eps_abs), float(eps_rel),
                                    iters.ctypes.data_as(ctypes.c_void_p))
    return int(bad), iters


def substeps(dt, dt_sub=DT_SUB):
    return int(lib().orc_substeps(float(dt), float(dt_sub)))


def history_run(state: State, T_hist, dt):
    """T_hist: (n, n_steps+1) temperatures per point."""
    T_hist = _f64(T_hist)
    n, m = T_hist.shape
    lib().orc_history_run(n, m - 1, _ptr(T_hist), float(dt), *[_ptr(a) for a in state.arrays()])
    return state


def _scan_params(scan):
    return np.array([scan.conductivity, scan.diffusivity, scan.T0, scan.T_clamp, float(scan.window)])


def temperature(scan, xyz, t):
    xyz = _f64(np.atleast_2d(xyz))
    tr, sp = _f64(scan.tracks), _scan_params(scan)
    out = np.empty(xyz.shape[0])
    lib().orc_temperature_n(_ptr(tr), tr.shape[0], _ptr(sp), _ptr(xyz), xyz.shape[0], float(t), _ptr(out))
    return out


def source_F(track_row, tau, k, alpha, xyz):
    tr = _f64(track_row)
    return lib().orc_source_F(_ptr(tr), float(tau), float(k), float(alpha), *map(float, xyz))


def scan_run(scan, xyz, state: State, z_top, h, t0, dt, n_steps, threads=0):
    xyz = _f64(xyz)
    tr, sp = _f64(scan.tracks), _scan_params(scan)
    lib().orc_scan_run(_ptr(tr), tr.shape[0], _ptr(sp), _ptr(xyz), xyz.shape[0], float(z_top), float(h),
                       float(t0), float(dt), int(n_steps), *[_ptr(a) for a in state.arrays()], int(threads))
    return state


def scan_run_implicit(scan, xyz, state: State, z_top, h, t0, dt, n_steps, dt_sub=DT_SUB, max_iter=CN_MAX_ITER,
                      threads=0):
    """scan_run with the implicit scheme; returns the number of substeps that
    hit max_iter."""
    xyz = _f64(xyz)
    tr, sp = _f64(scan.tracks), _scan_params(scan)
    return int(lib().orc_scan_run_implicit(_ptr(tr), tr.shape[0], _ptr(sp), _ptr(xyz), xyz.shape[0], float(z_top),
                                           float(h), float(t0), float(dt), int(n_steps), float(dt_sub),
                                           int(max_iter), *[_ptr(a) for a in state.arrays()], int(threads)))


def run_workload(wl, local_points, state: State = None, threads=0, layers=None, implicit=False):
    """Run every layer of a workload at the given local point numbers (with
    the explicit scheme, or the implicit one)."""
    xyz = wl.grid.coords(np.asarray(local_points))
    if state is None:
        state = State.initial(xyz.shape[0])
    for L in (wl.layers if layers is None else layers):
        if implicit:
            scan_run_implicit(wl.scan, xyz, state, L.z_top, wl.grid.h, wl.t0(L), wl.dt, L.step_end - L.step_begin,
                              threads=threads)
        else:
            scan_run(wl.scan, xyz, state, L.z_top, wl.grid.h, wl.t0(L), wl.dt, L.step_end - L.step_begin, threads)
    return state


def num_threads():
    return lib().orc_num_threads()


def run_phases(pw, local_points, state: State = None, threads=0):
    """Run the phases of a phased workload at the given local point numbers
    (scan_run for explicit phases, scan_run_implicit for implicit ones).
    Returns (state, substeps that hit the iteration cap)."""
    xyz = pw.grid.coords(np.asarray(local_points))
    if state is None:
        state = State.initial(xyz.shape[0])
    bad = 0
    for ph in pw.phases:
        if ph.scheme == "implicit":
            bad += scan_run_implicit(pw.scan, xyz, state, ph.z_top, pw.grid.h, ph.t0, ph.dt, ph.n_steps,
                                     threads=threads)
        else:
            scan_run(pw.scan, xyz, state, ph.z_top, pw.grid.h, ph.t0, ph.dt, ph.n_steps, threads)
    return state, bad
