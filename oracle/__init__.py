"""Python access to the CPU oracle (test infrastructure).

The oracle is a plain FP64 C simulator (oracle.c) of the LIF + delayed
delivery step.  Only tests, the smoke check and the benchmark's CPU-baseline
leg may import this module; the HIP library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

import netspec

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (FP contraction off)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Pop(C.Structure):
    _fields_ = [("instance", C.c_int32), ("size", C.c_int64)]


class _Proj(C.Structure):
    _fields_ = [("src_pop", C.c_int32), ("tgt_pop", C.c_int32), ("rule", C.c_int32),
                ("k", C.c_int64), ("p", C.c_double), ("w_mean", C.c_double),
                ("w_sd", C.c_double), ("delay_kind", C.c_int32), ("d0", C.c_double),
                ("d1", C.c_double), ("autapses", C.c_int32)]


class _Spec(C.Structure):
    _fields_ = [("model", C.c_int32), ("dt", C.c_double), ("tau_m", C.c_double),
                ("C_m", C.c_double), ("E_L", C.c_double), ("V_th", C.c_double),
                ("V_reset", C.c_double), ("t_ref", C.c_double), ("I_e", C.c_double),
                ("tau_syn", C.c_double), ("weight_unit", C.c_int32),
                ("poisson_lambda", C.c_double), ("w_ext", C.c_double),
                ("v0_lo", C.c_double), ("v0_hi", C.c_double),
                ("n_instances", C.c_int32), ("n_pops", C.c_int32),
                ("pops", C.POINTER(_Pop)), ("n_projs", C.c_int32),
                ("projs", C.POINTER(_Proj)), ("n_sel", C.c_int64),
                ("sel", C.POINTER(C.c_int64)), ("stdp_pop", C.c_int32),
                ("stdp_lambda", C.c_double), ("stdp_alpha", C.c_double), ("stdp_mu", C.c_double),
                ("stdp_tau_plus", C.c_double), ("stdp_tau_minus", C.c_double),
                ("stdp_w0", C.c_double), ("stdp_wmax", C.c_double),
                ("E_ex", C.c_double), ("E_in", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        L.orc_last_error.restype = C.c_char_p
        L.orc_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.orc_poisson_table.argtypes = [C.c_double, u32p, C.c_int]
        L.orc_constants.argtypes = [C.POINTER(_Spec), f64p]
        L.orc_build.argtypes = [C.POINTER(_Spec), C.c_uint64]
        L.orc_build.restype = P
        L.orc_free.argtypes = [P]
        for nm in ("orc_num_neurons", "orc_num_edges", "orc_current_step", "orc_spike_count"):
            getattr(L, nm).argtypes = [P]
            getattr(L, nm).restype = C.c_int64
        for nm in ("orc_max_delay", "orc_min_delay"):
            getattr(L, nm).argtypes = [P]
            getattr(L, nm).restype = C.c_int32
        L.orc_events.argtypes = [P]
        L.orc_events.restype = C.c_double
        L.orc_export_graph.argtypes = [P, i64p, i64p, f64p, i32p]
        L.orc_get_state.argtypes = [P, f64p, i32p, f64p, f64p]
        L.orc_set_weight.argtypes = [P, C.c_int64, C.c_double]
        L.orc_set_weights.argtypes = [P, f64p]
        L.orc_reset.argtypes = [P]
        L.orc_run.argtypes = [P, C.c_int64]
        L.orc_get_spikes.argtypes = [P, i64p, i64p]
        L.orc_run_frozen.argtypes = [P, i64p, i64p, C.c_int64, C.c_int64, P, P]
        L.orc_run_frozen_pre.argtypes = [P, i64p, i64p, C.c_int64, C.c_int64, P]
        L.orc_backward.argtypes = [P, i64p, i64p, C.c_int64, C.c_int64, f64p, f64p,
                                   C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _err(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed ({rc}): {lib().orc_last_error().decode()}")


_MODEL = {"delta": 0, "exp": 1, "alpha": 2, "cond": 3}
_RULE = {"fixed_indegree": 0, "pairwise": 1}
_DELAY = {"const": 0, "uniform_int": 1, "normal": 2}
_UNIT = {"native": 0, "psp_mV": 1}


class _SpecHolder:
    """Keeps the ctypes arrays alive while the C struct is in use."""

    def __init__(self, spec: netspec.NetSpec, sel: Optional[np.ndarray] = None):
        spec.validate()
        pops, projs = [], []
        for b, inst in enumerate(spec.instances):
            base = len(pops)
            for p in inst.pops:
                pops.append(_Pop(b, p.size))
            for pr in inst.projs:
                projs.append(_Proj(base + pr.src, base + pr.tgt, _RULE[pr.rule], pr.k, pr.p,
                                   pr.w_mean, pr.w_sd, _DELAY[pr.delay], pr.d0, pr.d1,
                                   int(pr.autapses)))
        self.pops = (_Pop * max(1, len(pops)))(*pops)
        self.projs = (_Proj * max(1, len(projs)))(*projs)
        self.sel = None
        if sel is not None:
            self.sel = np.ascontiguousarray(sel, dtype=np.int64)
        self.c = _Spec(_MODEL[spec.model], spec.dt, spec.tau_m, spec.C_m, spec.E_L, spec.V_th,
                       spec.V_reset, spec.t_ref, spec.I_e, spec.tau_syn, _UNIT[spec.weight_unit],
                       spec.poisson_lambda, spec.w_ext, spec.v0_lo, spec.v0_hi,
                       len(spec.instances), len(pops), self.pops, len(projs), self.projs,
                       0 if self.sel is None else len(self.sel),
                       None if self.sel is None else self.sel.ctypes.data_as(C.POINTER(C.c_int64)))
        self.c.E_ex, self.c.E_in = spec.E_ex, spec.E_in
        st = spec.stdp
        self.c.stdp_pop = -1 if st is None else st.pop
        if st is not None:
            self.c.stdp_lambda, self.c.stdp_alpha, self.c.stdp_mu = st.lam, st.alpha, st.mu
            self.c.stdp_tau_plus, self.c.stdp_tau_minus = st.tau_plus, st.tau_minus
            self.c.stdp_w0, self.c.stdp_wmax = st.w0, st.wmax


def philox4x64_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(np.asarray(ctr, np.uint64), np.asarray(key, np.uint64), out)
    return out


def poisson_table(lam: float) -> np.ndarray:
    thr = np.zeros(64, np.uint32)
    m = lib().orc_poisson_table(lam, thr, 64)
    if m < 0:
        raise RuntimeError(lib().orc_last_error().decode())
    return thr[:m].copy()


CONST_NAMES = ("P22", "P20", "P11", "P21", "P31", "P32", "P21s", "P22s", "jump", "conv",
               "n_ref", "tpeak")


def constants(spec: netspec.NetSpec) -> dict:
    h = _SpecHolder(spec)
    out = np.zeros(12, np.float64)
    _err(lib().orc_constants(C.byref(h.c), out), "constants")
    return dict(zip(CONST_NAMES, out.tolist()))


class OracleNet:
    """A network simulated by the oracle (FP64)."""

    def __init__(self, spec: netspec.NetSpec, seed: int, sel: Optional[np.ndarray] = None):
        self.spec = spec
        self._h = _SpecHolder(spec, sel)
        self.sel = self._h.sel
        self._p = lib().orc_build(C.byref(self._h.c), seed)
        if not self._p:
            raise RuntimeError("oracle build failed: " + lib().orc_last_error().decode())
        self.N = lib().orc_num_neurons(self._p)
        self.E = lib().orc_num_edges(self._p)
        self.n_rec = self.N if self.sel is None else len(self.sel)

    def __del__(self):
        p = getattr(self, "_p", None)
        if p:
            lib().orc_free(p)
            self._p = None

    @property
    def d_max(self) -> int:
        return lib().orc_max_delay(self._p)

    @property
    def d_min(self) -> int:
        return lib().orc_min_delay(self._p)

    @property
    def step(self) -> int:
        return lib().orc_current_step(self._p)

    @property
    def events(self) -> float:
        return lib().orc_events(self._p)

    def graph(self):
        src = np.zeros(self.E, np.int64)
        tgt = np.zeros(self.E, np.int64)
        w = np.zeros(self.E, np.float64)
        d = np.zeros(self.E, np.int32)
        _err(lib().orc_export_graph(self._p, src, tgt, w, d), "export")
        return src, tgt, w, d

    def state(self):
        V = np.zeros(self.N)
        r = np.zeros(self.N, np.int32)
        y1 = np.zeros(self.N)
        y2 = np.zeros(self.N)
        _err(lib().orc_get_state(self._p, V, r, y1, y2), "state")
        return V, r, y1, y2

    def set_weight(self, e: int, w: float) -> None:
        _err(lib().orc_set_weight(self._p, int(e), float(w)), "set_weight")

    def set_weights(self, w: np.ndarray) -> None:
        """All weights at once, canonical order."""
        w = np.ascontiguousarray(w, np.float64)
        assert w.shape == (self.E,)
        _err(lib().orc_set_weights(self._p, w), "set_weights")

    def reset(self) -> None:
        _err(lib().orc_reset(self._p), "reset")

    def run(self, n_steps: int) -> None:
        _err(lib().orc_run(self._p, n_steps), "run")

    def spikes(self):
        n = lib().orc_spike_count(self._p)
        st = np.zeros(n, np.int64)
        ids = np.zeros(n, np.int64)
        if n:
            _err(lib().orc_get_spikes(self._p, st, ids), "spikes")
        return st, ids

    def run_frozen(self, steps, ids, n_steps: int, record_x: bool = True, record_v: bool = True):
        st = np.ascontiguousarray(steps, np.int64)
        ii = np.ascontiguousarray(ids, np.int64)
        xt = np.zeros((n_steps, self.n_rec)) if record_x else None
        vt = np.zeros((n_steps, self.n_rec)) if record_v else None
        _err(lib().orc_run_frozen(self._p, st, ii, len(st), n_steps,
                                  None if xt is None else xt.ctypes.data,
                                  None if vt is None else vt.ctypes.data), "run_frozen")
        return xt, vt

    def run_frozen_pre(self, steps, ids, n_steps: int):
        """Frozen run; returns the pre-reset membrane potential [n_steps, n_rec]
        (NaN on refractory steps)."""
        st = np.ascontiguousarray(steps, np.int64)
        ii = np.ascontiguousarray(ids, np.int64)
        vp = np.zeros((n_steps, self.n_rec))
        _err(lib().orc_run_frozen_pre(self._p, st, ii, len(st), n_steps, vp.ctypes.data), "run_frozen_pre")
        return vp

    def backward(self, steps, ids, n_steps: int, vstar: np.ndarray):
        st = np.ascontiguousarray(steps, np.int64)
        ii = np.ascontiguousarray(ids, np.int64)
        vs = np.ascontiguousarray(vstar, np.float64)
        assert vs.shape == (n_steps, self.n_rec)
        grad = np.zeros(self.E)
        loss = C.c_double(0.0)
        _err(lib().orc_backward(self._p, st, ii, len(st), n_steps, vs, grad, C.byref(loss)),
             "backward")
        return grad, loss.value
