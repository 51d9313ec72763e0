"""Python binding of libcortex (MI355X LIF + delayed spike delivery).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of libcortex.so.  PyTorch supplies device memory (its caching
allocator, through the allocator callbacks of ``cortex_device``) and the
stream (the current torch stream).  The functions keep the C names;
``Network`` wraps them for convenience.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcortex.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cortex.h")

ABI_VERSION = 4
OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSUPPORTED, ETIMEOUT, ETRUNC = 0, -1, -2, -3, -4, -5, -6, -7
Q = dict(NEURONS=0, SYNAPSES=1, MIN_DELAY=2, MAX_DELAY=3, TILES=4, TILE_SIZE=5, RING_SLOTS=6,
         STEP=7, EVENTS=8, SPIKES=9, DEVICE_BYTES=10, EDGE_BYTES=11, BLOCK_SIZE=12, LDS_BYTES=13,
         OFFSET_BYTES=14, STEPS_PER_SYNC=15, RING_BYTES=16, PLAN=17, NPT=18, STAGE_RECORDS=19,
         STAGE_GROUP=20)
PLAN_AUTO, PLAN_RESIDENT, PLAN_STREAMED = 0, 1, 2
_PLAN = {"auto": PLAN_AUTO, "resident": PLAN_RESIDENT, "streamed": PLAN_STREAMED}


class CortexError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cortex status {status}: {msg}")
        self.status = status


class cortex_pop(C.Structure):
    _fields_ = [("instance", C.c_int32), ("size", C.c_int64)]


class cortex_proj(C.Structure):
    _fields_ = [("src_pop", C.c_int32), ("tgt_pop", C.c_int32), ("rule", C.c_int32),
                ("k", C.c_int64), ("p", C.c_double), ("w_mean", C.c_double), ("w_sd", C.c_double),
                ("delay_kind", C.c_int32), ("d0", C.c_double), ("d1", C.c_double),
                ("autapses", C.c_int32)]


class cortex_spec(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("struct_size", C.c_uint32), ("model", C.c_int32),
                ("precision", C.c_int32), ("weight_dtype", C.c_int32), ("weight_unit", C.c_int32),
                ("dt", C.c_double), ("tau_m", C.c_double), ("C_m", C.c_double), ("E_L", C.c_double),
                ("V_th", C.c_double), ("V_reset", C.c_double), ("t_ref", C.c_double),
                ("I_e", C.c_double), ("tau_syn", C.c_double), ("poisson_lambda", C.c_double),
                ("w_ext", C.c_double), ("v0_lo", C.c_double), ("v0_hi", C.c_double),
                ("n_instances", C.c_int32), ("n_pops", C.c_int32), ("pops", C.POINTER(cortex_pop)),
                ("n_projs", C.c_int32), ("projs", C.POINTER(cortex_proj)),
                ("tile_size", C.c_int32), ("block_size", C.c_int32), ("record_steps", C.c_int64),
                ("ckpt_every", C.c_int32), ("adjoint_steps", C.c_int64),
                ("spin_limit_log2", C.c_int32), ("steps_per_sync", C.c_int32),
                ("plan_kind", C.c_int32), ("wg_per_cu", C.c_int32),
                ("stdp_enable", C.c_int32), ("stdp_pop", C.c_int32), ("stdp_lambda", C.c_double),
                ("stdp_alpha", C.c_double), ("stdp_mu", C.c_double), ("stdp_tau_plus", C.c_double),
                ("stdp_tau_minus", C.c_double), ("stdp_w0", C.c_double), ("stdp_wmax", C.c_double),
                ("E_ex", C.c_double), ("E_in", C.c_double), ("stage_records", C.c_int64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class cortex_device(C.Structure):
    _fields_ = [("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """The loaded libcortex.so; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libcortex.so not built ({LIB_PATH}); run "
                               "python -m paper_2406_03762_amd.build")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i64 = C.c_int64
        L.cortex_last_error.restype = C.c_char_p
        L.cortex_build_network.argtypes = [C.POINTER(cortex_spec), C.c_uint64, C.POINTER(cortex_device),
                                           C.POINTER(P)]
        L.cortex_step.argtypes = [P, i64]
        L.cortex_plan.argtypes = [C.POINTER(cortex_spec), C.c_int32, i64, C.c_int32, C.POINTER(i64), C.c_int32]
        L.cortex_get_spikes.argtypes = [P, i64, i64, P, P, i64, C.POINTER(i64)]
        L.cortex_clear_spikes.argtypes = [P]
        L.cortex_run_frozen.argtypes = [P, P, P, i64, i64, P, P]
        L.cortex_run_frozen_noalloc.argtypes = [P, P, P, i64, i64, P, P]
        L.cortex_backward.argtypes = [P, P, P, C.POINTER(C.c_double)]
        L.cortex_set_weights.argtypes = [P, P]
        L.cortex_reset.argtypes = [P]
        L.cortex_get_state.argtypes = [P, P, P, P, P]
        L.cortex_state_size.argtypes = [P, C.POINTER(i64)]
        L.cortex_save_state.argtypes = [P, P, i64]
        L.cortex_load_state.argtypes = [P, P, i64]
        L.cortex_export_graph.argtypes = [P, P, P, P, P]
        L.cortex_export_canonical.argtypes = [P, P]
        L.cortex_export_tiles.argtypes = [P, P, P, P]
        L.cortex_query.argtypes = [P, C.c_int, C.POINTER(i64)]
        L.cortex_kernel_timing.argtypes = [P, C.c_int]
        L.cortex_kernel_times.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.cortex_destroy.argtypes = [P]
        L.cortex_destroy.restype = None
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != OK:
        raise CortexError(rc, lib().cortex_last_error().decode())


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _dev_ptr(t, name: str, dtype, numel: int, device=None) -> Optional[int]:
    """Address of a device buffer the library reads or writes, after checking
    that it is a contiguous torch tensor of `dtype` with `numel` elements on
    the network's GPU (host memory or a wrong type would be read through a
    wrong pointer on the device)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise CortexError(EINVAL, f"{name} must be a torch tensor on the GPU, not {type(t).__name__}")
    if not t.is_cuda:
        raise CortexError(EINVAL, f"{name} must be on the GPU (got {t.device})")
    if device is not None and t.device != torch.device(device):
        raise CortexError(EINVAL, f"{name} is on {t.device}, the network on {device}")
    if t.dtype != dtype:
        raise CortexError(EINVAL, f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise CortexError(EINVAL, f"{name} must be contiguous")
    if t.numel() != numel:
        raise CortexError(EINVAL, f"{name} must have {numel} elements (got {t.numel()})")
    return t.data_ptr()


_MODEL = {"delta": 0, "exp": 1, "alpha": 2, "cond": 3}
_RULE = {"fixed_indegree": 0, "pairwise": 1}
_DELAY = {"const": 0, "uniform_int": 1, "normal": 2}
_UNIT = {"native": 0, "psp_mV": 1}


def make_spec(net, tile_size: int = 0, block_size: int = 0, record_steps: int = 0,
              ckpt_every: int = 0, adjoint_steps: int = 0, spin_limit_log2: int = 0,
              steps_per_sync: int = 0, plan: str = "auto", wg_per_cu: int = 0, stage_records: int = 0):
    """Marshal a network description (netspec.NetSpec) into cortex_spec.
    ``plan``: "auto", "resident" or "streamed" (FP32 launch plan);
    ``stage_records``: streamed plan, records per tile staged per window (0:
    automatic, negative: no staging).

    Returns (spec, keepalive)."""
    pops, projs = [], []
    for b, inst in enumerate(net.instances):
        base = len(pops)
        for p in inst.pops:
            pops.append(cortex_pop(b, p.size))
        for pr in inst.projs:
            projs.append(cortex_proj(base + pr.src, base + pr.tgt, _RULE[pr.rule], pr.k, pr.p,
                                     pr.w_mean, pr.w_sd, _DELAY[pr.delay], pr.d0, pr.d1,
                                     int(pr.autapses)))
    pa = (cortex_pop * max(1, len(pops)))(*pops)
    qa = (cortex_proj * max(1, len(projs)))(*projs)
    s = cortex_spec()
    s.abi_version = ABI_VERSION
    s.struct_size = C.sizeof(cortex_spec)
    s.model = _MODEL[net.model]
    s.precision = 1 if net.precision == "fp64" else 0
    s.weight_dtype = 1 if net.weight_dtype == "bf16" else 0
    s.weight_unit = _UNIT[net.weight_unit]
    for f in ("dt", "tau_m", "C_m", "E_L", "V_th", "V_reset", "t_ref", "I_e", "tau_syn",
              "poisson_lambda", "w_ext", "v0_lo", "v0_hi"):
        setattr(s, f, getattr(net, f))
    s.n_instances = len(net.instances)
    s.n_pops = len(pops)
    s.pops = pa
    s.n_projs = len(projs)
    s.projs = qa
    s.tile_size = tile_size
    s.block_size = block_size
    s.record_steps = record_steps
    s.ckpt_every = ckpt_every
    s.adjoint_steps = adjoint_steps
    s.spin_limit_log2 = spin_limit_log2
    s.steps_per_sync = steps_per_sync
    s.plan_kind = _PLAN[plan]
    s.E_ex, s.E_in = getattr(net, "E_ex", 0.0), getattr(net, "E_in", -85.0)
    st = getattr(net, "stdp", None)
    if st is not None:
        s.stdp_enable, s.stdp_pop = 1, st.pop
        s.stdp_lambda, s.stdp_alpha, s.stdp_mu = st.lam, st.alpha, st.mu
        s.stdp_tau_plus, s.stdp_tau_minus, s.stdp_w0, s.stdp_wmax = st.tau_plus, st.tau_minus, st.w0, st.wmax
    s.wg_per_cu = wg_per_cu
    s.stage_records = stage_records
    return s, (pa, qa)


class _TorchAllocator:
    """Device memory from torch's caching allocator for cortex_device."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device
        self.live = {}
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        except Exception:
            return None
        p = t.data_ptr()
        self.live[p] = t
        return p

    def _free(self, ptr, user):
        self.live.pop(ptr, None)


def cortex_build_network(net, seed: int, device=None, stream=None, **plan):
    """Build on the current torch device/stream; returns (handle, keepalive)."""
    import torch
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    torch.cuda.set_device(device)
    alloc = _TorchAllocator(device)
    st = torch.cuda.current_stream(device) if stream is None else stream
    dev = cortex_device(C.c_void_p(st.cuda_stream), alloc.alloc_fn, alloc.free_fn, None)
    spec, keep = make_spec(net, **plan)
    h = C.c_void_p()
    _check(lib().cortex_build_network(C.byref(spec), seed, C.byref(dev), C.byref(h)))
    return h, (alloc, keep, dev, st)


PLAN_FIELDS = ("plan", "tiles", "T", "block_size", "npt", "W", "R", "H", "chunk", "ntb_max", "lds_bytes",
               "ring_bytes", "dmin", "dmax", "xcd_map", "thread_segments", "stage_records")


def cortex_plan(net, n_cu: int = 256, lds_per_cu: int = 163840, threads_per_cu: int = 2048, **plan) -> dict:
    """The FP32 launch plan of a network description on a device of the given
    size, made on the host (no GPU needed)."""
    spec, keep = make_spec(net, **plan)
    out = (C.c_int64 * len(PLAN_FIELDS))()
    _check(lib().cortex_plan(C.byref(spec), n_cu, lds_per_cu, threads_per_cu, out, len(PLAN_FIELDS)))
    return dict(zip(PLAN_FIELDS, list(out)))


def cortex_step(h, n_steps: int) -> None:
    _check(lib().cortex_step(h, n_steps))


def cortex_kernel_timing(h, on: bool = True) -> None:
    """Streamed plan: record per-kernel HIP events in the window graph."""
    _check(lib().cortex_kernel_timing(h, int(on)))


def cortex_kernel_times(h):
    """(staging copy ms, delivery launch ms, windows averaged) of the window
    graph's last replay."""
    ms = (C.c_double * 2)()
    nw = C.c_int32()
    _check(lib().cortex_kernel_times(h, ms, C.byref(nw)))
    return ms[0], ms[1], nw.value


def cortex_query(h, what: str) -> int:
    v = C.c_int64()
    _check(lib().cortex_query(h, Q[what], C.byref(v)))
    return v.value


def cortex_get_spikes(h, step0: int, step1: int):
    cnt = C.c_int64()
    rc = lib().cortex_get_spikes(h, step0, step1, None, None, 0, C.byref(cnt))
    if rc not in (OK, ETRUNC):
        _check(rc)
    n = cnt.value
    st = np.zeros(max(1, n), np.uint32)
    ids = np.zeros(max(1, n), np.uint32)
    _check(lib().cortex_get_spikes(h, step0, step1, st.ctypes.data, ids.ctypes.data, n, C.byref(cnt)))
    return st[:n], ids[:n]


def _net_facts(h):
    """(N, E, step, fp64) of a network handle."""
    v = C.c_int64()
    out = []
    for q in ("NEURONS", "SYNAPSES", "STEP"):
        _check(lib().cortex_query(h, Q[q], C.byref(v)))
        out.append(v.value)
    return out


def _raster(steps, ids):
    st = np.ascontiguousarray(steps, np.uint32)
    ii = np.ascontiguousarray(ids, np.uint32)
    if st.shape != ii.shape or st.ndim != 1:
        raise CortexError(EINVAL, "raster steps and ids must be 1-D arrays of one length")
    return st, ii


def cortex_run_frozen(h, steps, ids, n_steps: int, x_trace=None, v_trace=None, fp64: bool = False,
                      device=None) -> None:
    """x_trace / v_trace: device tensors [n_steps, N] (float64 for FP64
    networks, float32 otherwise) or None."""
    import torch
    st, ii = _raster(steps, ids)
    N = _net_facts(h)[0]
    dt = torch.float64 if fp64 else torch.float32
    xp = _dev_ptr(x_trace, "x_trace", dt, n_steps * N, device)
    vp = _dev_ptr(v_trace, "v_trace", dt, n_steps * N, device)
    _check(lib().cortex_run_frozen(h, st.ctypes.data if len(st) else None,
                                   ii.ctypes.data if len(ii) else None, len(st), n_steps, xp, vp))


def cortex_run_frozen_noalloc(h, steps, ids, n_steps: int, x_trace=None, v_trace=None, device=None) -> None:
    """cortex_run_frozen without device allocation (FP32 networks; the raster
    must fit the library's fixed scratch array)."""
    import torch
    st, ii = _raster(steps, ids)
    N = _net_facts(h)[0]
    xp = _dev_ptr(x_trace, "x_trace", torch.float32, n_steps * N, device)
    vp = _dev_ptr(v_trace, "v_trace", torch.float32, n_steps * N, device)
    _check(lib().cortex_run_frozen_noalloc(h, st.ctypes.data if len(st) else None,
                                           ii.ctypes.data if len(ii) else None, len(st), n_steps, xp, vp))


def cortex_set_weights(h, w_canonical, device=None) -> None:
    import torch
    E = _net_facts(h)[1]
    _check(lib().cortex_set_weights(h, _dev_ptr(w_canonical, "w_canonical", torch.float32, E, device)))


def cortex_backward(h, vstar, grad_w, device=None) -> float:
    """vstar: device float32 [T, N] with T = steps simulated since the build
    or reset; grad_w: device float32 [E] (written)."""
    import torch
    N, E, T = _net_facts(h)
    if vstar is None or grad_w is None:
        # let the library report its own state errors (adjoint not enabled)
        _check(lib().cortex_backward(h, None, None, None))
    loss = C.c_double()
    _check(lib().cortex_backward(h, _dev_ptr(vstar, "vstar", torch.float32, T * N, device),
                                 _dev_ptr(grad_w, "grad_w", torch.float32, E, device), C.byref(loss)))
    return loss.value


def cortex_reset(h) -> None:
    _check(lib().cortex_reset(h))


def cortex_clear_spikes(h) -> None:
    _check(lib().cortex_clear_spikes(h))


def cortex_get_state(h, N: int):
    V = np.zeros(N)
    r = np.zeros(N, np.int32)
    y1 = np.zeros(N)
    y2 = np.zeros(N)
    _check(lib().cortex_get_state(h, V.ctypes.data, r.ctypes.data, y1.ctypes.data, y2.ctypes.data))
    return V, r, y1, y2


def cortex_state_size(h) -> int:
    n = C.c_int64(0)
    _check(lib().cortex_state_size(h, C.byref(n)))
    return n.value


def cortex_save_state(h) -> np.ndarray:
    buf = np.zeros(cortex_state_size(h), np.uint8)
    _check(lib().cortex_save_state(h, buf.ctypes.data, buf.size))
    return buf


def cortex_load_state(h, buf) -> None:
    buf = np.ascontiguousarray(np.asarray(buf, dtype=np.uint8))
    _check(lib().cortex_load_state(h, buf.ctypes.data, buf.size))


def cortex_export_graph(h, E: int):
    src = np.zeros(E, np.int64)
    tgt = np.zeros(E, np.int64)
    w = np.zeros(E, np.float64)
    d = np.zeros(E, np.int32)
    _check(lib().cortex_export_graph(h, src.ctypes.data, tgt.ctypes.data, w.ctypes.data, d.ctypes.data))
    return src, tgt, w, d


def cortex_export_canonical(h, E: int):
    c = np.zeros(E, np.int64)
    _check(lib().cortex_export_canonical(h, c.ctypes.data))
    return c


def cortex_export_tiles(h, n_tiles: int):
    s = np.zeros(n_tiles, np.int64)
    z = np.zeros(n_tiles, np.int32)
    b = np.zeros(n_tiles, np.int32)
    _check(lib().cortex_export_tiles(h, s.ctypes.data, z.ctypes.data, b.ctypes.data))
    return s, z, b


def cortex_destroy(h) -> None:
    lib().cortex_destroy(h)


class Network:
    """A network living on one GPU (convenience wrapper over the C calls)."""

    def __init__(self, net, seed: int, **plan):
        import torch
        self.spec = net
        self._h, self._keep = cortex_build_network(net, seed, **plan)
        self.device = self._keep[0].device
        self.N = cortex_query(self._h, "NEURONS")
        self.E = cortex_query(self._h, "SYNAPSES")
        self.fp64 = net.precision == "fp64"
        self.torch = torch

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            cortex_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, what: str) -> int:
        return cortex_query(self._h, what)

    def kernel_timing(self, on: bool = True) -> None:
        cortex_kernel_timing(self._h, on)

    def kernel_times(self):
        return cortex_kernel_times(self._h)

    def step(self, n_steps: int) -> None:
        cortex_step(self._h, n_steps)

    def spikes(self, step0: int = 0, step1: Optional[int] = None):
        if step1 is None:
            step1 = self.query("STEP")
        return cortex_get_spikes(self._h, step0, step1)

    def run_frozen(self, steps, ids, n_steps: int, traces: bool = True):
        """Frozen-raster run; returns (x, v) device tensors [n_steps, N] or None."""
        if not traces:
            cortex_run_frozen(self._h, steps, ids, n_steps)
            return None, None
        dt = self.torch.float64 if self.fp64 else self.torch.float32
        x = self.torch.empty((n_steps, self.N), dtype=dt, device=self.device)
        v = self.torch.empty((n_steps, self.N), dtype=dt, device=self.device)
        cortex_run_frozen(self._h, steps, ids, n_steps, x, v, fp64=self.fp64, device=self.device)
        return x, v

    def backward(self, vstar, grad=None):
        """vstar: target voltages [T, N] (numpy or torch; converted to a
        float32 device tensor); returns (grad [E] float32 on the device, loss)."""
        if isinstance(vstar, np.ndarray):
            vstar = self.torch.as_tensor(vstar, dtype=self.torch.float32, device=self.device)
        if grad is None:
            grad = self.torch.empty(self.E, dtype=self.torch.float32, device=self.device)
        loss = cortex_backward(self._h, vstar, grad, device=self.device)
        return grad, loss

    def set_weights(self, w_canonical) -> None:
        """Replace all weights (float tensor or array [E], canonical order); at step 0."""
        if isinstance(w_canonical, np.ndarray):
            w_canonical = self.torch.as_tensor(w_canonical)
        w = w_canonical.detach().to(device=self.device, dtype=self.torch.float32).contiguous()
        cortex_set_weights(self._h, w, device=self.device)
        self.torch.cuda.current_stream(self.device).synchronize()

    def canonical_weights(self):
        """The stored weights as a float64 numpy array in canonical synapse order."""
        _, _, w, _ = self.graph()
        out = np.empty_like(w)
        out[self.canonical()] = w
        return out

    def reset(self) -> None:
        cortex_reset(self._h)

    def clear_spikes(self) -> None:
        cortex_clear_spikes(self._h)

    def state(self):
        return cortex_get_state(self._h, self.N)

    def save_state(self) -> np.ndarray:
        """The network's complete dynamic state as bytes (cortex_save_state)."""
        return cortex_save_state(self._h)

    def load_state(self, buf) -> None:
        """Restore a state saved by a network of the same spec, seed and plan."""
        cortex_load_state(self._h, buf)

    def graph(self):
        return cortex_export_graph(self._h, self.E)

    def canonical(self):
        return cortex_export_canonical(self._h, self.E)

    def tiles(self):
        return cortex_export_tiles(self._h, self.query("TILES"))


# ---------------------------------------------------------------------------
# Measuring autotuner with a disk cache
# ---------------------------------------------------------------------------

TUNED_TABLE = os.path.join(HERE, "tuned_plans.json")   # shipped, read-only
TUNE_CACHE = os.environ.get("CORTEX_TUNE_CACHE",
                            os.path.join(os.path.expanduser("~"), ".cache", "cortex", "tuned_plans.json"))
PLAN_KEYS = ("plan", "wg_per_cu", "block_size", "steps_per_sync", "tile_size")


def _device_desc():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", "") or ""
    return {"name": f"{p.name} {arch.split(':')[0]}".strip(), "n_cu": int(p.multi_processor_count)}


def _library_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    with open(LIB_PATH, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def tune_key(spec, device: dict) -> str:
    """Cache key of a network description on a device: the description's
    text (sizes, connectivity, delays, models, precision) and the device's
    name and compute-unit count."""
    import hashlib
    plastic = getattr(spec, "stdp", None)
    extra = "" if plastic is None else f"|{plastic!r}"
    if spec.model == "cond":
        extra += f"|E_ex={spec.E_ex}|E_in={spec.E_in}"
    return hashlib.sha256(f"{spec!r}{extra}|{device['name']}|{device['n_cu']}".encode()).hexdigest()[:24]


def _read_table(path: str) -> dict:
    import json
    try:
        with open(path) as f:
            t = json.load(f)
        return t if isinstance(t, dict) and t.get("format") == 1 else {"format": 1, "entries": {}}
    except (OSError, ValueError):
        return {"format": 1, "entries": {}}


def lookup_plan(spec, device: Optional[dict] = None, paths=None):
    """The tuned plan request of ``spec`` on ``device`` (the current GPU by
    default): the user cache first, then the table shipped with the package.
    Returns (request dict, entry) or (None, None)."""
    device = device or _device_desc()
    key = tune_key(spec, device)
    for path in (paths or (TUNE_CACHE, TUNED_TABLE)):
        e = _read_table(path)["entries"].get(key)
        if e:
            return dict(e["request"]), e
    return None, None


def plan_candidates(spec, n_cu: int, lds_per_cu: int = 163840, threads_per_cu: int = 2048,
                    tile_sizes=(0,), windows=None):
    """Distinct launch plans of an FP32 network: requests over the plan kind,
    workgroups per compute unit, block size, exchange window and tile size,
    resolved on the host; requests that resolve to the same plan are kept
    once, and requests the device cannot hold are dropped."""
    base = cortex_plan(spec, n_cu, lds_per_cu, threads_per_cu)
    w_top = min(8, base["dmin"])
    ws = windows or sorted({w_top, max(1, w_top - 1), max(1, w_top // 2)}, reverse=True)
    seen, out = set(), []
    for kind in ("resident", "streamed"):
        for pc in (1, 2):
            for bs in (0, 512):
                for W in ws:
                    for T in tile_sizes:
                        req = dict(plan=kind, wg_per_cu=pc, block_size=bs, steps_per_sync=W, tile_size=T)
                        try:
                            p = cortex_plan(spec, n_cu, lds_per_cu, threads_per_cu, **req)
                        except CortexError as e:
                            if e.status in (EUNSUPPORTED, EINVAL):
                                continue
                            raise
                        sig = tuple(p[f] for f in PLAN_FIELDS)
                        if sig not in seen:
                            seen.add(sig)
                            out.append((req, p))
    return out


def autotune(spec, seed: int, steps: int = 2000, warmup: int = 200, tile_sizes=(0,), windows=None,
             budget_s: float = 600.0, cache: Optional[str] = TUNE_CACHE, log=None):
    """Pick the launch plan of an FP32 network by measurement: every distinct
    candidate plan (plan_candidates) is built on the current GPU, run
    ``warmup`` closed-loop steps, then timed over ``steps`` steps; the fastest
    wins.  Candidates that cannot be built on this device are skipped;
    candidates are tried in the planner's order until ``budget_s`` seconds
    have passed.  The result is stored in the JSON cache ``cache`` (None: not
    stored) under tune_key(spec, device).  Returns (best request, timings:
    list of (request, plan, seconds per step or None))."""
    import json
    import time
    import torch
    device = _device_desc()
    cands = plan_candidates(spec, device["n_cu"], tile_sizes=tile_sizes, windows=windows)
    t_start = time.perf_counter()
    timings = []
    for req, p in cands:
        if time.perf_counter() - t_start > budget_s:
            break
        try:
            g = Network(spec, seed, **req)
        except CortexError as e:
            if e.status in (EUNSUPPORTED, EINVAL):
                timings.append((req, p, None))
                continue
            raise
        try:
            g.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g.step(steps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
        finally:
            g.close()
        timings.append((req, p, dt))
        if log:
            log(f"[tune] {req} -> tiles {p['tiles']} T {p['T']} W {p['W']}: {dt * 1e6:.2f} us/step")
    done = [t for t in timings if t[2] is not None]
    if not done:
        raise CortexError(EUNSUPPORTED, "no candidate plan fits this device")
    best_req, best_plan, best_dt = min(done, key=lambda t: t[2])
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        table = _read_table(cache)
        table["entries"][tune_key(spec, device)] = {
            "request": best_req, "plan": best_plan, "seconds_per_step": best_dt,
            "device": device, "library": _library_hash(), "steps": steps,
            "candidates": [{"request": r, "seconds_per_step": d} for r, _, d in timings],
        }
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best_req, timings


class VoltageLoss:
    """Membrane-voltage loss of a network as a function of its weights, for
    torch.autograd: ``VoltageLoss.apply(w, net, vstar, n_steps, raster)``
    resets ``net``, sets the weights ``w`` (canonical order), runs
    ``n_steps`` (closed loop, or open loop on ``raster = (steps, ids)``),
    and returns L = sum_b 1/(N_b T) sum (V - V*)^2; its gradient with respect
    to ``w`` is the adjoint's, with every spike held at the time it occurred
    in this run.  ``net`` must be built with ckpt_every > 0 and
    adjoint_steps >= n_steps."""

    _fn = None

    @classmethod
    def apply(cls, w, net, vstar, n_steps: int, raster=None):
        import torch

        if cls._fn is None:
            class _Fn(torch.autograd.Function):
                @staticmethod
                def forward(ctx, w_, net_, vstar_, n_steps_, raster_):
                    net_.reset()
                    net_.set_weights(w_)
                    if raster_ is None:
                        net_.step(n_steps_)
                    else:
                        net_.run_frozen(raster_[0], raster_[1], n_steps_, traces=False)
                    grad, loss = net_.backward(vstar_)
                    ctx.save_for_backward(grad)
                    return torch.tensor(loss, dtype=torch.float64, device=w_.device)

                @staticmethod
                def backward(ctx, g_out):
                    (grad,) = ctx.saved_tensors
                    return (g_out.to(grad.dtype) * grad).to(dtype=torch.float32), None, None, None, None

            cls._fn = _Fn
        return cls._fn.apply(w, net, vstar, n_steps, raster)


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/cortex.h."""
    import re
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cortex_[a-z_]+)\s*\(", txt)))
