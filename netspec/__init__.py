"""Network specifications and seeded synthetic inputs.

This module is shared by the HIP library's Python binding and by the CPU
oracle.  It describes *what* network to simulate (populations, projections,
neuron parameters, drive) and draws the seeded synthetic inputs that both
sides consume (spike rasters for open-loop runs, target voltage traces for the
adjoint loss, batch instance sizes).  It holds none of the simulation
arithmetic: propagators, unit conversions, random streams, delivery and
neuron updates are implemented separately on each side.

The workloads follow the networks of the paper's evaluation (Sec. IV): a
balanced random network with fixed in-degree (the verification case, minus
plasticity) and a layered cortical microcircuit stand-in (the internal circuit
of the multi-area evaluation model).  The paper's own data (connectome, cell
densities) is not used; every network here is synthetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

MODELS = ("delta", "exp", "alpha", "cond")
RULES = ("fixed_indegree", "pairwise")
DELAYS = ("const", "uniform_int", "normal")
WEIGHT_UNITS = ("native", "psp_mV")


@dataclass
class Population:
    name: str
    size: int


@dataclass
class Projection:
    """All synapses from population ``src`` onto population ``tgt``.

    rule "fixed_indegree": every target draws ``k`` sources uniformly with
    replacement (multapses allowed).  rule "pairwise": every (source, target)
    pair is connected independently with probability ``p``.
    Weight ~ Normal(w_mean, w_sd^2), clipped at zero so it keeps the sign of
    ``w_mean``; ``w_sd == 0`` gives a constant weight.
    delay "const": ``d0`` ms; "uniform_int": integer steps uniform on
    [int(d0), int(d1)]; "normal": Normal(d0 ms, d1^2 ms^2) rounded to the
    step grid and clipped below at one step.
    """
    src: int
    tgt: int
    rule: str
    w_mean: float
    w_sd: float = 0.0
    k: int = 0
    p: float = 0.0
    delay: str = "const"
    d0: float = 1.5
    d1: float = 0.0
    autapses: bool = False


@dataclass
class Instance:
    pops: List[Population]
    projs: List[Projection]

    @property
    def n_neurons(self) -> int:
        return sum(p.size for p in self.pops)


@dataclass(frozen=True)
class Stdp:
    """Spike-timing dependent plasticity of the synapses whose source and
    target both belong to population ``pop`` (global index, instance after
    instance): power-law potentiation and multiplicative depression with
    all-to-all pairing, every delay dendritic (the rule is stated in
    oracle/oracle.h).  ``w0`` and ``wmax`` are in the weights' unit."""
    pop: int = 0
    lam: float = 0.05
    alpha: float = 1.0
    mu: float = 0.4
    tau_plus: float = 15.0
    tau_minus: float = 30.0
    w0: float = 0.1
    wmax: float = 0.5


@dataclass
class NetSpec:
    """One or more independent network instances sharing a neuron model.

    Units: ms, mV, pF, pA.  ``weight_unit`` "native" means mV jumps for the
    delta model and pA current amplitudes for exp/alpha synapses; "psp_mV"
    means every weight (and ``w_ext``) is the peak of the postsynaptic
    potential it causes, converted by each implementation to a current.
    ``poisson_lambda`` is the mean Poisson count per neuron per step; every
    count adds ``w_ext`` through the same path as a synaptic input.
    """
    model: str = "delta"
    dt: float = 0.1
    tau_m: float = 20.0
    C_m: float = 250.0
    E_L: float = 0.0
    V_th: float = 20.0
    V_reset: float = 10.0
    t_ref: float = 2.0
    I_e: float = 0.0
    tau_syn: float = 0.5
    weight_unit: str = "native"
    poisson_lambda: float = 0.0
    w_ext: float = 0.0
    v0_lo: float = 0.0
    v0_hi: float = 20.0
    instances: List[Instance] = field(default_factory=list)
    precision: str = "fp32"      # "fp32" production or "fp64" verification
    weight_dtype: str = "fp32"   # storage type of weights in fp32 mode: fp32 | bf16
    # reversal potentials (mV) of the conductance model ("cond"); like stdp,
    # left out of repr() so that other models' descriptions do not change
    E_ex: float = field(default=0.0, repr=False)
    E_in: float = field(default=-85.0, repr=False)
    # plasticity (None: static synapses); left out of repr() so that the
    # description of a static network does not change with this option
    stdp: Optional[Stdp] = field(default=None, repr=False)

    @property
    def n_neurons(self) -> int:
        return sum(inst.n_neurons for inst in self.instances)

    def validate(self) -> None:
        assert self.model in MODELS, self.model
        assert self.weight_unit in WEIGHT_UNITS
        assert self.precision in ("fp32", "fp64")
        assert self.weight_dtype in ("fp32", "bf16")
        for inst in self.instances:
            for pr in inst.projs:
                assert pr.rule in RULES and pr.delay in DELAYS
                assert 0 <= pr.src < len(inst.pops) and 0 <= pr.tgt < len(inst.pops)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def brunel_instance(n_e: int, n_i: int, c_e: int, c_i: int, J: float, g: float,
                    w_rel_sd: float = 0.0, delay: str = "const",
                    d0: float = 1.5, d1: float = 0.0) -> Instance:
    """Balanced random network: fixed in-degree c_e from E and c_i from I.

    Excitatory weight J, inhibitory weight -g*J (with relative spread
    ``w_rel_sd``).
    """
    pops = [Population("E", n_e), Population("I", n_i)]
    projs = []
    for tgt in (0, 1):
        projs.append(Projection(src=0, tgt=tgt, rule="fixed_indegree", k=c_e,
                                w_mean=J, w_sd=w_rel_sd * J,
                                delay=delay, d0=d0, d1=d1))
        projs.append(Projection(src=1, tgt=tgt, rule="fixed_indegree", k=c_i,
                                w_mean=-g * J, w_sd=w_rel_sd * g * J,
                                delay=delay, d0=d0, d1=d1))
    return Instance(pops, projs)


def brunel_lambda(eta: float, theta: float, J: float, tau_m: float, dt: float) -> float:
    """Mean external Poisson count per step, eta * nu_thr * C_E * dt."""
    return eta * theta * dt / (J * tau_m)


def brunel_1250_fp64() -> NetSpec:
    """1,250-neuron delta-LIF balanced net, FP64 verification (100 ms)."""
    J, g = 0.1, 5.0
    s = NetSpec(model="delta", poisson_lambda=brunel_lambda(2.0, 20.0, J, 20.0, 0.1),
                w_ext=J, precision="fp64",
                instances=[brunel_instance(1000, 250, 100, 25, J, g)])
    return s


def brunel_112k_alpha(scale_n: float = 1.0, scale_k: float = 1.0) -> NetSpec:
    """112,500-neuron alpha-current LIF balanced net, FP32 (1 s).

    In-degree 9,000 E + 2,250 I, weights Normal(J, (0.1 J)^2) given as PSP
    peaks, delays uniform on 5..30 steps.  ``scale_n``/``scale_k`` shrink
    the network for tests (population sizes and in-degrees).
    """
    J, g = 0.1, 5.0
    n_e = int(round(90000 * scale_n))
    n_i = int(round(22500 * scale_n))
    c_e = max(1, int(round(9000 * scale_k)))
    c_i = max(1, int(round(2250 * scale_k)))
    inst = brunel_instance(n_e, n_i, c_e, c_i, J, g, w_rel_sd=0.1,
                           delay="uniform_int", d0=5, d1=30)
    return NetSpec(model="alpha", tau_syn=0.5, weight_unit="psp_mV",
                   poisson_lambda=brunel_lambda(2.0, 20.0, J, 20.0, 0.1), w_ext=J,
                   precision="fp32", instances=[inst])


# Layered microcircuit stand-in: four layers x {E, I}.  The real population
# sizes and connection table are not used; shares and probabilities are drawn
# here with a fixed seed.
MC_LAYER_SHARE = (0.3, 0.3, 0.1, 0.3)
MC_TOTAL = 77169
MC_TARGET_SYNAPSES = 3.0e8
MC_INH_RATIO = 1.5
MC_P_SPREAD = 1.3


def microcircuit_instance(total: int = MC_TOTAL, seed: int = 3,
                          target_synapses: float = MC_TARGET_SYNAPSES,
                          w_mean: float = 87.8, g: float = -4.0,
                          inh_ratio: float = MC_INH_RATIO,
                          p_spread: float = MC_P_SPREAD) -> Instance:
    """Eight populations (four layers x {E, I}) with a seeded random table of
    pairwise connection probabilities p[target, source], log-uniform over a
    range of ratio ``p_spread`` before scaling.  Every target population's row is then
    scaled so that it expects the same excitatory in-degree K_E, and its
    inhibitory columns so that |g| K_I = inh_ratio K_E (every population
    sees the same inhibition-dominated balance, as in the asynchronous
    irregular state of balanced networks; which population connects to
    which stays random).  K_E follows from ``target_synapses`` expected
    synapses in all.  ``total`` scales the populations; keep
    target_synapses / total fixed for a same-in-degree copy of another
    size."""
    sizes = []
    for share in MC_LAYER_SHARE:
        n = int(round(total * share))
        sizes += [int(round(n * 0.8)), n - int(round(n * 0.8))]
    sizes[-2] += total - sum(sizes)
    names = ["L23E", "L23I", "L4E", "L4I", "L5E", "L5I", "L6E", "L6I"]
    rng = np.random.default_rng(seed)
    p = np.exp(rng.uniform(0.0, np.log(p_spread), size=(8, 8)))
    n = np.asarray(sizes, dtype=np.float64)
    exc = np.array([s % 2 == 0 for s in range(8)])
    k_e = target_synapses / (float(n.sum()) * (1.0 + inh_ratio / abs(g)))
    k_i = inh_ratio * k_e / abs(g)
    for t in range(8):
        p[t, exc] *= k_e / float((p[t, exc] * n[exc]).sum())
        p[t, ~exc] *= k_i / float((p[t, ~exc] * n[~exc]).sum())
    p = np.clip(p, 0.0, 1.0)
    pops = [Population(nm, sz) for nm, sz in zip(names, sizes)]
    projs = []
    for t in range(8):
        for s in range(8):
            w = w_mean if s % 2 == 0 else g * w_mean
            projs.append(Projection(src=s, tgt=t, rule="pairwise", p=float(p[t, s]),
                                    w_mean=w, w_sd=abs(0.1 * w), delay="normal",
                                    d0=1.5, d1=0.75))
    return Instance(pops, projs)


# Background Poisson count per neuron and step (weight MC_W_EXT pA, exp
# currents) of the microcircuit stand-in.  The drive alone would hold the
# free membrane at lambda/dt * w_ext * tau_syn * tau_m / C = 28 mV, above
# threshold; the inhibition-dominated recurrence brings every population
# down to about 3.5 Hz (CV about 0.45) in the CPU reference (a
# same-in-degree quarter-size copy, 0.5 s), within the 1-10 Hz asked of the
# stand-in.
MC_LAMBDA = 0.8
MC_W_EXT = 87.8


def microcircuit_77k(total: int = MC_TOTAL, target_synapses: Optional[float] = None,
                     lam: float = MC_LAMBDA) -> NetSpec:
    """Eight-population exp-current LIF microcircuit stand-in, FP32 (1 s).
    With ``total`` below 77,169 and no ``target_synapses``, a copy with the
    same mean in-degree (about 3,900)."""
    if target_synapses is None:
        target_synapses = MC_TARGET_SYNAPSES * total / MC_TOTAL
    return NetSpec(model="exp", tau_syn=0.5, weight_unit="native",
                   poisson_lambda=lam, w_ext=MC_W_EXT, precision="fp32",
                   v0_lo=0.0, v0_hi=20.0,
                   instances=[microcircuit_instance(total, target_synapses=target_synapses)])


def batch_sizes(n_instances: int = 64, lo: int = 1250, hi: int = 50000,
                seed: int = 4, multiple: int = 50) -> List[int]:
    """Instance sizes, log-uniform on [lo, hi], rounded to ``multiple``."""
    rng = np.random.default_rng(seed)
    x = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_instances))
    return [int(max(lo, min(hi, multiple * round(v / multiple)))) for v in x]


def batched_brunel(sizes: Optional[List[int]] = None) -> NetSpec:
    """Many independent delta-LIF Brunel instances with in-degree 10% of each
    population, FP32 (200 ms); the adjoint workload."""
    sizes = batch_sizes() if sizes is None else sizes
    J, g = 0.1, 5.0
    insts = []
    for n in sizes:
        n_e, n_i = (4 * n) // 5, n - (4 * n) // 5
        insts.append(brunel_instance(n_e, n_i, max(1, n_e // 10), max(1, n_i // 10), J, g))
    return NetSpec(model="delta", poisson_lambda=brunel_lambda(2.0, 20.0, J, 20.0, 0.1),
                   w_ext=J, precision="fp32", instances=insts)


def brunel_2m_bf16(scale_n: float = 1.0) -> NetSpec:
    """2M-neuron delta-LIF balanced net, bf16 weights, delays 5..30 steps."""
    J, g = 0.1, 5.0
    n_e = int(round(1_600_000 * scale_n))
    n_i = int(round(400_000 * scale_n))
    inst = brunel_instance(n_e, n_i, 9000, 2250, J, g, w_rel_sd=0.1,
                           delay="uniform_int", d0=5, d1=30)
    return NetSpec(model="delta", poisson_lambda=brunel_lambda(2.0, 20.0, J, 20.0, 0.1),
                   w_ext=J, precision="fp32", weight_dtype="bf16", instances=[inst])


def small_brunel(model: str = "delta", n_e: int = 80, n_i: int = 20, c_e: int = 8,
                 c_i: int = 2, delay: str = "uniform_int", d0: float = 2, d1: float = 7,
                 w_rel_sd: float = 0.1, precision: str = "fp32", lam: float = 2.0,
                 J: float = 0.1, g: float = 5.0, weight_unit: str = "native") -> NetSpec:
    """A tiny balanced net for brute-force and parity tests."""
    inst = brunel_instance(n_e, n_i, c_e, c_i, J, g, w_rel_sd=w_rel_sd,
                           delay=delay, d0=d0, d1=d1)
    return NetSpec(model=model, poisson_lambda=lam, w_ext=J, precision=precision,
                   weight_unit=weight_unit, instances=[inst])


# ---------------------------------------------------------------------------
# Seeded synthetic inputs
# ---------------------------------------------------------------------------

def synthetic_raster(n_neurons: int, n_steps: int, p_spike: float, seed: int,
                     step0: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Bernoulli spike raster: every (step, neuron) spikes with ``p_spike``.

    Returns (steps, ids) as uint32 arrays sorted by (step, id).
    """
    rng = np.random.default_rng(seed)
    steps_l, ids_l = [], []
    chunk = max(1, int(4_000_000 // max(1, n_neurons)))
    for s0 in range(0, n_steps, chunk):
        s1 = min(n_steps, s0 + chunk)
        m = rng.random((s1 - s0, n_neurons)) < p_spike
        st, nid = np.nonzero(m)
        steps_l.append((st + s0 + step0).astype(np.uint32))
        ids_l.append(nid.astype(np.uint32))
    if not steps_l:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    return np.concatenate(steps_l), np.concatenate(ids_l)


def sparse_raster(n_neurons: int, n_steps: int, p_spike: float, seed: int,
                  step0: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """Like synthetic_raster for large, sparse rasters: per step a binomial
    number of distinct neurons drawn uniformly."""
    rng = np.random.default_rng(seed)
    counts = rng.binomial(n_neurons, p_spike, size=n_steps)
    steps_l, ids_l = [], []
    for s, c in enumerate(counts):
        if c:
            ids_l.append(np.sort(rng.choice(n_neurons, size=int(c), replace=False)).astype(np.uint32))
            steps_l.append(np.full(int(c), s + step0, np.uint32))
    if not steps_l:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    return np.concatenate(steps_l), np.concatenate(ids_l)


def refractory_raster(n_neurons: int, n_steps: int, p_spike: float, seed: int,
                      n_ref: int) -> Tuple[np.ndarray, np.ndarray]:
    """Bernoulli raster thinned so no neuron spikes again within ``n_ref``
    steps of its previous spike (a raster a refractory neuron can produce)."""
    steps, ids = synthetic_raster(n_neurons, n_steps, p_spike, seed)
    last = np.full(n_neurons, -10**9, dtype=np.int64)
    keep = np.zeros(len(steps), dtype=bool)
    for k in range(len(steps)):
        i = ids[k]
        if int(steps[k]) - last[i] > n_ref:
            keep[k] = True
            last[i] = steps[k]
    return steps[keep], ids[keep]


def target_trace(n_neurons: int, n_steps: int, lo: float, hi: float,
                 seed: int) -> np.ndarray:
    """Target voltage trace V*[step, neuron] ~ Uniform[lo, hi] (float64)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n_steps, n_neurons))


def refractory_raster(n_neurons: int, n_steps: int, p_spike: float, n_ref: int, seed: int,
                      step0: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """A raster in which every neuron spikes with probability ``p_spike`` per
    step but never within ``n_ref`` steps of its previous spike (as a
    refractory neuron would); sorted by (step, id)."""
    rng = np.random.default_rng(seed)
    last = np.full(n_neurons, -10 ** 9, np.int64)
    steps_l, ids_l = [], []
    for s in range(n_steps):
        cand = np.nonzero(rng.random(n_neurons) < p_spike)[0]
        ok = cand[s - last[cand] > n_ref]
        if len(ok):
            last[ok] = s
            ids_l.append(ok.astype(np.uint32))
            steps_l.append(np.full(len(ok), s + step0, np.uint32))
    if not steps_l:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint32)
    return np.concatenate(steps_l), np.concatenate(ids_l)


def sample_targets(n_neurons: int, n_sample: int, seed: int) -> np.ndarray:
    """Sorted distinct neuron ids for sampled checks at full size."""
    rng = np.random.default_rng(seed)
    n_sample = min(n_sample, n_neurons)
    return np.sort(rng.choice(n_neurons, size=n_sample, replace=False)).astype(np.int64)


def with_precision(spec: NetSpec, precision: str) -> NetSpec:
    return replace(spec, precision=precision)
