"""More pins of the CPU oracle: the parts the single-instance pins leave open.

- several instances: every instance draws its synapses and its Poisson drive
  from the Philox key (seed, instance) with instance-local counters, checked
  by regenerating the streams with numpy's Philox;
- the loss of the adjoint normalises each instance by its own size,
  1/(N_b T), checked against a numpy loss on the oracle's own voltage trace
  and by central differences;
- the Poisson stream: the 32-bit half and the word of the documented block
  that give the count of neuron i at step n, checked exactly;
- a Poisson input given as a PSP peak (weight unit psp_mV): the external
  events produce the superposition of unit responses (scipy matrix
  exponential) scaled so that one event peaks at w_ext mV.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import netspec
from netspec import Instance, NetSpec, Population
from tests.test_oracle_pins import _loss, _system, np_philox


def three_instance_spec(model="delta"):
    """Three balanced instances of different size, normal weights and
    integer-uniform delays, so that every word of an edge block is used."""
    J = 0.1 if model == "delta" else 40.0
    insts = [netspec.brunel_instance(ne, ni, ce, ci, J, 5.0, w_rel_sd=0.1, delay="uniform_int", d0=2, d1=9)
             for ne, ni, ce, ci in ((24, 6, 5, 2), (40, 10, 7, 3), (56, 14, 9, 4))]
    return NetSpec(model=model, tau_syn=0.5, poisson_lambda=0.0, instances=insts)


def test_instances_draw_edges_from_their_own_key_with_local_counters(orc):
    spec = three_instance_spec()
    seed = 61
    net = orc.OracleNet(spec, seed)
    src, tgt, w, d = net.graph()
    offs = np.cumsum([0] + [inst.n_neurons for inst in spec.instances])
    rng = np.random.default_rng(2)
    checked = 0
    for b, inst in enumerate(spec.instances):
        n_e, n_i = inst.pops[0].size, inst.pops[1].size
        c_e, c_i = inst.projs[0].k, inst.projs[1].k
        k_tot = c_e + c_i
        lo, hi = offs[b], offs[b + 1]
        es = np.nonzero((tgt >= lo) & (tgt < hi))[0]
        assert len(es) == (n_e + n_i) * k_tot
        # every source lies in the same instance
        assert np.all((src[es] >= lo) & (src[es] < hi))
        for e in rng.choice(es, size=30, replace=False):
            tl = int(tgt[e] - lo)
            slot_all = int(e - es[0] - tl * k_tot)
            is_e_tgt = tl < n_e
            from_e = slot_all < c_e
            proj_local = (0 if from_e else 1) if is_e_tgt else (2 if from_e else 3)
            slot = slot_all if from_e else slot_all - c_e
            wd = np_philox((tl, slot, proj_local, 1), (seed, b))
            ns, base = (n_e, 0) if from_e else (n_i, n_e)
            t_in_pop = tl if is_e_tgt else tl - n_e
            if from_e == is_e_tgt:        # same population: no autapse
                sl = (wd[0] * (ns - 1)) >> 64
                sl += 1 if sl >= t_in_pop else 0
            else:
                sl = (wd[0] * ns) >> 64
            assert src[e] == lo + base + sl
            assert d[e] == 2 + ((wd[1] * 8) >> 64)
            u1 = ((wd[2] >> 11) + 1) * 2.0 ** -53
            u2 = (wd[3] >> 11) * 2.0 ** -53
            z0 = math.sqrt(-2.0 * math.log(u1)) * math.cos(6.283185307179586 * u2)
            mean, sd = (0.1, 0.01) if from_e else (-0.5, 0.05)
            assert w[e] == pytest.approx(mean + sd * z0, rel=1e-14, abs=1e-17)
            checked += 1
    assert checked == 90


def _counting_spec(lam, sizes):
    """Delta neurons with no leak (P22 == 1), no synapses and w_ext = 1: the
    membrane potential counts the Poisson events exactly."""
    insts = [Instance([Population("A", n)], []) for n in sizes]
    return NetSpec(model="delta", tau_m=1e300, poisson_lambda=lam, w_ext=1.0, V_th=1e12,
                   V_reset=0.0, v0_lo=0.0, v0_hi=0.0, instances=insts)


@pytest.mark.parametrize("lam", [0.3, 2.0])
def test_poisson_count_is_the_documented_word_and_half(orc, lam):
    # count of neuron i (instance-local l) at step n: the number of table
    # thresholds at or below the 32-bit half (n & 1: high) of word (n & 7) >> 1
    # of the block with counter (l, n >> 3, 0, 2) and key (seed, instance)
    sizes = [37, 50]
    spec = _counting_spec(lam, sizes)
    seed, T = 19, 64
    net = orc.OracleNet(spec, seed)
    _, v = net.run_frozen(np.zeros(0, np.int64), np.zeros(0, np.int64), T, record_x=False)
    k = np.rint(np.diff(np.vstack([np.zeros((1, sum(sizes))), v]), axis=0)).astype(np.int64)
    thr = orc.poisson_table(lam).astype(np.uint64)
    rng = np.random.default_rng(4)
    for _ in range(120):
        b = int(rng.integers(0, 2))
        lid = int(rng.integers(0, sizes[b]))
        n = int(rng.integers(0, T))
        words = np_philox((lid, n >> 3, 0, 2), (seed, b))
        word = words[(n & 7) >> 1]
        u = (word >> 32) if (n & 1) else (word & 0xFFFFFFFF)
        expect = int(np.count_nonzero(thr <= u))
        assert k[n, (0 if b == 0 else sizes[0]) + lid] == expect
    assert k.sum() > 0


def test_adjoint_loss_normalises_each_instance_by_its_own_size(orc):
    spec = three_instance_spec("exp")
    N, T = spec.n_neurons, 90
    steps, ids = netspec.refractory_raster(N, T, 0.03, seed=7, n_ref=20)
    vstar = netspec.target_trace(N, T, 0.0, 10.0, seed=8)
    net = orc.OracleNet(spec, 23)
    grad, L = net.backward(steps, ids, T, vstar)
    net.reset()
    _, v = net.run_frozen(steps, ids, T)
    assert L == pytest.approx(_loss(v, vstar, spec), rel=1e-12)
    # the loss with one normalisation over all neurons differs (instances
    # of 30, 50 and 70 neurons)
    assert abs(L - ((v - vstar) ** 2).sum() / (N * T)) > 1e-3 * L
    # central differences of the numpy loss on edges of every instance
    _, tgt, w, _ = net.graph()
    offs = np.cumsum([0] + [inst.n_neurons for inst in spec.instances])
    rng = np.random.default_rng(5)
    for b in range(3):
        es = np.nonzero((tgt >= offs[b]) & (tgt < offs[b + 1]) & (grad != 0))[0]
        for e in rng.choice(es, size=5, replace=False):
            h = 1e-3 * max(abs(w[e]), 1e-3)
            vals = []
            for sgn in (1, -1):
                net.set_weight(e, w[e] + sgn * h)
                net.reset()
                _, vv = net.run_frozen(steps, ids, T)
                vals.append(_loss(vv, vstar, spec))
            net.set_weight(e, w[e])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert fd == pytest.approx(grad[e], rel=1e-5, abs=1e-9 * max(1.0, abs(L)) / h)


def _unit_response(model, t, tm=20.0, ts=0.5, C=250.0):
    """Membrane response at t to one unit synaptic input at t = 0 (exp: a
    current jump of 1 pA; alpha: a current whose peak is 1 pA)."""
    A = _system(model, tm, ts, C)
    x0 = np.array([0.0, 1.0]) if model == "exp" else np.array([0.0, 0.0, math.e / ts])
    return (scipy.linalg.expm(A * t) @ x0)[0]


@pytest.mark.parametrize("model", ["exp", "alpha"])
def test_external_events_in_psp_units_peak_at_w_ext(orc, model):
    # one neuron, rare Poisson events of w_ext = 0.5 mV (PSP peak): the trace
    # is the superposition of unit responses scaled by w_ext / peak, and an
    # isolated event peaks at w_ext on the step grid
    lam, seed, T, w_ext = 0.001, 3, 20000, 0.5
    inst = Instance([Population("A", 1)], [])
    spec = NetSpec(model=model, tau_syn=0.5, weight_unit="psp_mV", poisson_lambda=lam, w_ext=w_ext,
                   V_th=1e9, v0_lo=0.0, v0_hi=0.0, instances=[inst])
    net = orc.OracleNet(spec, seed)
    _, v = net.run_frozen(np.zeros(0, np.int64), np.zeros(0, np.int64), T, record_x=False)
    v = v[:, 0]
    thr = orc.poisson_table(lam).astype(np.uint64)
    counts = np.zeros(T, np.int64)
    for blk in range(T // 8):
        words = np_philox((0, blk, 0, 2), (seed, 0))
        for n in range(8 * blk, 8 * blk + 8):
            word = words[(n & 7) >> 1]
            u = (word >> 32) if (n & 1) else (word & 0xFFFFFFFF)
            counts[n] = int(np.count_nonzero(thr <= u))
    ev = np.nonzero(counts)[0]
    assert 5 <= len(ev) <= 60
    res = scipy.optimize.minimize_scalar(lambda t: -_unit_response(model, t), bounds=(1e-6, 40.0),
                                         method="bounded", options={"xatol": 1e-10})
    scale = w_ext / (-res.fun)
    # unit response on the step grid: powers of the one-step matrix exponential
    M = scipy.linalg.expm(_system(model, 20.0, 0.5, 250.0) * 0.1)
    x = np.array([0.0, 1.0]) if model == "exp" else np.array([0.0, 0.0, math.e / 0.5])
    h = np.zeros(T)
    for j in range(1, T):
        x = M @ x
        h[j] = x[0]
    ref = np.zeros(T)
    for n in ev:
        ref[n:] += counts[n] * scale * h[:T - n]
    assert np.allclose(v, ref, rtol=1e-9, atol=1e-12)
    # an event with no other event within 40 ms before and after it
    iso = [n for n in ev if np.all(np.abs(ev[ev != n] - n) > 400) and n + 400 < T and counts[n] == 1]
    assert iso
    n = iso[0]
    assert w_ext * (1 - 2e-3) < v[n:n + 400].max() <= w_ext * (1 + 1e-9)
