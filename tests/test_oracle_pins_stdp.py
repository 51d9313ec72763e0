"""Pins of the oracle's spike-timing dependent plasticity (the rule stated in
oracle/oracle.h): a two-neuron network driven by a frozen raster, whose
weights and delivered inputs are written out by hand from the rule;
clipping at both bounds; static synapses untouched; a closed-loop run and
the replay of its own raster agree exactly."""
import math

import numpy as np
import pytest

import netspec
import oracle

DT = 0.1
D = 15            # 1.5 ms in steps
LAM, ALPHA, MU, TP, TM, W0 = 0.1, 0.5, 0.4, 15.0, 30.0, 0.1


def _pair_spec(w_init, lam=LAM, alpha=ALPHA, wmax=10.0):
    # two E neurons (no autapses: each one's single in-synapse comes from the
    # other) and one I neuron fed by an E neuron (a static synapse)
    pops = [netspec.Population("E", 2), netspec.Population("I", 1)]
    projs = [netspec.Projection(0, 0, "fixed_indegree", w_init, k=1, delay="const", d0=1.5),
             netspec.Projection(0, 1, "fixed_indegree", w_init, k=1, delay="const", d0=1.5)]
    st = netspec.Stdp(pop=0, lam=lam, alpha=alpha, mu=MU, tau_plus=TP, tau_minus=TM, w0=W0, wmax=wmax)
    return netspec.NetSpec(model="delta", poisson_lambda=0.0, w_ext=0.0, V_th=1e9, V_reset=0.0,
                           v0_lo=0.0, v0_hi=0.0, instances=[netspec.Instance(pops, projs)], stdp=st)


RASTER = [(10, 0), (20, 1), (60, 0), (100, 1), (200, 0)]


def _run(spec, T=300):
    o = oracle.OracleNet(spec, 3)
    st = np.array([s for s, _ in RASTER], np.int64)
    ids = np.array([i for _, i in RASTER], np.int64)
    x, _ = o.run_frozen(st, ids, T)
    src, tgt, w, d = o.graph()
    return o, x, {(int(a), int(b)): float(c) for a, b, c in zip(src, tgt, w)}, d


def _pot(w, x, lam=LAM):
    return w + lam * W0 ** (1.0 - MU) * w ** MU * x


def test_two_neuron_pairings_follow_the_rule_by_hand():
    w_init = 0.1
    o, x, w, d = _run(_pair_spec(w_init))
    assert np.all(d == D)
    # synapse 0 -> 1: pre spikes 10, 60, 200; post spikes 20, 100
    w01_1 = w_init                                    # first pre spike, no post spike before -5
    a = _pot(w01_1, math.exp(-(35 - 10) * DT / TP))   # post 20 reaches the synapse at 35
    w01_2 = a * (1.0 - LAM * ALPHA * math.exp(-(45 - 20) * DT / TM))
    x0_60 = 1.0 + math.exp(-(60 - 10) * DT / TP)      # presynaptic trace after the spike at 60
    a = _pot(w01_2, x0_60 * math.exp(-(115 - 60) * DT / TP))
    y1_185 = (1.0 + math.exp(-(100 - 20) * DT / TM)) * math.exp(-(185 - 100) * DT / TM)
    w01_3 = a * (1.0 - LAM * ALPHA * y1_185)
    # synapse 1 -> 0: pre spikes 20, 100; post spikes 10, 60, 200
    w10_1 = w_init                                    # y_0(5) = 0
    a = _pot(w10_1, math.exp(-(25 - 20) * DT / TP))   # post 10 arrives at 25
    a = _pot(a, math.exp(-(75 - 20) * DT / TP))       # post 60 arrives at 75
    y0_85 = (1.0 + math.exp(-(60 - 10) * DT / TM)) * math.exp(-(85 - 60) * DT / TM)
    w10_2 = a * (1.0 - LAM * ALPHA * y0_85)
    assert w[(0, 1)] == pytest.approx(w01_3, rel=1e-12)
    assert w[(1, 0)] == pytest.approx(w10_2, rel=1e-12)
    # each spike is delivered with the weight it has just been given
    assert x[25, 1] == pytest.approx(w01_1, rel=1e-12)
    assert x[75, 1] == pytest.approx(w01_2, rel=1e-12)
    assert x[215, 1] == pytest.approx(w01_3, rel=1e-12)
    assert x[35, 0] == pytest.approx(w10_1, rel=1e-12)
    assert x[115, 0] == pytest.approx(w10_2, rel=1e-12)
    # the static E -> I synapse keeps its weight and delivers it
    (src_i,) = [s for (s, t) in w if t == 2]
    assert w[(src_i, 2)] == w_init
    steps_i = [s + D for s, i in RASTER if i == src_i]
    assert all(x[s, 2] == w_init for s in steps_i)
    assert w01_3 != w_init and w10_2 != w_init


def test_weights_are_clipped_at_both_bounds():
    # strong potentiation saturates at w_max ...
    _, _, w, _ = _run(_pair_spec(0.1, lam=5.0, alpha=0.0, wmax=0.15))
    assert w[(1, 0)] == 0.15 and w[(0, 1)] == 0.15
    # ... and depression with lambda alpha y > 1 stops at zero
    _, _, w, _ = _run(_pair_spec(0.1, lam=1.0, alpha=3.0))
    assert w[(1, 0)] == 0.0


def test_closed_loop_run_and_the_replay_of_its_raster_give_the_same_weights():
    spec = netspec.small_brunel(n_e=160, n_i=40, c_e=16, c_i=4, delay="uniform_int", d0=2, d1=9,
                                J=0.5, lam=1.2)
    spec = netspec.NetSpec(**{**spec.__dict__, "stdp": netspec.Stdp(pop=0, w0=0.5, wmax=2.0)})
    T = 2000
    a = oracle.OracleNet(spec, 8)
    _, _, w_before, _ = a.graph()
    a.run(T)
    st, ids = a.spikes()
    assert len(st) > 200
    _, _, w_closed, _ = a.graph()
    b = oracle.OracleNet(spec, 8)
    b.run_frozen(st, ids, T, record_x=False, record_v=False)
    _, _, w_replay, _ = b.graph()
    assert np.array_equal(w_closed, w_replay)
    src, tgt, _, _ = a.graph()
    plastic = (src < 160) & (tgt < 160)
    assert np.count_nonzero(w_closed[plastic] != w_before[plastic]) > 0.5 * plastic.sum()
    assert np.array_equal(w_closed[~plastic], w_before[~plastic])
    # a reset keeps the weights and restarts the traces
    a.reset()
    _, _, w_after_reset, _ = a.graph()
    assert np.array_equal(w_after_reset, w_closed)
