"""Pins of the oracle's conductance-based synapses (the conductance form of
Eq. 3 with exponential conductances, rule in oracle/oracle.h): the membrane
trace against an independent numerical solution of the ODE with the
conductances held over each step, for an excitatory and an inhibitory
synapse and a refractory stretch; the conductance decay and the channel of
external events."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import netspec
import oracle

DT, TM, C, EL, TS = 0.1, 20.0, 250.0, -70.0, 2.0
EEX, EIN = 0.0, -85.0


def _pair(w, t_ref=2.0, V_th=1e9):
    pops = [netspec.Population("A", 2)]
    projs = [netspec.Projection(0, 0, "fixed_indegree", w, k=1, delay="const", d0=1.0)]
    return netspec.NetSpec(model="cond", tau_m=TM, C_m=C, E_L=EL, V_th=V_th, V_reset=-75.0, t_ref=t_ref,
                           tau_syn=TS, poisson_lambda=0.0, w_ext=0.0, v0_lo=-65.0, v0_hi=-65.0,
                           instances=[netspec.Instance(pops, projs)], E_ex=EEX, E_in=EIN)


def _ode_trace(g_ex, g_in, v0, refr):
    """V after each step, the conductances held at g_ex[n], g_in[n] over step
    n (refractory steps clamp V to the reset), by an ODE solver."""
    v, out = v0, []
    gL = C / TM
    for n in range(len(g_ex)):
        if refr[n]:
            v = -75.0
        else:
            f = lambda t, y: [(-gL * (y[0] - EL) + g_ex[n] * (EEX - y[0]) + g_in[n] * (EIN - y[0])) / C]
            v = solve_ivp(f, (0.0, DT), [v], rtol=1e-12, atol=1e-12, method="DOP853").y[0, -1]
        out.append(v)
    return np.array(out)


@pytest.mark.parametrize("w", [12.0, -20.0])
def test_membrane_follows_the_ode_with_conductances_held_over_each_step(w):
    spec = _pair(w)
    T = 200
    st = np.array([5], np.int64)
    ids = np.array([0], np.int64)     # neuron 0 drives neuron 1 (d = 10 steps)
    o = oracle.OracleNet(spec, 1)
    x, v = o.run_frozen(st, ids, T)
    a = 5 + 10                         # arrival step: consumed by the update of step a
    P11 = math.exp(-DT / TS)
    g = np.zeros(T)                    # conductance during step n (held from its start)
    for n in range(a + 1, T):
        g[n] = abs(w) * P11 ** (n - a - 1)
    g_ex, g_in = (g, np.zeros(T)) if w > 0 else (np.zeros(T), g)
    ref = _ode_trace(g_ex, g_in, -65.0, np.zeros(T, bool))
    assert np.allclose(v[:, 1], ref, rtol=0, atol=1e-9)
    assert x[a, 1] == w and np.count_nonzero(x[:, 1]) == 1
    # the channel: depolarising towards E_ex, hyperpolarising towards E_in
    assert (v[a + 20, 1] > -65.0) == (w > 0)
    # the conductance state decays with tau_syn
    _, _, gex_end, gin_end = o.state()
    assert (gex_end[1] if w > 0 else gin_end[1]) == pytest.approx(abs(w) * P11 ** (T - a - 1), rel=1e-12)


def test_refractory_steps_clamp_v_while_conductances_integrate():
    spec = _pair(12.0, t_ref=3.0)
    T = 120
    st = np.array([5, 18], np.int64)
    ids = np.array([0, 1], np.int64)   # the input arrives at 15; neuron 1 spikes at 18
    o = oracle.OracleNet(spec, 1)
    _, v = o.run_frozen(st, ids, T)
    P11 = math.exp(-DT / TS)
    g = np.zeros(T)
    for n in range(16, T):
        g[n] = 12.0 * P11 ** (n - 16)
    refr = np.zeros(T, bool)
    refr[19:49] = True                 # 30 steps after the spike at 18
    ref = _ode_trace(g, np.zeros(T), -65.0, refr)
    ref[18] = -75.0                    # the spike step itself ends at the reset
    assert np.allclose(v[:, 1], ref, rtol=0, atol=1e-9)


def test_external_events_enter_the_channel_of_their_sign():
    pops = [netspec.Population("A", 3)]
    for w_ext in (2.0, -2.0):
        spec = netspec.NetSpec(model="cond", tau_m=TM, C_m=C, E_L=EL, V_th=1e9, tau_syn=TS, poisson_lambda=1.0,
                               w_ext=w_ext, v0_lo=-70.0, v0_hi=-70.0,
                               instances=[netspec.Instance(pops, [])], E_ex=EEX, E_in=EIN)
        o = oracle.OracleNet(spec, 4)
        o.run(50)
        _, _, gex, gin = o.state()
        assert np.all(gex > 0) == (w_ext > 0) and np.all(gin > 0) == (w_ext < 0)
        # stationary mean lambda |w_ext| / (1 - e^{-dt/tau_syn}) = 41 nS, sd about 6
        g = gex if w_ext > 0 else gin
        assert np.all((g > 15.0) & (g < 80.0))


def cond_net():
    """1,000 conductance-LIF neurons (800 E / 200 I, in-degree 80 + 20,
    1 nS / -5 nS, delays 1-2 ms) driven just below threshold by Poisson
    events of 0.5 nS."""
    inst = netspec.brunel_instance(800, 200, 80, 20, 1.0, 5.0, w_rel_sd=0.1, delay="uniform_int", d0=10, d1=20)
    return netspec.NetSpec(model="cond", tau_m=TM, C_m=C, E_L=EL, V_th=-50.0, V_reset=-60.0, tau_syn=TS,
                           poisson_lambda=0.45, w_ext=0.5, v0_lo=-70.0, v0_hi=-50.0, instances=[inst],
                           E_ex=EEX, E_in=EIN)


def test_closed_loop_conductance_network_fires_with_both_channels_open():
    o = oracle.OracleNet(cond_net(), 2)
    o.run(5000)
    st, ids = o.spikes()
    rate = len(st) / (1000 * 0.5)
    assert 1.0 < rate < 100.0
    _, _, gex, gin = o.state()
    assert gex.mean() > 1.0 and gin.mean() > 1.0
