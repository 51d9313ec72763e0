"""E->E spike-timing dependent plasticity on the GPU (streamed plan, one
plasticity pass per window before delivery) against the oracle's rule.

Open loop, the weights after a raster and the inputs they deliver match the
oracle's; closed loop, the weights the GPU ends with are those the oracle
computes from the GPU's own raster (the weights are a function of the
raster alone, at any size); a synapse that needs more postsynaptic spikes
than a neuron keeps makes the call fail with CORTEX_ETRUNC.
"""
import numpy as np
import pytest

import netspec
from tests import helpers

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def cx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_03762_amd as m
    m.lib()
    return m


def _plastic(spec, **kw):
    st = netspec.Stdp(pop=0, **kw)
    return netspec.NetSpec(**{**spec.__dict__, "stdp": st})


def _check_weights(wg, wo, wmax):
    bad = np.abs(wg - wo) > 1e-4 * np.abs(wo) + 1e-6 * wmax
    if bad.any():
        k = np.nonzero(bad)[0]
        print(f"{len(k)} weights differ; first: gpu {wg[k[:5]]} oracle {wo[k[:5]]}", flush=True)
    assert not bad.any()


@pytest.mark.parametrize("d0,d1,tile", [(2, 9, 128), (5, 30, 256), (15, 15, 200)])
def test_plastic_open_loop_weights_and_inputs_match_oracle(cx, orc, d0, d1, tile):
    base = netspec.small_brunel(n_e=800, n_i=200, c_e=80, c_i=20, delay="uniform_int", d0=d0, d1=d1,
                                w_rel_sd=0.1, J=0.2)
    spec = _plastic(base, lam=0.05, alpha=1.0, w0=0.2, wmax=0.6)
    # the GPU updates a synapse when the spike's delivery window starts, the
    # oracle when the spike is emitted: spikes only in steps both have
    # delivered by the end (more than d_min steps before it)
    T = 600
    steps, ids = netspec.refractory_raster(1000, T - 40, 0.01, 20, seed=17)
    case(f"plastic open loop delays {d0}..{d1} tile {tile}")
    g = cx.Network(spec, 19, tile_size=tile)
    assert g.query("PLAN") == cx.PLAN_STREAMED and g.query("STEPS_PER_SYNC") <= 21
    x, _ = g.run_frozen(steps, ids, T)
    xg = x.cpu().numpy().astype(np.float64)
    # rows (target, source, delay, weight); the synapses of one (source,
    # target, delay) take the same updates, which keep their order
    gt, gs, gd, gw = helpers.sorted_edges(*g.graph())
    o = orc.OracleNet(spec, 19)
    _, _, w0_, _ = o.graph()
    xo, _ = o.run_frozen(steps, ids, T)
    src, tgt, w, d = o.graph()
    ot, os_, od, ow = helpers.sorted_edges(src, tgt, w, d)
    assert np.array_equal(gs, os_) and np.array_equal(gt, ot) and np.array_equal(gd, od)
    plastic = (os_ < 800) & (ot < 800)
    _, _, _, ow0 = helpers.sorted_edges(src, tgt, w0_, d)
    changed = np.count_nonzero(ow[plastic] != ow0[plastic])
    print(f"plastic synapses {plastic.sum()}, changed {changed}", flush=True)
    assert changed > 0.5 * plastic.sum()
    _check_weights(gw, ow, 0.6)
    assert np.array_equal(gw[~plastic], ow0[~plastic].astype(np.float32).astype(np.float64))
    # inputs delivered with the updated weights: within 1e-4 of the largest
    # possible input (plastic weights counted at w_max)
    wb = np.where((src < 800) & (tgt < 800), np.maximum(np.abs(w0_), 0.6), np.abs(w0_))
    B = helpers.abs_input_bound(src, tgt, wb, d, steps, ids, 1000, T)
    assert np.abs(xo).max() > 0
    assert np.all(np.abs(xg - xo) <= 1e-4 * B + 1e-30)


def test_plastic_closed_loop_weights_follow_from_its_own_raster(cx, orc):
    base = netspec.small_brunel(n_e=4000, n_i=1000, c_e=400, c_i=100, delay="uniform_int", d0=5, d1=30,
                                w_rel_sd=0.1, J=0.1, lam=2.0)
    spec = _plastic(base, lam=0.05, alpha=1.0, w0=0.1, wmax=0.3)
    T = 3000
    case("plastic closed loop 5,000 neurons 300 ms")
    g = cx.Network(spec, 23, record_steps=T)
    assert g.query("STEPS_PER_SYNC") == 5 and g.query("MIN_DELAY") == 5
    g.step(T)
    st, ids = g.spikes(0, T)
    gt, gs, gd, gw = helpers.sorted_edges(*g.graph())
    g.close()
    rates = helpers.rates_and_cv(st, ids, spec, 500, T)
    print("rates/cv", rates, "spikes", len(st), flush=True)
    assert len(st) > 2000
    # the spikes the GPU delivered by step T (its windows end at T, a
    # multiple of W): those emitted before T - d_min
    W, dmin = 5, 5
    assert T % W == 0
    keep = st < T - dmin
    o = orc.OracleNet(spec, 23)
    o.run_frozen(st[keep].astype(np.int64), ids[keep].astype(np.int64), T, record_x=False, record_v=False)
    src, tgt, w, d = o.graph()
    ot, os_, od, ow = helpers.sorted_edges(src, tgt, w, d)
    assert np.array_equal(gs, os_) and np.array_equal(gt, ot) and np.array_equal(gd, od)
    plastic = (os_ < 4000) & (ot < 4000)
    assert np.count_nonzero(gw[plastic] != gw[plastic][0]) > 0
    _check_weights(gw, ow, 0.3)


def test_history_too_short_is_an_error_not_a_wrong_weight(cx):
    # neuron 0 -> 1 plastic: 0 spikes once, 1 spikes 40 times, then 0 again:
    # the second delivery needs all 40 post spikes, more than a neuron keeps
    pops = [netspec.Population("E", 2)]
    projs = [netspec.Projection(0, 0, "fixed_indegree", 0.1, k=1, delay="const", d0=0.5)]
    spec = netspec.NetSpec(model="delta", poisson_lambda=0.0, w_ext=0.0, V_th=1e9, V_reset=0.0, v0_lo=0.0,
                           v0_hi=0.0, instances=[netspec.Instance(pops, projs)],
                           stdp=netspec.Stdp(pop=0, w0=0.1, wmax=1.0))
    post = [(30 + 25 * k, 1) for k in range(40)]
    raster = sorted([(5, 0)] + post + [(30 + 25 * 40 + 10, 0)])
    st = np.array([s for s, _ in raster], np.uint32)
    ids = np.array([i for _, i in raster], np.uint32)
    case("plastic history overflow")
    g = cx.Network(spec, 1, plan="streamed")
    with pytest.raises(cx.CortexError) as e:
        g.run_frozen(st, ids, int(st.max()) + 20, traces=False)
    assert e.value.status == cx.ETRUNC
    # and a raster that breaks the refractory period is refused up front
    g2 = cx.Network(spec, 1, plan="streamed")
    with pytest.raises(cx.CortexError) as e:
        g2.run_frozen(np.array([5, 6], np.uint32), np.array([0, 0], np.uint32), 20, traces=False)
    assert e.value.status == cx.EINVAL
