"""Parity of the HIP library (through its C ABI) with the CPU oracle.

Integers (graph structure, Poisson counts, FP64 rasters) must match bit for
bit; FP32 inputs within 1e-5 of the summed absolute weights of the events
they add up; FP32 closed-loop rasters statistically (population rate within
2 %, ISI CV within 5 %).
"""
import math

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


def test_graph_matches_oracle_fixed_indegree(cx, orc):
    spec = netspec.small_brunel(n_e=800, n_i=200, c_e=80, c_i=20, delay="uniform_int", d0=5, d1=30,
                                w_rel_sd=0.1)
    case("graph fixed-indegree N=1000 T=128 seed 7")
    g = cx.Network(spec, 7, tile_size=128)
    o = orc.OracleNet(spec, 7)
    assert g.E == o.E == 1000 * 100
    assert g.query("TILES") == 8 and g.query("MIN_DELAY") == 5 and g.query("MAX_DELAY") == 30
    gt, gs, gd, gw = helpers.sorted_edges(*g.graph())
    ot, os_, od, ow = helpers.sorted_edges(*o.graph())
    assert np.array_equal(gt, ot) and np.array_equal(gs, os_) and np.array_equal(gd, od)
    w32 = ow.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(gw - w32) <= np.spacing(np.abs(w32).astype(np.float32)).astype(np.float64))


def test_graph_matches_oracle_pairwise_normal_delays(cx, orc):
    inst = netspec.microcircuit_instance(total=1500, target_synapses=1500 * 150.0)
    spec = netspec.NetSpec(model="exp", instances=[inst], poisson_lambda=0.5, w_ext=80.0)
    case("graph pairwise N=1500 auto tiles seed 3")
    g = cx.Network(spec, 3)
    o = orc.OracleNet(spec, 3)
    assert g.E == o.E
    assert g.query("MIN_DELAY") == o.d_min and g.query("MAX_DELAY") == o.d_max
    gt, gs, gd, gw = helpers.sorted_edges(*g.graph())
    ot, os_, od, ow = helpers.sorted_edges(*o.graph())
    assert np.array_equal(gt, ot) and np.array_equal(gs, os_) and np.array_equal(gd, od)
    w32 = ow.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(gw - w32) <= np.spacing(np.abs(w32).astype(np.float32)).astype(np.float64))


def test_tiles_partition_the_targets_and_own_their_in_edges(cx):
    # Eq. 8-10: disjoint tiles covering V; Eq. 5/14: a tile's sub-graph holds
    # exactly the in-edges of its targets
    spec = netspec.small_brunel(n_e=700, n_i=170, c_e=30, c_i=8)
    case("tiles N=870 T=100")
    g = cx.Network(spec, 2, tile_size=100)
    start, size, inst = g.tiles()
    assert start[0] == 0 and np.all(start[1:] == start[:-1] + size[:-1])
    assert start[-1] + size[-1] == g.N and size[-1] == 70
    src, tgt, w, d = g.graph()
    tile_of = np.searchsorted(start, tgt, side="right") - 1
    counts = np.bincount(tile_of, minlength=len(start))
    assert counts.sum() == g.E
    for t in range(len(start)):
        assert counts[t] == 38 * size[t]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_initial_state_matches_oracle(cx, orc, precision):
    spec = netspec.small_brunel(n_e=300, n_i=75, precision=precision)
    g = cx.Network(spec, 11)
    o = orc.OracleNet(spec, 11)
    V, r, _, _ = g.state()
    Vo = o.state()[0]
    if precision == "fp64":
        assert np.array_equal(V, Vo)
    else:
        assert np.array_equal(V, Vo.astype(np.float32).astype(np.float64))
    assert np.all(r == 0)


def _counting_spec(lam, n, precision):
    inst = netspec.Instance([netspec.Population("A", n)], [])
    return netspec.NetSpec(model="delta", tau_m=1e300, poisson_lambda=lam, w_ext=1.0, V_th=1e12,
                           V_reset=0.0, v0_lo=0.0, v0_hi=0.0, instances=[inst], precision=precision)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_poisson_counts_bit_exact(cx, orc, precision):
    n, T = 3000, 300
    spec = _counting_spec(2.0, n, precision)
    case(f"poisson counts {precision}")
    g = cx.Network(spec, 5, tile_size=256 if precision == "fp32" else 0)
    o = orc.OracleNet(spec, 5)
    _, v = g.run_frozen(np.zeros(0), np.zeros(0), T)
    _, vo = o.run_frozen(np.zeros(0, np.int64), np.zeros(0, np.int64), T, record_x=False)
    v = v.cpu().numpy().astype(np.float64)
    assert np.array_equal(np.diff(v, axis=0), np.diff(vo, axis=0))
    assert np.array_equal(v[0], vo[0])


def test_fp64_closed_loop_raster_bit_exact_brunel_1250(cx, orc):
    spec = netspec.brunel_1250_fp64()
    case("brunel 1,250 FP64 closed loop 1000 steps")
    g = cx.Network(spec, 1, record_steps=1000)
    g.step(1000)
    st, ids = g.spikes(0, 1000)
    o = orc.OracleNet(spec, 1)
    o.run(1000)
    ost, oids = o.spikes()
    assert len(ost) > 1000
    assert np.array_equal(st.astype(np.int64), ost) and np.array_equal(ids.astype(np.int64), oids)
    V, r, _, _ = g.state()
    Vo, ro, _, _ = o.state()
    assert np.array_equal(V, Vo) and np.array_equal(r, ro)
    # the pull counts events on arrival (step + 15 < 1000), the oracle on emission
    src, _, _, _ = o.graph()
    outdeg = np.bincount(src, minlength=spec.n_neurons)
    assert g.query("EVENTS") == outdeg[oids[ost + 15 < 1000]].sum()


@pytest.mark.parametrize("model", ["delta", "exp", "alpha"])
def test_fp64_frozen_traces_bit_exact(cx, orc, model):
    spec = netspec.small_brunel(model=model, n_e=400, n_i=100, c_e=40, c_i=10, delay="uniform_int",
                                d0=2, d1=9, w_rel_sd=0.0, precision="fp64",
                                J=0.1 if model == "delta" else 20.0)
    T = 150
    steps, ids = netspec.synthetic_raster(500, T, 0.02, seed=4)
    case(f"fp64 frozen {model}")
    g = cx.Network(spec, 9)
    o = orc.OracleNet(spec, 9)
    x, v = g.run_frozen(steps, ids, T)
    xo, vo = o.run_frozen(steps, ids, T)
    assert np.array_equal(x.cpu().numpy(), xo)
    assert np.array_equal(v.cpu().numpy(), vo)
    # the same run split over several calls reproduces every bit
    g.reset()
    parts = [g.run_frozen(steps, ids, k) for k in (40, 1, 59, 50)]
    assert np.array_equal(np.concatenate([p[0].cpu().numpy() for p in parts]), xo)


def _fp32_open_loop(cx, orc, spec, T, p, seed, tile_size, sel=None):
    N = spec.n_neurons
    steps, ids = netspec.synthetic_raster(N, T, p, seed=seed)
    g = cx.Network(spec, seed, tile_size=tile_size)
    x, v = g.run_frozen(steps, ids, T)
    o = orc.OracleNet(spec, seed, sel=sel)
    xo, vo = o.run_frozen(steps, ids, T)
    src, tgt, w, d = o.graph()
    cols = np.arange(N) if sel is None else np.asarray(sel)
    B = helpers.abs_input_bound(src, tgt, w, d, steps, ids, N, T)[:, cols]
    xg = x.cpu().numpy().astype(np.float64)[:, cols]
    vg = v.cpu().numpy().astype(np.float64)[:, cols]
    return g, xg, vg, xo, vo, B, steps, ids


# tile 256: segments of ~26 synapses (lanes over the flattened synapses);
# tiles 1024 and 2048 (two neurons per thread): ~102 and ~205 (waves over
# whole segments)
@pytest.mark.parametrize("model,d0,d1,tile", [("delta", 5, 30, 256), ("exp", 1, 12, 256), ("alpha", 5, 30, 256),
                                              ("alpha", 1, 1, 256), ("alpha", 5, 5, 1024), ("exp", 1, 12, 2048)])
def test_fp32_open_loop_delivery_matches_oracle(cx, orc, model, d0, d1, tile):
    spec = netspec.small_brunel(model=model, n_e=2400, n_i=600, c_e=240, c_i=60, delay="uniform_int",
                                d0=d0, d1=d1, w_rel_sd=0.1, weight_unit="psp_mV")
    case(f"fp32 open loop {model} delays {d0}..{d1} tile {tile}")
    g, xg, vg, xo, vo, B, _, _ = _fp32_open_loop(cx, orc, spec, 200, 0.01, 13, tile)
    assert g.query("TILES") == -(-3000 // tile)
    assert np.all(np.abs(xg - xo) <= 1e-5 * B + 1e-30)
    assert np.abs(xo).max() > 0
    assert np.all(np.abs(vg - vo) <= 1e-4 * (1.0 + np.abs(vo)))


def test_fp32_open_loop_with_32bit_rings(cx, orc):
    # delays of 1..200 steps: 64-bit rings of 201 slots cannot fit the
    # workgroup-local memory of the chip, so the planner scales 32-bit sums
    # by the largest exact input bound of any neuron
    spec = netspec.small_brunel(model="exp", n_e=24000, n_i=6000, c_e=80, c_i=20, delay="uniform_int",
                                d0=1, d1=200, w_rel_sd=0.1, J=20.0)
    case("fp32 open loop, 32-bit rings, delays 1..200")
    g, xg, vg, xo, vo, B, _, _ = _fp32_open_loop(cx, orc, spec, 260, 0.01, 23, 0)
    assert g.query("RING_BYTES") == 4 and g.query("RING_SLOTS") == 200
    assert np.all(np.abs(xg - xo) <= 1e-5 * B + 1e-30)
    assert np.abs(xo).max() > 0
    assert np.all(np.abs(vg - vo) <= 1e-4 * (1.0 + np.abs(vo)))


# tile 192: segments of ~19 synapses (lanes over the flattened synapses);
# tile 1024: ~102 (waves over whole segments)
@pytest.mark.parametrize("steps_per_sync,tile", [(0, 192), (1, 192), (2, 192), (0, 1024), (3, 1024)])
def test_fp32_integer_weights_give_exact_sums_across_calls(cx, orc, steps_per_sync, tile):
    spec = netspec.small_brunel(n_e=1600, n_i=400, c_e=160, c_i=40, delay="uniform_int", d0=3, d1=17,
                                w_rel_sd=0.0, J=1.0, g=2.0)
    T = 160
    steps, ids = netspec.synthetic_raster(2000, T, 0.02, seed=21)
    case(f"fp32 integer weights, split calls, steps_per_sync={steps_per_sync}, tile {tile}")
    g = cx.Network(spec, 17, tile_size=tile, steps_per_sync=steps_per_sync)
    o = orc.OracleNet(spec, 17)
    xo, _ = o.run_frozen(steps, ids, T)
    parts = [g.run_frozen(steps, ids, k)[0].cpu().numpy() for k in (1, 63, 16, 80)]
    assert np.array_equal(np.concatenate(parts).astype(np.float64), xo)
    # a call ending at step T has delivered the spikes of steps < T - d_min;
    # later ones are delivered by the next call
    src, _, _, _ = o.graph()
    outdeg = np.bincount(src, minlength=2000)
    m = steps < T - g.query("MIN_DELAY")
    assert g.query("EVENTS") == outdeg[ids[m]].sum()


def test_fp32_closed_loop_statistics_scaled_brunel_112k(cx, orc):
    spec = netspec.brunel_112k_alpha(scale_n=0.1, scale_k=0.1)
    T = 10000
    case("fp32 closed loop brunel 112k x0.1, 1 s")
    g = cx.Network(spec, 2, record_steps=T)
    g.step(T)
    st, ids = g.spikes(0, T)
    o = orc.OracleNet(spec, 2)
    o.run(T)
    ost, oids = o.spikes()
    rg = helpers.rates_and_cv(st, ids, spec, 1000, T)
    ro = helpers.rates_and_cv(ost, oids, spec, 1000, T)
    print("gpu", rg, "oracle", ro, flush=True)
    for (rate_g, cv_g), (rate_o, cv_o) in zip(rg, ro):
        assert rate_o > 0.5
        assert abs(rate_g - rate_o) <= 0.02 * rate_o
        assert abs(cv_g - cv_o) <= 0.05 * cv_o
    # every delivered event is a (spike, out-synapse) pair
    src, _, _, _ = o.graph()
    outdeg = np.bincount(src, minlength=spec.n_neurons)
    m = st < T - g.query("MIN_DELAY")
    assert g.query("EVENTS") == outdeg[ids[m]].sum()


def test_fp32_results_do_not_depend_on_the_plan(cx):
    # fixed-point input sums make the FP32 path independent of tile size,
    # spike-exchange window and workgroup size, bit for bit
    spec = netspec.brunel_112k_alpha(scale_n=0.05, scale_k=0.05)
    T = 1500
    outs = []
    for plan in (dict(), dict(tile_size=300, steps_per_sync=2), dict(tile_size=128, block_size=256,
                                                                   steps_per_sync=1)):
        case(f"plan {plan}")
        g = cx.Network(spec, 4, record_steps=T, **plan)
        g.step(700)
        g.step(T - 700)
        st, ids = g.spikes(0, T)
        V, r, y1, y2 = g.state()
        outs.append((st, ids, V, r, y1, y2, g.query("EVENTS")))
        g.close()
    assert len(outs[0][0]) > 1000
    for o in outs[1:]:
        for a, b in zip(outs[0][:6], o[:6]):
            assert np.array_equal(a, b)


def test_full_size_brunel_112k_sampled_open_loop(cx, orc):
    spec = netspec.brunel_112k_alpha()
    N = spec.n_neurons
    sel = np.unique(np.concatenate([[0, 439, 440, N - 1],
                                    netspec.sample_targets(N, 28, seed=5)]))
    T = 60
    case("brunel 112k full size sampled open loop")
    g, xg, vg, xo, vo, B, _, _ = _fp32_open_loop(cx, orc, spec, T, 0.002, 2, 0, sel=sel)
    assert g.E == 112500 * 11250
    assert np.all(np.abs(xg - xo) <= 1e-5 * B + 1e-30)
    assert np.all(np.abs(vg - vo) <= 1e-4 * (1.0 + np.abs(vo)))


def test_error_paths(cx):
    import ctypes as C
    spec = netspec.small_brunel()
    g = cx.Network(spec, 1, record_steps=10)
    with pytest.raises(cx.CortexError) as e:
        g.step(-1)
    assert e.value.status == cx.EINVAL
    with pytest.raises(cx.CortexError) as e:
        g.run_frozen(np.array([3, 1]), np.array([0, 0]), 5)
    assert e.value.status == cx.EINVAL
    with pytest.raises(cx.CortexError) as e:
        g.backward(None)
    assert e.value.status in (cx.ESTATE, cx.EUNSUPPORTED)
    g.step(20)
    cnt = C.c_int64()
    rc = cx.lib().cortex_get_spikes(g._h, 0, 20, None, None, 0, C.byref(cnt))
    assert rc == cx.ETRUNC


BATCH_SIZES = [200, 450, 1000, 2200, 5000]


def test_batched_instances_graph_and_tiles(cx, orc):
    spec = netspec.batched_brunel(BATCH_SIZES)
    case("batched graph, 5 instances")
    g = cx.Network(spec, 4)
    o = orc.OracleNet(spec, 4)
    assert g.E == o.E
    start, size, inst = g.tiles()
    # tiles never straddle instances; instances with more synapses per target
    # get smaller tiles
    bounds = np.cumsum([0] + BATCH_SIZES)
    for b in range(len(BATCH_SIZES)):
        m = inst == b
        assert start[m][0] == bounds[b] and start[m][-1] + size[m][-1] == bounds[b + 1]
    tmax = [size[inst == b].max() for b in range(len(BATCH_SIZES))]
    assert tmax[-1] <= tmax[0]
    gt, gs, gd, gw = helpers.sorted_edges(*g.graph())
    ot, os_, od, ow = helpers.sorted_edges(*o.graph())
    assert np.array_equal(gt, ot) and np.array_equal(gs, os_) and np.array_equal(gd, od)
    assert np.array_equal(gw, ow.astype(np.float32).astype(np.float64))


def test_batched_open_loop_matches_oracle(cx, orc):
    spec = netspec.batched_brunel(BATCH_SIZES)
    case("batched open loop")
    g, xg, vg, xo, vo, B, _, _ = _fp32_open_loop(cx, orc, spec, 120, 0.01, 4, 0)
    assert np.all(np.abs(xg - xo) <= 1e-5 * B + 1e-30)
    assert np.all(np.abs(vg - vo) <= 1e-4 * (1.0 + np.abs(vo)))


def _adjoint_case(cx, orc, spec, T, ckpt, seed, p_spike=0.02):
    import torch
    N = spec.n_neurons
    steps, ids = netspec.refractory_raster(N, T, p_spike, seed=seed, n_ref=20)
    vstar = netspec.target_trace(N, T, 10.0, 20.0, seed=seed + 1)
    g = cx.Network(spec, seed, ckpt_every=ckpt, adjoint_steps=T)
    g.run_frozen(steps, ids, T, traces=False)
    vs = torch.tensor(vstar, dtype=torch.float32, device="cuda")
    grad, loss = g.backward(vs)
    o = orc.OracleNet(spec, seed)
    gro, loss_o = o.backward(steps, ids, T, vstar.astype(np.float32).astype(np.float64))
    return g, o, grad.cpu().numpy().astype(np.float64), loss, gro, loss_o


@pytest.mark.parametrize("model", ["delta", "exp", "alpha"])
def test_adjoint_matches_oracle_on_frozen_raster(cx, orc, model):
    spec = netspec.small_brunel(model=model, n_e=400, n_i=100, c_e=40, c_i=10, delay="uniform_int",
                                d0=2, d1=9, w_rel_sd=0.1, J=0.1 if model == "delta" else 20.0)
    case(f"adjoint {model}")
    g, o, gr, loss, gro, loss_o = _adjoint_case(cx, orc, spec, 260, 50, 31)
    assert loss == pytest.approx(loss_o, rel=1e-5)
    scale = np.abs(gro).max()
    assert scale > 0
    # The forward runs in FP32: its membrane potentials carry relative
    # errors near 1e-7, which reach every gradient through V - V*, so the
    # absolute error is a fraction of the largest gradient rather than of
    # each one (measured: at most 5.4e-6 of it over the three models); 2e-5
    # checks the small gradients too, down to that level.
    assert np.allclose(gr, gro, rtol=1e-3, atol=2e-5 * scale)
    # synapses whose source never spikes early enough have no gradient at all
    zero = gro == 0.0
    assert zero.any() and np.all(gr[zero] == 0.0)
    # canonical order of the export matches the oracle's edge order
    canon = g.canonical()
    src, tgt, w, d = g.graph()
    os_, ot, ow, od = o.graph()
    assert np.array_equal(os_[canon], src) and np.array_equal(ot[canon], tgt) and np.array_equal(od[canon], d)


def test_set_weights_gradient_matches_oracle_and_finite_differences(cx, orc):
    import torch
    spec = netspec.small_brunel(model="exp", n_e=400, n_i=100, c_e=40, c_i=10, delay="uniform_int",
                                d0=2, d1=9, w_rel_sd=0.1, J=20.0)
    T, seed = 200, 37
    N = spec.n_neurons
    steps, ids = netspec.refractory_raster(N, T, 0.02, seed=seed, n_ref=20)
    vstar = netspec.target_trace(N, T, 10.0, 20.0, seed=seed + 1)
    case("set weights: gradient vs oracle and finite differences")
    g = cx.Network(spec, seed, ckpt_every=50, adjoint_steps=T)
    w0 = g.canonical_weights()
    rng = np.random.default_rng(seed + 2)
    w1 = (w0 * (1.0 + 0.3 * rng.standard_normal(w0.size))).astype(np.float32)
    vs = torch.tensor(vstar, dtype=torch.float32, device="cuda")
    w = torch.tensor(w1, device="cuda", requires_grad=True)
    raster = (steps, ids)
    loss = cx.VoltageLoss.apply(w, g, vs, T, raster)
    loss.backward()
    gr = w.grad.detach().cpu().numpy().astype(np.float64)
    # the stored weights are the new ones
    assert np.array_equal(g.canonical_weights(), w1.astype(np.float64))
    # oracle with the same weights (canonical order is shared)
    o = orc.OracleNet(spec, seed)
    for e in range(o.E):
        o.set_weight(e, float(w1[e]))
    gro, loss_o = o.backward(steps, ids, T, vstar.astype(np.float32).astype(np.float64))
    assert float(loss) == pytest.approx(loss_o, rel=1e-5)
    assert np.allclose(gr, gro, rtol=1e-3, atol=1e-4 * np.abs(gro).max())
    # central differences of the GPU loss (quadratic in w with frozen spikes)
    for e in np.argsort(-np.abs(gr))[:4]:
        h = 0.2 * abs(float(w1[e]))
        lp = float(cx.VoltageLoss.apply(torch.tensor(np.where(np.arange(w1.size) == e, w1 + h, w1)
                                                     .astype(np.float32), device="cuda"), g, vs, T, raster))
        lm = float(cx.VoltageLoss.apply(torch.tensor(np.where(np.arange(w1.size) == e, w1 - h, w1)
                                                     .astype(np.float32), device="cuda"), g, vs, T, raster))
        h_eff = float(np.float32(w1[e] + h)) - float(np.float32(w1[e] - h))
        assert (lp - lm) / h_eff == pytest.approx(gr[e], rel=2e-2)


def test_autotune_returns_the_fastest_valid_plan(cx, tmp_path):
    import json
    spec = netspec.batched_brunel([600, 1200, 2400])
    case("autotune on 3 batched instances")
    cache = str(tmp_path / "plans.json")
    best, timings = cx.autotune(spec, 9, steps=300, warmup=50, cache=cache)
    timed = [(r, p, t) for r, p, t in timings if t is not None]
    assert len(timed) >= 2 and all(t > 0 for _, _, t in timed)
    assert best == min(timed, key=lambda rpt: rpt[2])[0]
    # both plan kinds and both occupancies were measured
    assert {r["plan"] for r, _, _ in timed} == {"resident", "streamed"}
    assert {r["wg_per_cu"] for r, _, _ in timed} == {1, 2}
    # the cache holds the winner under this network and device
    got, entry = cx.lookup_plan(spec, paths=[cache])
    assert got == best and entry["library"] == cx._library_hash()
    assert len(json.load(open(cache))["entries"]) == 1
    g = cx.Network(spec, 9, **got)
    assert g.query("STEPS_PER_SYNC") == best["steps_per_sync"]
    g.step(100)
    assert g.query("SPIKES") > 0


def test_adjoint_batched_instances(cx, orc):
    spec = netspec.batched_brunel([300, 700, 1500])
    case("adjoint batched")
    g, o, gr, loss, gro, loss_o = _adjoint_case(cx, orc, spec, 230, 100, 41)
    assert loss == pytest.approx(loss_o, rel=1e-5)
    assert np.allclose(gr, gro, rtol=1e-3, atol=1e-4 * np.abs(gro).max())


def test_adjoint_closed_loop_is_repeatable_and_restores_state(cx):
    import torch
    spec = netspec.batched_brunel([1000, 2000])
    T = 300
    case("adjoint closed loop")
    g = cx.Network(spec, 6, ckpt_every=100, adjoint_steps=T)
    g.step(T)
    before = g.state()
    vs = torch.tensor(netspec.target_trace(spec.n_neurons, T, 10.0, 20.0, seed=3), dtype=torch.float32,
                      device="cuda")
    g1, l1 = g.backward(vs)
    g1 = g1.cpu().numpy().copy()
    after = g.state()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    g2, l2 = g.backward(vs)
    assert l1 == l2 and np.array_equal(g1, g2.cpu().numpy())
    assert np.count_nonzero(g1) > 0
