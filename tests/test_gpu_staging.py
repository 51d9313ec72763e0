"""Tile-major staging of a window's records (streamed plan, short segments)
against delivery straight from the graph.  The input rings add 32-bit
fixed-point integers, so the order of the additions does not change the sums:
a closed-loop run must give the same raster, state and event count bit for
bit whether every window's records are staged, delivered from the graph, or
split between the two (a staging capacity below a window's load)."""
import numpy as np
import pytest

import netspec

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


@pytest.mark.parametrize("wdt", ["bf16", "fp32"])
def test_staged_direct_and_mixed_delivery_give_identical_runs(cx, wdt):
    # 100,000 neurons with the in-degree of the two-million-neuron network,
    # tiles of 128: segments of about 14 synapses
    spec = netspec.brunel_2m_bf16(scale_n=0.05)
    spec.weight_dtype = wdt
    chunks = [32 * 5, 3, 32 * 5 + 17, 32 * 5]
    T = sum(chunks)
    runs = []
    for stage in (0, -1, 3000, 64):
        case(f"{wdt} weights, stage_records={stage}, {T} steps")
        g = cx.Network(spec, 5, record_steps=T, plan="streamed", tile_size=128, steps_per_sync=5,
                       stage_records=stage)
        assert g.query("PLAN") == cx.PLAN_STREAMED
        staged = g.query("STAGE_RECORDS")
        assert (staged > 0) == (stage >= 0) and (stage <= 0 or staged == stage)
        for c in chunks:
            g.step(c)
        st, ids = g.spikes(0, T)
        V, r, _, _ = g.state()
        runs.append((st, ids, np.asarray(V), np.asarray(r), g.query("EVENTS")))
        g.close()
    st, ids = runs[0][0], runs[0][1]
    rate = len(st) / (spec.n_neurons * T * spec.dt * 1e-3)
    print("spikes", len(st), "rate", rate, flush=True)
    assert 1.0 < rate < 50.0
    for other in runs[1:]:
        for a, b in zip(runs[0][:4], other[:4]):
            assert np.array_equal(a, b)
        assert runs[0][4] == other[4]


def test_kernel_timing_reports_both_launches_and_changes_nothing(cx):
    spec = netspec.brunel_2m_bf16(scale_n=0.05)
    T = 32 * 5 * 2
    runs = []
    for timing in (False, True):
        case(f"kernel timing {'on' if timing else 'off'}")
        g = cx.Network(spec, 5, record_steps=T, plan="streamed", tile_size=128, steps_per_sync=5)
        if timing:
            g.kernel_timing(True)
        g.step(T)
        st, ids = g.spikes(0, T)
        if timing:
            copy_ms, deliver_ms, nw = g.kernel_times()
            print("copy", copy_ms, "deliver", deliver_ms, flush=True)
            # every delivery launch but the last (whose interval the next
            # launch would close)
            assert nw == T // 5 - 1 and copy_ms > 0 and deliver_ms > 0
        runs.append((st, ids, g.query("EVENTS")))
        g.close()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    assert runs[0][2] == runs[1][2]


@pytest.mark.parametrize("wdt", ["bf16", "fp32"])
def test_items_past_the_copy_buffer_write_straight_to_the_runs(cx, orc, wdt):
    """A small inhibitory population that every target samples a thousand
    times has long rows (about 64 synapses per tile), so that a copy work
    item of 64 spikes, most of them inhibitory, holds several times the
    records of the copy's workgroup-local buffer and writes them straight to
    the tile runs.  Open loop: staged and direct delivery give the same
    inputs and potentials bit for bit, and sampled targets match the
    oracle."""
    from tests import helpers
    spec = netspec.small_brunel(n_e=100000, n_i=2000, c_e=1000, c_i=1000, delay="uniform_int", d0=5, d1=30)
    spec.weight_dtype = wdt
    N, T = spec.n_neurons, 40
    rng = np.random.default_rng(47)
    p = np.where(np.arange(N) < 100000, 0.002, 0.05)
    st, ids = np.nonzero(rng.random((T, N)) < p)
    steps, ids = st.astype(np.uint32), ids.astype(np.uint32)
    outs = []
    for stage in (40000, -1):
        case(f"{wdt} weights, long inhibitory rows, stage_records={stage}")
        g = cx.Network(spec, 7, plan="streamed", tile_size=128, steps_per_sync=5, stage_records=stage)
        assert g.query("STAGE_RECORDS") == max(stage, 0)
        # a window holds ~500 inhibitory spikes of 16 x 64 records per tile group:
        # far past the 7,424 (bf16) or 3,712 (fp32) records an item can hold
        assert g.query("STAGE_GROUP") == (16 if stage > 0 else 0)
        x, v = g.run_frozen(steps, ids, T)
        outs.append((x.cpu().numpy(), v.cpu().numpy()))
        g.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    sel = np.unique(np.concatenate([[0, 99999, 100000, N - 1], netspec.sample_targets(N, 20, seed=9)]))
    o = orc.OracleNet(spec, 7, sel=sel)
    src, tgt, w, d = o.graph()
    if wdt == "bf16":
        from tests.golden.make_closed_loop_stats import bf16_rne
        w = bf16_rne(w)
        o.set_weights(w)
    xo, vo = o.run_frozen(steps, ids, T)
    B = helpers.abs_input_bound(src, tgt, np.abs(w), d, steps, ids, N, T)[:, sel]
    xg, vg = outs[0][0][:, sel].astype(np.float64), outs[0][1][:, sel].astype(np.float64)
    assert np.abs(xo).max() > 0
    assert np.all(np.abs(xg - xo) <= 1e-5 * B + 1e-30)
    assert np.all(np.abs(vg - vo) <= 1e-4 * (1.0 + np.abs(vo)))
