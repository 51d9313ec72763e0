"""The bench's roofline arithmetic on the host, with a stand-in network whose
queries return fixed sizes: algorithmic bytes per launch of the delivery
launch (records) and of the staging copy (records read and written plus one
descriptor per delivered spike and tile), the delivery launch's per-window
state bytes, the dominant kernel, and the traffic figure's tie to the source
it was measured on."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
import bench  # noqa: E402


class FakeNet:
    def __init__(self, **q):
        self.q = q

    def query(self, what):
        return self.q[what]


def _streamed(**over):
    q = dict(PLAN=2, STEPS_PER_SYNC=5, EDGE_BYTES=4, TILES=100, STAGE_RECORDS=4096, RING_SLOTS=30,
             TILE_SIZE=1024, RING_BYTES=4, NEURONS=100 * 1024)
    q.update(over)
    return FakeNet(**q)


def test_streamed_roofline_bytes_and_dominant_kernel():
    sim_steps, steps = 1000, 2
    launches = sim_steps // 5
    run = {"events": 4.0e9 * steps, "spikes": 2.0e5 * steps, "gpu_ms_per_step": 80.0}
    r = bench.roofline(_streamed(), run, steps, sim_steps, ktimes=(0.30, 0.20, launches - 1))
    ev = 4.0e9 / launches
    sp = 2.0e5 / launches
    d, c = r["kernels"]["stream_kernel"], r["kernels"]["gather_copy_kernel"]
    assert d["algorithmic_bytes_per_launch"] == pytest.approx(ev * 4)
    assert c["algorithmic_bytes_per_launch"] == pytest.approx(ev * 8 + sp * 100 * 8)
    assert d["achieved_GBps"] == pytest.approx(ev * 4 / 0.20e-3 / 1e9)
    # ring rows that can hold sums, in and out, and 16 B of neuron state, in and out
    state = 100 * (30 - 5) * 1024 * 4 * 2 + 100 * 1024 * 16 * 2
    assert d["state_bytes_per_launch"] == state
    assert d["frac_with_state"] == pytest.approx((ev * 4 + state) / 0.20e-3 / 1e9 / bench.HBM_PEAK_GBS)
    # the copy takes longer here: it is the dominant kernel
    assert r["kernel"] == "gather_copy_kernel"
    assert r["frac"] == pytest.approx(c["frac"])
    assert r["window_ms"] == pytest.approx(80.0 / launches)


def test_state_bytes_count_the_synaptic_currents_of_exp_and_alpha():
    run = {"events": 1.0e9, "spikes": 1.0e5, "gpu_ms_per_step": 10.0}
    per = {}
    for model in ("delta", "exp", "alpha"):
        r = bench.roofline(_streamed(), run, 1, 1000, ktimes=(0.1, 0.1, 199), model=model)
        per[model] = r["kernels"]["stream_kernel"]["state_bytes_per_launch"]
    n = 100 * 1024
    assert per["exp"] - per["delta"] == n * 4 * 2
    assert per["alpha"] - per["exp"] == n * 4 * 2


def test_resident_roofline_is_the_step_kernel():
    net = FakeNet(PLAN=1, STEPS_PER_SYNC=5, EDGE_BYTES=6, TILES=256)
    run = {"events": 9.0e9, "spikes": 8.0e5, "gpu_ms_per_step": 46.0}
    r = bench.roofline(net, run, 1, 10000)
    assert r["kernel"] == "step_kernel" and "kernels" not in r
    assert r["achieved"] == pytest.approx(9.0e9 * 6 / 46.0e-3 / 1e9)


def test_traffic_is_reported_only_for_the_sources_it_was_measured_on(monkeypatch):
    for k in ("step_kernel", "stream_kernel", "gather_copy_kernel"):
        per_event, h = bench.TRAFFIC[k]
        assert per_event > 0
        monkeypatch.setattr(bench, "source_hash", lambda kernel, h=h: h)
        assert bench.traffic_per_event(k) == per_event
        monkeypatch.setattr(bench, "source_hash", lambda kernel: "0" * 16)
        assert bench.traffic_per_event(k) is None
