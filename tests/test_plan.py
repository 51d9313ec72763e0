"""The launch planner, on the host alone (cortex_plan): for every workload and
every explicit plan request, either a plan whose every kernel index stays
inside its array (the library checks each plan before it returns it), or an
error status; never a plan outside the kernels' limits.  In particular no
resident plan puts four neurons per thread in workgroups other than 512
threads (the launch bound of that kernel variant), including the packing of
48 batched instances."""
import itertools

import numpy as np
import pytest

import netspec
import paper_2406_03762_amd as cx

MI355X = dict(n_cu=256, lds_per_cu=163840, threads_per_cu=2048)


def step_lds(R, T, W, ntb, chunk, rb):
    """The resident kernel's LDS, array by array in its carve-up order."""
    b = chunk * 16 + R * T * rb + (chunk + 1) * 4 + W * T * 4 + (W * ntb + 1) * 4 + W * ntb * 4
    b += (20 + 4 + 8 + 20) * 4 + T * 4 + 32 * 4 + 16 * T + 512 * 4
    return (b + 15) & ~15


def stream_lds(R, T, W, chunk):
    """The streamed kernel's LDS, array by array in its carve-up order."""
    b = chunk * 16 + R * T * 4 + (chunk + 1) * 4 + ((W * T * 2 + 3) & ~3) + T * 4 + 512 * 4 + 32 * 4
    b += 9 * 4 + 8 * 4 + (20 + 20 + 8) * 4
    return (b + 15) & ~15


def check(p, spec):
    assert p["lds_bytes"] <= MI355X["lds_per_cu"]
    assert p["npt"] in (1, 2, 4) and p["npt"] * p["block_size"] >= p["T"]
    assert 1 <= p["W"] <= min(8, p["dmin"]) and p["R"] == p["dmax"] - p["dmin"] + p["W"]
    assert p["H"] & (p["H"] - 1) == 0
    if p["plan"] == cx.PLAN_RESIDENT:
        assert p["npt"] != 4 or p["block_size"] == 512
        assert p["H"] >= 2 * p["dmin"] + 2 * p["W"] + 2
        assert p["lds_bytes"] == step_lds(p["R"], p["T"], p["W"], p["ntb_max"], p["chunk"], p["ring_bytes"])
        assert p["tiles"] <= MI355X["n_cu"] * (MI355X["threads_per_cu"] // p["block_size"])
    else:
        assert p["plan"] == cx.PLAN_STREAMED
        assert p["T"] % 4 == 0 and p["ring_bytes"] == 4 and p["H"] >= p["dmin"] + 2 * p["W"]
        assert p["lds_bytes"] == stream_lds(p["R"], p["T"], p["W"], p["chunk"])
        assert p["chunk"] >= p["block_size"]   # 64 descriptor slots per wave
    if spec.weight_dtype == "bf16":
        assert p["R"] * p["T"] <= 65536


WORKLOADS = {
    "brunel_112k": netspec.brunel_112k_alpha(),
    "microcircuit_77k": netspec.microcircuit_77k(),
    "brunel_2m_bf16": netspec.brunel_2m_bf16(),
    "batched_64": netspec.batched_brunel(),
    "batched_48": netspec.batched_brunel(netspec.batch_sizes()[:48]),
    "small": netspec.small_brunel(n_e=6400, n_i=1600, c_e=160, c_i=40, delay="uniform_int", d0=2, d1=12),
}


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_automatic_plans_pass_their_checks(name):
    spec = WORKLOADS[name]
    p = cx.cortex_plan(spec, **MI355X)
    check(p, spec)
    if name == "brunel_2m_bf16":
        # 240 MB of rings cannot be resident in 40 MB of LDS
        assert p["plan"] == cx.PLAN_STREAMED and p["thread_segments"] == 1
    if name == "brunel_112k":
        assert p["plan"] == cx.PLAN_RESIDENT and p["tiles"] == 256 and p["W"] == 5


@pytest.mark.parametrize("name", ["small", "batched_48", "brunel_112k"])
def test_every_explicit_request_is_a_checked_plan_or_an_error(name):
    spec = WORKLOADS[name]
    seen = 0
    for tile, bs, w, kind, pc in itertools.product((0, 64, 128, 300, 1000, 1024, 2048), (0, 256, 512, 1024),
                                                  (0, 1, 2), ("auto", "resident", "streamed"), (0, 1, 2)):
        try:
            p = cx.cortex_plan(spec, tile_size=tile, block_size=bs, steps_per_sync=w, plan=kind, wg_per_cu=pc,
                               **MI355X)
        except cx.CortexError as e:
            assert e.status in (cx.EINVAL, cx.EUNSUPPORTED), e
            continue
        check(p, spec)
        if kind != "auto":
            assert p["plan"] == (cx.PLAN_RESIDENT if kind == "resident" else cx.PLAN_STREAMED)
        seen += 1
    assert seen > 20


def test_four_neurons_per_thread_only_in_512_thread_workgroups():
    spec = WORKLOADS["small"]
    with pytest.raises(cx.CortexError) as e:
        cx.cortex_plan(spec, tile_size=1024, block_size=256, plan="resident", **MI355X)
    assert e.value.status in (cx.EINVAL, cx.EUNSUPPORTED)
    p = cx.cortex_plan(spec, tile_size=2048, block_size=512, plan="resident", **MI355X)
    assert p["npt"] == 4 and p["block_size"] == 512


def test_adjoint_needs_the_resident_plan():
    with pytest.raises(cx.CortexError) as e:
        cx.cortex_plan(WORKLOADS["brunel_2m_bf16"], ckpt_every=100, adjoint_steps=1000, **MI355X)
    assert e.value.status == cx.EUNSUPPORTED


@pytest.mark.parametrize("name", ["brunel_112k", "brunel_2m_bf16", "batched_64"])
def test_autotuner_candidates_are_distinct_checked_plans(name):
    spec = WORKLOADS[name]
    cands = cx.plan_candidates(spec, MI355X["n_cu"], MI355X["lds_per_cu"], MI355X["threads_per_cu"])
    sigs = {tuple(p[f] for f in cx.PLAN_FIELDS) for _, p in cands}
    assert len(sigs) == len(cands) >= 2
    for req, p in cands:
        check(p, spec)
        assert set(req) == set(cx.PLAN_KEYS)
        assert cx.cortex_plan(spec, **MI355X, **req) == p


def test_tuned_plan_table_lookup(tmp_path):
    import json
    spec = WORKLOADS["small"]
    dev = {"name": "AMD Instinct MI355X gfx950", "n_cu": 256}
    other = {"name": "AMD Instinct MI355X gfx950", "n_cu": 128}
    req = dict(plan="streamed", wg_per_cu=2, block_size=0, steps_per_sync=1, tile_size=0)
    path = tmp_path / "plans.json"
    path.write_text(json.dumps({"format": 1, "entries": {cx.tune_key(spec, dev): {"request": req}}}))
    got, entry = cx.lookup_plan(spec, dev, paths=[str(path)])
    assert got == req and entry["request"] == req
    assert cx.lookup_plan(spec, other, paths=[str(path)]) == (None, None)
    assert cx.lookup_plan(WORKLOADS["brunel_112k"], dev, paths=[str(path)]) == (None, None)
    # a missing or foreign file is an empty table
    assert cx.lookup_plan(spec, dev, paths=[str(tmp_path / "none.json")]) == (None, None)


def test_plasticity_plans_are_streamed_with_short_windows():
    base = netspec.small_brunel(n_e=800, n_i=200, c_e=80, c_i=20, delay="const", d0=3.0, J=0.2)
    spec = netspec.NetSpec(**{**base.__dict__, "stdp": netspec.Stdp(pop=0, w0=0.2, wmax=0.6)})
    p = cx.cortex_plan(spec, **MI355X)
    check(p, spec)
    # a source spikes at most once per window: W <= n_ref + 1 = 21
    assert p["plan"] == cx.PLAN_STREAMED and p["W"] == 8
    short = netspec.NetSpec(**{**spec.__dict__, "t_ref": 0.3})   # n_ref = 3
    assert cx.cortex_plan(short, **MI355X)["W"] == 4
    with pytest.raises(cx.CortexError) as e:
        cx.cortex_plan(short, steps_per_sync=8, **MI355X)
    assert e.value.status == cx.EINVAL
    with pytest.raises(cx.CortexError) as e:
        cx.cortex_plan(spec, plan="resident", **MI355X)
    assert e.value.status == cx.EUNSUPPORTED
    bf16 = netspec.NetSpec(**{**spec.__dict__, "weight_dtype": "bf16"})
    with pytest.raises(cx.CortexError) as e:
        cx.cortex_plan(bf16, **MI355X)
    assert e.value.status == cx.EUNSUPPORTED
    bad = netspec.NetSpec(**{**spec.__dict__, "stdp": netspec.Stdp(pop=5)})
    with pytest.raises(cx.CortexError) as e:
        cx.cortex_plan(bad, **MI355X)
    assert e.value.status == cx.EINVAL


def test_conductance_plans_are_resident_with_64_bit_rings():
    inst = netspec.brunel_instance(800, 200, 80, 20, 1.0, 5.0, delay="uniform_int", d0=10, d1=20)
    spec = netspec.NetSpec(model="cond", tau_m=20.0, C_m=250.0, E_L=-70.0, V_th=-50.0, V_reset=-60.0,
                           tau_syn=2.0, poisson_lambda=0.45, w_ext=0.5, instances=[inst])
    p = cx.cortex_plan(spec, **MI355X)
    check(p, spec)
    assert p["plan"] == cx.PLAN_RESIDENT and p["ring_bytes"] == 8
    for bad, status in ((dict(plan="streamed"), cx.EUNSUPPORTED),):
        with pytest.raises(cx.CortexError) as e:
            cx.cortex_plan(spec, **bad, **MI355X)
        assert e.value.status == status
    psp = netspec.NetSpec(**{**spec.__dict__, "weight_unit": "psp_mV"})
    with pytest.raises(cx.CortexError) as e:
        cx.cortex_plan(psp, **MI355X)
    assert e.value.status == cx.EINVAL
    # a network too large for the resident plan is refused, not streamed
    big = netspec.brunel_2m_bf16()
    big = netspec.NetSpec(**{**big.__dict__, "model": "cond", "weight_dtype": "fp32", "tau_syn": 2.0})
    with pytest.raises(cx.CortexError) as e:
        cx.cortex_plan(big, **MI355X)
    assert e.value.status == cx.EUNSUPPORTED


def test_staging_applies_to_one_instance_with_short_segments():
    big = netspec.brunel_2m_bf16()
    p = cx.cortex_plan(big, **MI355X)
    check(p, big)
    # a window at 50 Hz: K T W dt 50 Hz records per tile, 4-byte records within 4 GiB
    K, T, W = 11250, p["T"], p["W"]
    want = -(-int(np.ceil(K * T * W * big.dt * 1e-3 * 50.0)) // 64) * 64
    assert p["thread_segments"] == 1 and p["stage_records"] == max(4096, want)
    assert p["stage_records"] * p["tiles"] * 4 <= 4 << 30
    assert cx.cortex_plan(big, stage_records=-1, **MI355X)["stage_records"] == 0
    assert cx.cortex_plan(big, stage_records=5000, **MI355X)["stage_records"] == 5000
    # rounded up to whole 16-byte pieces of 4-byte records
    for asked, got in ((5001, 5004), (1, 4), (4, 4)):
        assert cx.cortex_plan(big, stage_records=asked, **MI355X)["stage_records"] == got
    # long segments, or several instances: no staging
    s50 = netspec.brunel_2m_bf16(scale_n=0.025)
    assert cx.cortex_plan(s50, plan="streamed", **MI355X)["stage_records"] == 0
    assert cx.cortex_plan(s50, plan="streamed", tile_size=64, **MI355X)["stage_records"] > 0
    multi = netspec.batched_brunel([2000, 3000])
    p = cx.cortex_plan(multi, plan="streamed", tile_size=64, **MI355X)
    assert p["thread_segments"] == 1 and p["stage_records"] == 0
