"""Checkpoint and resume (cortex_save_state / cortex_load_state): a network
built from the same spec and seed and loaded with a state saved after T1
steps continues exactly as the saved network does over the next T2 steps --
the same spikes, the same neuron state, the same event count and, with
plasticity, the same weights, bit for bit.  T1 is not a multiple of the
exchange window, so the state is saved inside a window's cycle."""
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


def _plastic(spec, **kw):
    return netspec.NetSpec(**{**spec.__dict__, "stdp": netspec.Stdp(pop=0, **kw)})


def _resume_matches(cx, spec, seed, T1, T2, plan_kind, weights=False, **req):
    a = cx.Network(spec, seed, record_steps=T1 + T2, **req)
    assert a.query("PLAN") == plan_kind
    a.step(T1)
    buf = a.save_state()
    assert buf.size == cx.cortex_state_size(a._h)
    a.step(T2)
    sa, ia = a.spikes(0, T1 + T2)
    stat_a = a.state()
    ev_a = a.query("EVENTS")
    w_a = a.graph()[2] if weights else None
    a.close()

    b = cx.Network(spec, seed, record_steps=T1 + T2, **req)
    b.load_state(buf)
    assert b.query("STEP") == T1
    b.step(T2)
    sb, ib = b.spikes(0, T1 + T2)
    stat_b = b.state()
    ev_b = b.query("EVENTS")
    w_b = b.graph()[2] if weights else None
    b.close()

    print("spikes", len(sa), "events", ev_a, flush=True)
    assert len(sa) > 100 and np.count_nonzero(sa >= T1) > 50
    assert np.array_equal(sa, sb) and np.array_equal(ia, ib)
    for x, y in zip(stat_a, stat_b):
        assert np.array_equal(x, y)
    assert ev_a == ev_b
    if weights:
        assert np.array_equal(w_a, w_b)
    return buf


def test_resume_resident_plan(cx):
    spec = netspec.small_brunel(model="alpha", n_e=4000, n_i=1000, c_e=400, c_i=100, delay="uniform_int",
                                d0=5, d1=30, J=0.1, lam=2.0, weight_unit="psp_mV")
    case("resident plan, 5,000 neurons, save at step 1,003")
    _resume_matches(cx, spec, 31, 1003, 1500, cx.PLAN_RESIDENT, plan="resident")


def test_resume_streamed_plan_with_staging(cx):
    spec = netspec.brunel_2m_bf16(scale_n=0.05)
    case("streamed plan with staging, 100,000 neurons bf16, save at step 1,003")
    _resume_matches(cx, spec, 5, 1003, 600, cx.PLAN_STREAMED, plan="streamed", tile_size=128, steps_per_sync=5)


def test_resume_streamed_plan_with_plasticity(cx):
    base = netspec.small_brunel(n_e=4000, n_i=1000, c_e=400, c_i=100, delay="uniform_int", d0=5, d1=30,
                                w_rel_sd=0.1, J=0.1, lam=2.0)
    spec = _plastic(base, lam=0.05, alpha=1.0, w0=0.1, wmax=0.3)
    case("streamed plan with E->E plasticity, 5,000 neurons, save at step 1,001")
    _resume_matches(cx, spec, 23, 1001, 1000, cx.PLAN_STREAMED, weights=True)


def test_state_of_another_network_is_refused(cx):
    spec = netspec.small_brunel(n_e=800, n_i=200, c_e=80, c_i=20)
    case("state errors")
    a = cx.Network(spec, 1, record_steps=100)
    a.step(50)
    buf = a.save_state()
    a.close()
    for other in (dict(seed=2), dict(seed=1, record_steps=200)):
        g = cx.Network(spec, other.get("seed"), record_steps=other.get("record_steps", 100))
        with pytest.raises(cx.CortexError) as e:
            g.load_state(buf)
        assert e.value.status == cx.EINVAL
        g.close()
    g = cx.Network(spec, 1, record_steps=100)
    with pytest.raises(cx.CortexError) as e:
        g.load_state(buf[:100])
    assert e.value.status == cx.EINVAL
    g.close()
    f = cx.Network(spec, 1, ckpt_every=50, adjoint_steps=100)
    with pytest.raises(cx.CortexError) as e:
        f.save_state()
    assert e.value.status == cx.EUNSUPPORTED
    f.close()


def test_resume_fp64_verify_mode(cx):
    spec = netspec.brunel_1250_fp64()
    case("FP64 verify mode, 1,250 neurons, save at step 151")
    a = cx.Network(spec, 1, record_steps=400)
    a.step(151)
    buf = a.save_state()
    a.step(249)
    sa, ia = a.spikes(0, 400)
    stat_a = a.state()
    a.close()
    b = cx.Network(spec, 1, record_steps=400)
    b.load_state(buf)
    b.step(249)
    sb, ib = b.spikes(0, 400)
    stat_b = b.state()
    b.close()
    print("spikes", len(sa), flush=True)
    assert np.count_nonzero(sa >= 151) > 50
    assert np.array_equal(sa, sb) and np.array_equal(ia, ib)
    for x, y in zip(stat_a, stat_b):
        assert np.array_equal(x, y)
