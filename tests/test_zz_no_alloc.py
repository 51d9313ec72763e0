"""The allocation-free frozen run (cortex_run_frozen_noalloc, through the C
ABI) against cortex_run_frozen: the same traces, bit for bit, on two calls in
a row (the second one smaller), on both launch plans."""
import ctypes as C

import numpy as np
import pytest

import netspec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2406_03762_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("plan", ["resident", "streamed"])
def test_noalloc_run_matches_run_frozen_on_two_calls(cx, plan):
    import torch
    spec = netspec.small_brunel(model="alpha", n_e=1600, n_i=400, c_e=160, c_i=40, delay="uniform_int",
                                d0=3, d1=17, w_rel_sd=0.1, weight_unit="psp_mV")
    print(f"[case] noalloc vs run_frozen, plan {plan}", flush=True)
    ga = cx.Network(spec, 17, plan=plan, tile_size=300)
    gb = cx.Network(spec, 17, plan=plan, tile_size=300)
    steps, ids = netspec.synthetic_raster(2000, 200, 0.02, seed=21)
    done = 0
    for T, keep in ((150, 1.0), (40, 0.3)):
        # the second call: fewer steps and a thinned raster
        m = np.random.default_rng(T).random(len(steps)) < keep
        st, ii = steps[m], ids[m]
        xa = torch.empty((T, ga.N), dtype=torch.float32, device="cuda")
        va = torch.empty_like(xa)
        xb = torch.full_like(xa, np.nan)
        vb = torch.full_like(xa, np.nan)
        cx.cortex_run_frozen(ga._h, st, ii, T, xa, va, device=ga.device)
        sb = np.ascontiguousarray(st, np.uint32)
        ib = np.ascontiguousarray(ii, np.uint32)
        rc = cx.lib().cortex_run_frozen_noalloc(gb._h, sb.ctypes.data, ib.ctypes.data, len(sb), T,
                                               xb.data_ptr(), vb.data_ptr())
        assert rc == cx.OK, cx.lib().cortex_last_error().decode()
        torch.cuda.synchronize()
        assert torch.equal(xa, xb) and torch.equal(va, vb)
        assert float(xa.abs().max()) > 0
        done += T
        assert gb.query("STEP") == done and gb.query("EVENTS") == ga.query("EVENTS")
    # too large for the fixed array: rejected before any device work
    rc = cx.lib().cortex_run_frozen_noalloc(gb._h, None, None, 0, 10 ** 8, None, None)
    assert rc == cx.EINVAL and "allocation-free" in cx.lib().cortex_last_error().decode()
    ga.close()
    gb.close()


def test_noalloc_run_rejects_fp64(cx):
    spec = netspec.small_brunel(precision="fp64")
    g = cx.Network(spec, 3)
    rc = cx.lib().cortex_run_frozen_noalloc(g._h, None, None, 0, 5, None, None)
    assert rc == cx.EUNSUPPORTED
    g.close()
