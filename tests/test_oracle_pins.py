"""Pins of the CPU oracle against things other than itself.

Each test checks an oracle function against a library routine (numpy's
Philox, scipy's Poisson CDF and matrix exponential, scipy.signal.lfilter), a
closed form of the linear LIF ODE, brute force on tiny inputs, or exact
invariants of the generated graph.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import scipy.signal
import scipy.stats

import netspec
from netspec import Instance, NetSpec, Population, Projection

TWO64 = 2.0 ** 64


def np_philox(ctr, key):
    """Block at counter ``ctr`` from numpy's Philox4x64-10 (which increments
    its counter before producing output)."""
    v = (sum(int(x) << (64 * i) for i, x in enumerate(ctr)) - 1) % (1 << 256)
    cm1 = np.array([(v >> (64 * i)) & (2 ** 64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=cm1, key=np.array(key, dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


# ---------------------------------------------------------------- Philox

def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(11)
    cases = [((0, 0, 0, 0), (0, 0)), ((2 ** 64 - 1, 2 ** 64 - 1, 5, 1), (7, 9))]
    for _ in range(40):
        cases.append((tuple(int(x) for x in rng.integers(0, 2 ** 63, 4)),
                      tuple(int(x) for x in rng.integers(0, 2 ** 63, 2))))
    for ctr, key in cases:
        assert [int(x) for x in orc.philox4x64_10(ctr, key)] == np_philox(ctr, key)


# ---------------------------------------------------------------- Poisson

@pytest.mark.parametrize("lam", [0.5, 0.8, 2.0, 5.0])
def test_poisson_table_matches_scipy_cdf(orc, lam):
    thr = orc.poisson_table(lam)
    m = np.arange(len(thr))
    ref = np.floor(scipy.stats.poisson.cdf(m, lam) * 2.0 ** 32)
    assert np.all(np.abs(thr.astype(np.float64) - ref) <= 1.0)
    assert np.all(np.diff(thr.astype(np.int64)) >= 0)
    # counts run up to M = len(thr): the mass folded into M (counts above M)
    # is below 2^-32, and the last entry still separates more than that
    M = len(thr)
    assert scipy.stats.poisson.sf(M, lam) <= 2.0 ** -32 * 1.01
    assert scipy.stats.poisson.sf(M - 1, lam) > 2.0 ** -32 * 0.99


def _counting_spec(lam, n=2000):
    # delta neuron with no leak (P22 == 1), no synapses, w_ext = 1: the
    # membrane potential counts the Poisson events exactly
    inst = Instance([Population("A", n)], [])
    return NetSpec(model="delta", tau_m=1e300, poisson_lambda=lam, w_ext=1.0,
                   V_th=1e12, V_reset=0.0, v0_lo=0.0, v0_hi=0.0, instances=[inst])


@pytest.mark.parametrize("lam", [0.8, 2.0])
def test_poisson_counts_statistics(orc, lam):
    n, T = 2000, 500
    net = orc.OracleNet(_counting_spec(lam, n), seed=5)
    _, v = net.run_frozen(np.zeros(0, np.int64), np.zeros(0, np.int64), T, record_x=False)
    v = np.vstack([np.zeros((1, n)), v])
    k = np.rint(np.diff(v, axis=0)).astype(np.int64)
    assert np.allclose(np.diff(v, axis=0), k)
    draws = k.size
    assert abs(k.mean() - lam) < 5 * math.sqrt(lam / draws)
    assert abs(k.var() - lam) < 5 * lam * math.sqrt(2.0 / draws) + 5 * lam / math.sqrt(draws)
    kmax = int(scipy.stats.poisson.ppf(1 - 1e-6, lam))
    obs = np.bincount(np.minimum(k.ravel(), kmax), minlength=kmax + 1)
    p = scipy.stats.poisson.pmf(np.arange(kmax + 1), lam)
    p[-1] = scipy.stats.poisson.sf(kmax - 1, lam)
    chi2 = ((obs - draws * p) ** 2 / (draws * p)).sum()
    assert scipy.stats.chi2.sf(chi2, kmax) > 1e-4
    # successive steps and neighbouring neurons are uncorrelated
    a = (k[1:] - lam).ravel()
    b = (k[:-1] - lam).ravel()
    assert abs((a * b).mean() / lam) < 5 / math.sqrt(a.size)
    c = (k[:, 1:] - lam).ravel()
    d = (k[:, :-1] - lam).ravel()
    assert abs((c * d).mean() / lam) < 5 / math.sqrt(c.size)


# ---------------------------------------------------------------- propagators

def _system(model, tm, ts, C):
    """Linear ODE matrix: delta (U); exp (U, I); alpha (U, y2, y1)."""
    if model == "delta":
        return np.array([[-1.0 / tm]])
    if model == "exp":
        return np.array([[-1.0 / tm, 1.0 / C], [0.0, -1.0 / ts]])
    return np.array([[-1.0 / tm, 1.0 / C, 0.0], [0.0, -1.0 / ts, 1.0], [0.0, 0.0, -1.0 / ts]])


@pytest.mark.parametrize("model,ts", [("delta", 0.5), ("exp", 0.5), ("exp", 2.0),
                                      ("alpha", 0.5), ("alpha", 5.0)])
def test_propagators_match_matrix_exponential(orc, model, ts):
    s = NetSpec(model=model, tau_syn=ts, tau_m=20.0, C_m=250.0, dt=0.1,
                instances=[Instance([Population("A", 1)], [])])
    k = orc.constants(s)
    M = scipy.linalg.expm(_system(model, 20.0, ts, 250.0) * 0.1)
    assert k["P22"] == pytest.approx(M[0, 0], rel=1e-13)
    # constant current: augmented state (U, I_e)
    Ma = scipy.linalg.expm(np.array([[-1 / 20.0, 1 / 250.0], [0.0, 0.0]]) * 0.1)
    assert k["P20"] == pytest.approx(Ma[0, 1], rel=1e-12)
    if model == "exp":
        assert k["P21"] == pytest.approx(M[0, 1], rel=1e-12)
        assert k["P11"] == pytest.approx(M[1, 1], rel=1e-13)
    if model == "alpha":
        assert k["P32"] == pytest.approx(M[0, 1], rel=1e-12)
        assert k["P31"] == pytest.approx(M[0, 2], rel=1e-11)
        assert k["P22s"] == pytest.approx(M[1, 1], rel=1e-13)
        assert k["P21s"] == pytest.approx(M[1, 2], rel=1e-13)
        assert k["P11"] == pytest.approx(M[2, 2], rel=1e-13)
    assert k["n_ref"] == 20


def _unit_psp(model, t, tm=20.0, ts=0.5, C=250.0):
    """Membrane response at t to a unit synaptic input at t = 0 (exp: current
    jump of 1; alpha: current whose peak is 1)."""
    A = _system(model, tm, ts, C)
    x0 = np.array([0.0, 1.0]) if model == "exp" else np.array([0.0, 0.0, math.e / ts])
    return (scipy.linalg.expm(A * t) @ x0)[0]


@pytest.mark.parametrize("model,ts", [("exp", 0.5), ("alpha", 0.5), ("alpha", 2.0)])
def test_psp_conversion_is_peak_of_unit_response(orc, model, ts):
    s = NetSpec(model=model, tau_syn=ts, weight_unit="psp_mV",
                instances=[Instance([Population("A", 1)], [])])
    k = orc.constants(s)
    res = scipy.optimize.minimize_scalar(lambda t: -_unit_psp(model, t, ts=ts),
                                         bounds=(1e-6, 40.0), method="bounded",
                                         options={"xatol": 1e-10})
    peak = -res.fun
    assert 1.0 / k["conv"] == pytest.approx(peak, rel=1e-9)
    assert k["tpeak"] == pytest.approx(res.x, rel=1e-4)


# ---------------------------------------------------------------- LIF closed forms

def _single(I_e, model="delta", v0=0.0):
    inst = Instance([Population("A", 1)], [])
    return NetSpec(model=model, I_e=I_e, poisson_lambda=0.0, v0_lo=v0, v0_hi=v0,
                   instances=[inst])


@pytest.mark.parametrize("vinf", [25.0, 30.0, 40.0])
def test_constant_current_firing_times(orc, vinf):
    tm, C, dt, theta, vr, nref = 20.0, 250.0, 0.1, 20.0, 10.0, 20
    net = orc.OracleNet(_single(vinf * C / tm), seed=1)
    net.run(4000)
    st, _ = net.spikes()
    lnp = -dt / tm     # log of the per-step decay e^{-dt/tm}
    k_first = math.ceil(math.log(1.0 - theta / vinf) / lnp)
    k_period = math.ceil(math.log((vinf - theta) / (vinf - vr)) / lnp)
    expect = [k_first - 1]
    while expect[-1] + nref + k_period < 4000:
        expect.append(expect[-1] + nref + k_period)
    assert st.tolist() == expect


def test_subthreshold_relaxation_and_refractory_clamp(orc):
    tm, C, dt, vinf, vr = 20.0, 250.0, 0.1, 25.0, 10.0
    net = orc.OracleNet(_single(vinf * C / tm, v0=3.0), seed=1)
    V0 = net.state()[0][0]
    assert V0 == 3.0
    T = 400
    _, v = net.run_frozen(np.array([150]), np.array([0]), T)
    v = v[:, 0]
    n = np.arange(T)
    p = math.exp(-dt / tm)
    free = vinf + (V0 - vinf) * p ** (n + 1)
    assert np.allclose(v[:150], free[:150], rtol=1e-12, atol=0)
    assert np.all(v[150:171] == vr)     # reset at the spike step, then 20 clamped steps
    after = vinf + (vr - vinf) * p ** (n[171:] - 170)
    assert np.allclose(v[171:], after, rtol=1e-12)


def _pair_spec(model, w, d_ms, weight_unit="native"):
    inst = Instance([Population("A", 1), Population("B", 1)],
                    [Projection(src=0, tgt=1, rule="fixed_indegree", k=1, w_mean=w,
                                delay="const", d0=d_ms)])
    return NetSpec(model=model, tau_syn=0.5, poisson_lambda=0.0, V_th=1e9, v0_lo=0.0,
                   v0_hi=0.0, weight_unit=weight_unit, instances=[inst])


@pytest.mark.parametrize("model", ["delta", "exp", "alpha"])
def test_single_psp_shape_and_arrival_step(orc, model):
    w = 0.7 if model == "delta" else 35.0
    net = orc.OracleNet(_pair_spec(model, w, 1.0), seed=2)
    src, tgt, ww, d = net.graph()
    assert src.tolist() == [0] and tgt.tolist() == [1] and d.tolist() == [10] and ww[0] == w
    T = 200
    x, v = net.run_frozen(np.array([50]), np.array([0]), T)
    arr = 60
    assert x[arr, 1] == w and np.count_nonzero(x[:, 1]) == 1
    vb = v[:, 1]
    assert np.all(vb[:arr] == 0.0)
    n = np.arange(arr, T)
    if model == "delta":
        ref = w * np.exp(-0.1 / 20.0) ** (n - arr)
        assert np.allclose(vb[arr:], ref, rtol=1e-12)
    else:
        # the current jumps after the membrane update of the arrival step
        assert vb[arr] == 0.0
        ref = np.array([w * _unit_psp(model, (m - arr) * 0.1) for m in n[1:]])
        assert np.allclose(vb[arr + 1:], ref, rtol=1e-10, atol=1e-14)


def test_psp_unit_weight_peaks_at_requested_mv(orc):
    net = orc.OracleNet(_pair_spec("alpha", 0.1, 1.0, weight_unit="psp_mV"), seed=2)
    _, v = net.run_frozen(np.array([5]), np.array([0]), 400)
    # the grid maximum can only undershoot the continuous peak slightly
    assert 0.1 * (1 - 1e-3) < v[:, 1].max() <= 0.1 * (1 + 1e-12)


# ---------------------------------------------------------------- graph

def test_fixed_indegree_invariants_and_stream_layout(orc):
    J, g = 0.1, 5.0
    spec = netspec.small_brunel(n_e=400, n_i=100, c_e=40, c_i=10, delay="uniform_int",
                                d0=5, d1=30, w_rel_sd=0.1)
    seed = 77
    net = orc.OracleNet(spec, seed)
    src, tgt, w, d = net.graph()
    N = 500
    assert net.E == N * 50
    # canonical order: targets ascending, in-degree exact per projection
    assert np.all(np.diff(tgt) >= 0)
    for i in range(0, N, 37):
        s = src[tgt == i]
        assert len(s) == 50
        assert np.all(s[:40] < 400) and np.all(s[40:] >= 400)
        assert i not in s.tolist()                # no autapses
    assert d.min() >= 5 and d.max() <= 30
    cnt = np.bincount(d - 5, minlength=26)
    assert scipy.stats.chisquare(cnt).pvalue > 1e-4
    cnt_src = np.bincount(src[src < 400], minlength=400)
    assert scipy.stats.chisquare(cnt_src).pvalue > 1e-4
    we = w[src < 400]
    wi = w[src >= 400]
    assert abs(we.mean() - J) < 5 * 0.1 * J / math.sqrt(len(we))
    assert abs(we.std() / (0.1 * J) - 1) < 0.05
    assert abs(wi.mean() + g * J) < 5 * 0.1 * g * J / math.sqrt(len(wi))
    # documented stream layout, regenerated with numpy's Philox
    rng = np.random.default_rng(0)
    for e in rng.choice(net.E, size=60, replace=False):
        i, slot_all = int(tgt[e]), int(e - 50 * tgt[e])
        is_e_tgt = i < 400
        proj_local = (0 if slot_all < 40 else 1) if is_e_tgt else (2 if slot_all < 40 else 3)
        slot = slot_all if slot_all < 40 else slot_all - 40
        wd = np_philox((i, slot, proj_local, 1), (seed, 0))
        if slot_all < 40:
            ns, base, t_in_pop = 400, 0, i
            same = is_e_tgt
        else:
            ns, base, t_in_pop = 100, 400, i - 400
            same = not is_e_tgt
        if same:
            sl = (wd[0] * (ns - 1)) >> 64
            sl += 1 if sl >= t_in_pop else 0
        else:
            sl = (wd[0] * ns) >> 64
        assert src[e] == base + sl
        assert d[e] == 5 + ((wd[1] * 26) >> 64)
        u1 = ((wd[2] >> 11) + 1) * 2.0 ** -53
        u2 = (wd[3] >> 11) * 2.0 ** -53
        z0 = math.sqrt(-2.0 * math.log(u1)) * math.cos(6.283185307179586 * u2)
        mean, sd = (J, 0.1 * J) if slot_all < 40 else (-g * J, 0.1 * g * J)
        assert w[e] == pytest.approx(mean + sd * z0, rel=1e-14, abs=1e-17)


def test_pairwise_bernoulli_invariants(orc):
    n = 300
    p = 0.1
    inst = Instance([Population("A", n)],
                    [Projection(src=0, tgt=0, rule="pairwise", p=p, w_mean=1.0,
                                delay="normal", d0=1.5, d1=0.75)])
    spec = NetSpec(model="exp", instances=[inst])
    seed = 9
    net = orc.OracleNet(spec, seed)
    src, tgt, w, d = net.graph()
    counts = np.bincount(tgt, minlength=n)
    assert abs(counts.mean() - (n - 1) * p) < 5 * math.sqrt((n - 1) * p * (1 - p) / n)
    for i in range(0, n, 29):
        s = src[tgt == i]
        assert len(np.unique(s)) == len(s) and i not in s.tolist()
        assert np.all(np.diff(s) > 0)
        # pair (i, j) exists iff the documented word is below p 2^64
        expect = []
        thr = int(math.ldexp(p, 64))
        for j in range(n):
            if j == i:
                continue
            if np_philox((i, j >> 2, 0, 5), (seed, 0))[j & 3] < thr:
                expect.append(j)
        assert s.tolist() == expect
    # rounded normal delays, clipped below at one step: exact pmf
    k = np.arange(1, d.max() + 1)
    cdf = scipy.stats.norm.cdf
    pmf = cdf((k + 0.5 - 15.0) / 7.5) - cdf((k - 0.5 - 15.0) / 7.5)
    pmf[0] = cdf((1.5 - 15.0) / 7.5)
    obs = np.bincount(d, minlength=d.max() + 1)[1:]
    keep = len(d) * pmf > 20
    chi2 = (((obs - len(d) * pmf) ** 2) / (len(d) * pmf))[keep].sum()
    assert scipy.stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4


def test_selected_targets_get_the_same_in_edges(orc):
    spec = netspec.small_brunel(n_e=200, n_i=50, c_e=20, c_i=5)
    full = orc.OracleNet(spec, 3)
    sel = np.array([0, 7, 120, 201, 249])
    part = orc.OracleNet(spec, 3, sel=sel)
    fs, ft, fw, fd = full.graph()
    ps, pt, pw, pd = part.graph()
    m = np.isin(ft, sel)
    assert np.array_equal(fs[m], ps) and np.array_equal(ft[m], pt)
    assert np.array_equal(fw[m], pw) and np.array_equal(fd[m], pd)


# ---------------------------------------------------------------- delivery

def dense_input(src, tgt, w, d, steps, ids, N, T):
    """x[n, i] = sum_d sum_j W_d[i, j] s_j(n - d), brute force."""
    S = np.zeros((T, N))
    S[steps, ids] = 1.0
    x = np.zeros((T, N))
    for dv in np.unique(d):
        Wd = np.zeros((N, N))
        m = d == dv
        np.add.at(Wd, (tgt[m], src[m]), w[m])
        if dv < T:
            x[dv:] += S[:T - dv] @ Wd.T
    return x


@pytest.mark.parametrize("model", ["delta", "exp", "alpha"])
def test_delivery_matches_dense_brute_force(orc, model):
    spec = netspec.small_brunel(model=model, n_e=48, n_i=12, c_e=6, c_i=2, delay="uniform_int",
                                d0=1, d1=7)
    net = orc.OracleNet(spec, 4)
    src, tgt, w, d = net.graph()
    T = 200
    steps, ids = netspec.synthetic_raster(60, T, 0.05, seed=8)
    x, _ = net.run_frozen(steps, ids, T)
    ref = dense_input(src, tgt, w, d, steps.astype(np.int64), ids.astype(np.int64), 60, T)
    assert np.allclose(x, ref, rtol=1e-12, atol=1e-14)
    # every pushed edge is one synaptic event
    outdeg = np.bincount(src, minlength=60)
    assert net.events == outdeg[ids].sum()


def test_selected_target_trace_equals_full_columns(orc):
    spec = netspec.small_brunel(model="alpha", n_e=48, n_i=12, c_e=6, c_i=2)
    sel = np.array([3, 17, 59])
    steps, ids = netspec.synthetic_raster(60, 150, 0.05, seed=8)
    xf, vf = orc.OracleNet(spec, 4).run_frozen(steps, ids, 150)
    xs, vs = orc.OracleNet(spec, 4, sel=sel).run_frozen(steps, ids, 150)
    assert np.array_equal(xf[:, sel], xs) and np.array_equal(vf[:, sel], vs)


# ---------------------------------------------------------------- adjoint

def _loss(v, vstar, spec):
    L = 0.0
    off = 0
    T = v.shape[0]
    for inst in spec.instances:
        nb = inst.n_neurons
        L += ((v[:, off:off + nb] - vstar[:, off:off + nb]) ** 2).sum() / (nb * T)
        off += nb
    return L


@pytest.mark.parametrize("model", ["delta", "exp", "alpha"])
def test_adjoint_matches_central_differences(orc, model):
    spec = netspec.small_brunel(model=model, n_e=24, n_i=6, c_e=5, c_i=2, delay="uniform_int",
                                d0=1, d1=6, J=0.1 if model == "delta" else 40.0)
    T = 120
    steps, ids = netspec.refractory_raster(30, T, 0.03, seed=12, n_ref=20)
    vstar = netspec.target_trace(30, T, 10.0, 20.0, seed=13)
    net = orc.OracleNet(spec, 21)
    grad, L = net.backward(steps, ids, T, vstar)
    net.reset()
    _, v = net.run_frozen(steps, ids, T)
    assert L == pytest.approx(_loss(v, vstar, spec), rel=1e-12)
    _, _, w, _ = net.graph()
    rng = np.random.default_rng(1)
    checked = 0
    for e in rng.permutation(net.E):
        h = 1e-3 * max(abs(w[e]), 1e-3)
        vals = []
        for sgn in (1, -1):
            net.set_weight(e, w[e] + sgn * h)
            net.reset()
            _, v = net.run_frozen(steps, ids, T)
            vals.append(_loss(v, vstar, spec))
        net.set_weight(e, w[e])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert fd == pytest.approx(grad[e], rel=1e-5, abs=1e-9 * max(1.0, abs(L)) / h)
        checked += 1
        if checked == 25:
            break
    assert np.count_nonzero(grad) > 0


@pytest.mark.parametrize("model", ["delta", "exp", "alpha"])
def test_adjoint_without_resets_is_a_linear_filter(orc, model):
    # sources in A spike; targets in B never do, so V_B is a linear
    # time-invariant response to its input
    nA, nB, T = 20, 5, 150
    w0 = 0.2 if model == "delta" else 30.0
    inst = Instance([Population("A", nA), Population("B", nB)],
                    [Projection(src=0, tgt=1, rule="fixed_indegree", k=6, w_mean=w0,
                                w_sd=0.1 * w0, delay="uniform_int", d0=1, d1=9)])
    spec = NetSpec(model=model, tau_syn=0.5, poisson_lambda=0.0, V_th=1e9, instances=[inst])
    steps, ids = netspec.refractory_raster(nA, T, 0.05, seed=3, n_ref=20)
    vstar = netspec.target_trace(nA + nB, T, 0.0, 5.0, seed=4)
    net = orc.OracleNet(spec, 5)
    grad, _ = net.backward(steps, ids, T, vstar)
    net.reset()
    _, v = net.run_frozen(steps, ids, T)
    src, tgt, _, d = net.graph()
    N = nA + nB
    lprime = 2.0 * (v - vstar) / (N * T)
    p22 = math.exp(-0.1 / 20.0)
    if model == "delta":
        # g_n = sum_{k >= n} P22^{k-n} l'_k
        g = scipy.signal.lfilter([1.0], [1.0, -p22], lprime[::-1], axis=0)[::-1]
    else:
        h = np.array([0.0] + [_unit_psp(model, j * 0.1) for j in range(1, T)])
        g = np.zeros_like(lprime)
        for n in range(T):
            g[n] = (h[:T - n, None] * lprime[n:]).sum(axis=0)
    ref = np.zeros(net.E)
    for q in range(len(steps)):
        m, j = int(steps[q]), int(ids[q])
        for e in np.nonzero(src == j)[0]:
            if m + d[e] < T:
                ref[e] += g[m + d[e], tgt[e]]
    assert np.allclose(grad, ref, rtol=1e-9, atol=1e-15 * np.abs(ref).max())
