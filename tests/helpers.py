"""Shared test helpers: spike statistics and graph comparison."""
import numpy as np
import scipy.sparse


def pop_ranges(spec):
    out = []
    g = 0
    for inst in spec.instances:
        for p in inst.pops:
            out.append((g, g + p.size))
            g += p.size
    return out


def rates_and_cv(steps, ids, spec, t0_steps, t1_steps, dt=0.1):
    """Per-population rate (Hz) and mean ISI CV over neurons with >= 3 spikes,
    for spikes with step in [t0, t1)."""
    steps = np.asarray(steps, np.int64)
    ids = np.asarray(ids, np.int64)
    m = (steps >= t0_steps) & (steps < t1_steps)
    steps, ids = steps[m], ids[m]
    T = (t1_steps - t0_steps) * dt * 1e-3
    order = np.lexsort((steps, ids))
    steps, ids = steps[order], ids[order]
    res = []
    for a, b in pop_ranges(spec):
        sel = (ids >= a) & (ids < b)
        rate = sel.sum() / ((b - a) * T)
        cvs = []
        s_ids, s_st = ids[sel], steps[sel]
        if len(s_ids):
            bounds = np.flatnonzero(np.diff(s_ids)) + 1
            for grp in np.split(s_st, bounds):
                if len(grp) >= 3:
                    isi = np.diff(grp).astype(np.float64)
                    cvs.append(isi.std() / isi.mean())
        res.append((rate, float(np.mean(cvs)) if cvs else float("nan")))
    return res


def sorted_edges(src, tgt, w, d):
    """Edges as rows (tgt, src, d, w) in lexicographic order."""
    order = np.lexsort((w, d, src, tgt))
    return tgt[order], src[order], d[order], w[order]


def abs_input_bound(src, tgt, w, d, steps, ids, N, T):
    """B[n, i] = sum over events arriving at (n, i) of |w| (sparse, per delay)."""
    S = scipy.sparse.csr_matrix((np.ones(len(steps)), (np.asarray(steps, np.int64),
                                                       np.asarray(ids, np.int64))), shape=(T, N))
    B = np.zeros((T, N))
    for dv in np.unique(d):
        m = d == dv
        Wd = scipy.sparse.csr_matrix((np.abs(w[m]), (tgt[m], src[m])), shape=(N, N))
        if dv < T:
            B[dv:] += (S[:T - dv] @ Wd.T).toarray()
    return B
