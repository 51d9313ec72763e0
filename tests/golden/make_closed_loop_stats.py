"""Write the closed-loop statistics of the CPU oracle for the full-size FP32
workloads (the expected values of the GPU statistical-parity tests).

Calls only the oracle: builds the named network, runs it closed loop in FP64
for the stated number of steps and stores, per population, the firing rate
and the mean ISI coefficient of variation (first 100 ms discarded; CV over
neurons with at least 3 spikes), plus the total spike count and a hash of the
network description so that a changed workload is detected.

    python tests/golden/make_closed_loop_stats.py brunel_112k_alpha
    python tests/golden/make_closed_loop_stats.py microcircuit_77k
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import netspec  # noqa: E402
import oracle  # noqa: E402
from tests import helpers  # noqa: E402

def bf16_rne(x):
    """Round float64 values to the nearest bfloat16 (8 significant bits),
    ties to even."""
    m, e = np.frexp(np.asarray(x, np.float64))
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


WORKLOADS = {
    # name: (spec factory, seed, steps)
    "brunel_112k_alpha": (netspec.brunel_112k_alpha, 2, 10000),
    # 5 s: the smallest population (1,543 neurons at about 3 Hz) then gives
    # about 22,000 spikes, a rate known to 0.7 %
    "microcircuit_77k": (netspec.microcircuit_77k, 3, 50000),
    # same in-degree as the two-million-neuron bf16 network, 1 % / 2.5 % of
    # its neurons (a surrogate: the full size does not fit the host)
    "brunel_2m_bf16_surrogate_20k": (lambda: netspec.brunel_2m_bf16(scale_n=0.01), 5, 10000),
    "brunel_2m_bf16_surrogate_50k": (lambda: netspec.brunel_2m_bf16(scale_n=0.025), 5, 10000),
}


def spec_hash(spec) -> str:
    text = repr(spec)
    if spec.model == "cond":   # fields repr() leaves out
        text += f"|E_ex={spec.E_ex}|E_in={spec.E_in}"
    if spec.stdp is not None:
        text += f"|{spec.stdp!r}"
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def path_of(name: str) -> str:
    return os.path.join(HERE, f"closed_loop_{name}.json")


def main(name: str) -> None:
    make, seed, steps = WORKLOADS[name]
    spec = make()
    t0 = time.time()
    o = oracle.OracleNet(spec, seed)
    t_build = time.time() - t0
    print(f"[golden] {name}: built N={o.N} E={o.E} in {t_build:.0f} s", flush=True)
    if spec.weight_dtype == "bf16":
        # the weights the library stores
        _, _, w, _ = o.graph()
        o.set_weights(bf16_rne(w))
        del w
    t0 = time.time()
    chunk = 2500
    for s in range(0, steps, chunk):
        o.run(min(chunk, steps - s))
        print(f"[golden] {name}: step {s + chunk}/{steps} ({time.time() - t0:.0f} s)", flush=True)
    st, ids = o.spikes()
    stats = helpers.rates_and_cv(st, ids, spec, 1000, steps)
    out = {
        "workload": name, "seed": seed, "steps": steps, "discard_steps": 1000,
        "spec_hash": spec_hash(spec), "neurons": int(o.N), "synapses": int(o.E),
        "spikes": int(len(st)), "events": float(o.events),
        "rates_hz": [r for r, _ in stats], "cv": [c for _, c in stats],
        "oracle_run_s": time.time() - t0,
    }
    with open(path_of(name), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
