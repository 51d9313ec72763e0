"""Throughput of the LIF + delayed delivery step on one MI355X.

Headline workload: the largest single-GPU network, a balanced random network
of 2,000,000 delta-current LIF neurons (1.6 M E / 0.4 M I) with in-degree
9,000 E + 2,250 I (2.25e10 synapses, 16-bit records and bf16 weights, FP32
accumulation), delays uniform on 5..30 steps, dt = 0.1 ms.  Its input rings
(240 MB) exceed the chip's workgroup-local memory, so it runs the streamed
plan: one kernel launch per window of 5 steps over all tiles, replayed from a
captured HIP graph.  One benchmark step simulates 1 s (10,000 time steps);
inputs (graph, state) are resident in HBM before the timed region.  Prints
one JSON line; secondary workloads (the 112,500-neuron alpha net on the
resident persistent plan, the microcircuit stand-in, the FP64 verification
net, the batched instances and the adjoint) are reported beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SIM_STEPS_PER_BENCH_STEP = 10000      # 1 s of biological time at dt = 0.1 ms
CSRC = os.path.join(ROOT, "paper_2406_03762_amd", "csrc")

# HBM bytes per synaptic event of a kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (each scaled by its reading for a plain device copy of known
# size, as the summaries under profiles/ state), valid only for the sources
# they were measured on: {kernel: (bytes per event, source hash)}.
TRAFFIC = {
    # 112,500-neuron alpha net, one 1000-step launch: (3.2547e6 KiB x 2.0
    # + 3.8464e4 KiB x 1.0) x 1024 / 9.708e8 events
    "step_kernel": (6.907, "382a76f1b7e1aa7d"),
    # two-million-neuron bf16 net, the 2,000 window launches of each kernel
    # in the timed second of a run after one second of warmup, 1.59677e11
    # events: delivery (5.4019e8 KiB x 2.0 + 4.4249e8 KiB x 1.0) x 1024,
    # staging copy (4.7085e8 KiB x 2.0 + 6.3850e8 KiB x 1.0) x 1024
    "stream_kernel": (9.766, "15876bd72a0de29e"),
    "gather_copy_kernel": (10.133, "9ef9851f1adbe75b"),
}


def source_hash(kernel: str) -> str:
    files = {"step_kernel": ["step.hip", "deliver.hpp"], "stream_kernel": ["stream.hip", "deliver.hpp"],
             "gather_copy_kernel": ["gather.hip"]}[kernel]
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_per_event(kernel: str):
    t = TRAFFIC.get(kernel)
    if t is None or source_hash(kernel) != t[1]:
        return None
    return t[0]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed_run(net, torch, steps, warmup, sim_steps, name):
    """`warmup` untimed, then `steps` timed calls of cortex_step(sim_steps),
    bracketed by synchronisations; HIP events on the caller's stream around
    each call (the library orders its own graph stream inside them)."""
    for w in range(warmup):
        net.step(sim_steps)
        torch.cuda.synchronize()
        log(f"[bench] {name}: warmup {w + 1}/{warmup} done")
    if net.query("PLAN") == 2:
        net.kernel_timing(True)   # launches time themselves from here on (sums cleared)
    stream = torch.cuda.current_stream()
    ev0, sp0 = net.query("EVENTS"), net.query("SPIKES")
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        net.step(sim_steps)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    events = net.query("EVENTS") - ev0
    spikes = net.query("SPIKES") - sp0
    sim_s = steps * sim_steps * net.spec.dt * 1e-3
    out = {"wall_s": wall, "events": events, "spikes": spikes, "sim_s": sim_s,
           "events_per_s": events / wall, "rtf": wall / sim_s,
           "firing_rate_hz": spikes / (net.N * sim_s), "gpu_ms_per_step": float(np.mean(kern_ms))}
    log(f"[bench] {name}: {steps} x {sim_steps} steps in {wall:.3f} s, {out['events_per_s']:.3e} events/s, "
        f"rate {out['firing_rate_hz']:.2f} Hz, rtf {out['rtf']:.3f}")
    return out


def roofline(net, run, steps, sim_steps, ktimes=None, model="delta"):
    """Roofline of the dominant kernel: its algorithmic bytes per launch over
    its average launch duration.  Resident plan: one persistent launch per
    call (event-timed calls).  Streamed plan: per window a delivery launch
    and, when the plan stages records, a staging copy; their mean durations
    over the timed region are measured by the launches themselves on the
    device clock (from a launch's start to the next launch's: its duration
    and the gap before the next).
    Algorithmic bytes: the delivery
    launch reads each delivered record once (record bytes per event); the
    copy reads it from the graph and writes it to the tile's run (twice
    that), and reads one 8-byte descriptor per (delivered spike, tile).
    The delivery launch also carries per-window state, reported beside it
    (state_bytes_per_launch, frac_with_state), not in `frac`: the ring rows
    that can hold sums, (R - W) x T cells per tile, loaded and written back,
    and every neuron's state (membrane, refractory count, cached Poisson
    counts and, for exp/alpha currents, the synaptic currents) loaded and
    stored."""
    streamed = net.query("PLAN") == 2
    W = net.query("STEPS_PER_SYNC")
    launches = -(-sim_steps // W) if streamed else 1
    B_rec = net.query("EDGE_BYTES")
    events_per_launch = run["events"] / steps / launches
    spikes_per_launch = run["spikes"] / steps / launches
    desc_bytes = spikes_per_launch * net.query("TILES") * 8
    out = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "launches_per_step": launches,
           "record_bytes": B_rec}
    if not streamed:
        kernel, alg, avg_s = "step_kernel", events_per_launch * B_rec, run["gpu_ms_per_step"] * 1e-3
    else:
        copy_ms, deliver_ms, nw = ktimes
        if nw == 0:
            raise RuntimeError("no per-kernel timing from the window graph")
        staged = net.query("STAGE_RECORDS") > 0
        per = {"stream_kernel": (events_per_launch * B_rec, deliver_ms * 1e-3)}
        if staged:
            per["gather_copy_kernel"] = (events_per_launch * 2 * B_rec + desc_bytes, copy_ms * 1e-3)
        kernel = max(per, key=lambda k: per[k][1])
        alg, avg_s = per[kernel]
        out["kernels"] = {}
        for k, (b, t) in per.items():
            tk = traffic_per_event(k)
            out["kernels"][k] = {"algorithmic_bytes_per_launch": b, "avg_launch_ms": t * 1e3,
                                 "achieved_GBps": b / t / 1e9, "frac": b / t / 1e9 / HBM_PEAK_GBS,
                                 "traffic": None if tk is None else tk * events_per_launch}
        ring = (net.query("TILES") * (net.query("RING_SLOTS") - W) * net.query("TILE_SIZE")
                * net.query("RING_BYTES") * 2)
        per_neuron = 16 + (4 if model in ("exp", "alpha") else 0) + (4 if model == "alpha" else 0)
        state = ring + net.query("NEURONS") * per_neuron * 2
        sk = out["kernels"]["stream_kernel"]
        sk["state_bytes_per_launch"] = state
        sk["frac_with_state"] = (sk["algorithmic_bytes_per_launch"] + state) / (sk["avg_launch_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        out["window_ms"] = run["gpu_ms_per_step"] / launches
        out["timed_windows"] = nw
    achieved = alg / avg_s / 1e9
    tpe = traffic_per_event(kernel)
    out.update({"achieved": achieved, "frac": achieved / HBM_PEAK_GBS,
                "traffic": None if tpe is None else tpe * events_per_launch, "kernel": kernel,
                "algorithmic_bytes_per_launch": alg, "avg_launch_ms": avg_s * 1e3,
                "descriptor_bytes_per_launch": desc_bytes})
    return out


def cpu_baseline(spec, rate_hz, seed, n_targets, n_steps):
    """The CPU oracle on a bounded sample of the same workload: every synapse
    into `n_targets` sampled neurons (weights as the network stores them),
    those neurons' updates, driven for `n_steps` by a replayed raster of all
    sources at the measured rate.  Events/s is a per-event rate, so it scales
    to the whole network."""
    import oracle
    import netspec
    N = spec.n_neurons
    sel = np.arange(0, N, N // n_targets)[:n_targets]
    t0 = time.perf_counter()
    o = oracle.OracleNet(spec, seed, sel=sel)
    t_build = time.perf_counter() - t0
    p = rate_hz * spec.dt * 1e-3
    steps, ids = netspec.sparse_raster(N, n_steps, p, seed=seed + 100)
    t0 = time.perf_counter()
    o.run_frozen(steps, ids, n_steps, record_x=False, record_v=False)
    t_run = time.perf_counter() - t0
    ev = o.events
    return {
        "value": ev / t_run,
        "unit": "synaptic events/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{len(sel)} of {N} targets with all {o.E} of their synapses, "
                   f"{n_steps} steps of a replayed {rate_hz:.2f} Hz raster of all sources; "
                   f"{ev:.3e} events in {t_run:.2f} s (graph build {t_build:.1f} s excluded)"),
    }


def choose_plan(cx, spec, seed, args):
    """The launch plan request of a timed network: the command line's, else
    a freshly measured one (--autotune), else the tuned table's entry for
    this network on this device, else the planner's default."""
    explicit = dict(tile_size=args.tile_size, block_size=args.block_size, wg_per_cu=args.wg_per_cu,
                    steps_per_sync=getattr(args, "steps_per_sync", 0))
    if getattr(args, "stage_records", 0):
        explicit["stage_records"] = args.stage_records
    if any(explicit.values()):
        return explicit, "command line"
    if args.autotune:
        best, _ = cx.autotune(spec, seed, steps=1000, warmup=100, cache=cx.TUNE_CACHE, log=log)
        return best, "autotuned in this run"
    req, entry = cx.lookup_plan(spec)
    if req is not None:
        same = entry.get("library") == cx._library_hash()
        return req, "tuned table" + ("" if same else " (tuned with another build of the library)")
    return {}, "planner default"


def brunel_112k(cx, torch, netspec, args):
    """The 112,500-neuron alpha-current net on the resident persistent plan."""
    spec = netspec.brunel_112k_alpha()
    req, plan_source = choose_plan(cx, spec, 2, argparse.Namespace(tile_size=0, block_size=0, wg_per_cu=0,
                                                                   autotune=args.autotune))
    log(f"[bench] brunel_112k: building, plan {req} ({plan_source})")
    t0 = time.perf_counter()
    net = cx.Network(spec, 2, **req)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    run = timed_run(net, torch, args.steps, args.warmup, SIM_STEPS_PER_BENCH_STEP, "brunel_112k")
    out = dict(run, neurons=net.N, synapses=net.E, graph_build_s=t_build, tiles=net.query("TILES"),
               tile_size=net.query("TILE_SIZE"), block_size=net.query("BLOCK_SIZE"),
               steps_per_sync=net.query("STEPS_PER_SYNC"),
               plan="streamed" if net.query("PLAN") == 2 else "resident", plan_request=req, plan_source=plan_source,
               roofline=roofline(net, run, args.steps, SIM_STEPS_PER_BENCH_STEP))
    net.close()
    return out


def _pack_instances(cx, netspec, spec, seed):
    """Greedy packing of the instances into as few co-resident launches as the
    device allows: each group is the longest prefix of the remaining
    instances whose resident plan fits."""
    groups, rest = [], list(spec.instances)
    while rest:
        k = len(rest)
        while True:
            sub = netspec.NetSpec(**{**spec.__dict__, "instances": rest[:k]})
            try:
                net = cx.Network(sub, seed, plan="resident")
                break
            except cx.CortexError as e:
                if e.status != cx.EUNSUPPORTED or k == 1:
                    raise
                k = max(1, (k * 3) // 4)
        groups.append((sub, net))
        rest = rest[k:]
    return groups


def batched_and_adjoint(cx, torch, seed, sim_steps):
    """Secondary figures on the batched workload (64 Brunel instances of
    log-uniform size 1,250-50,000, delta LIF, 1.5 ms delays): all instances in
    one launch per window (streamed plan, captured graph), the resident
    persistent plan packed into as few co-resident launches as fit, and the
    instances one after another; then the adjoint against its forward."""
    import netspec
    spec = netspec.batched_brunel()
    out = {"workload": "64 balanced delta-LIF instances, N log-uniform 1,250-50,000 (seeded), "
                       "in-degree 10% of each population, delay 1.5 ms, FP32",
           "sim_steps": sim_steps, "neurons": spec.n_neurons}

    def timed(nets):
        for net in nets:
            net.step(200)
        torch.cuda.synchronize()
        e0 = [net.query("EVENTS") for net in nets]
        t0 = time.perf_counter()
        for net in nets:
            net.step(sim_steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return sum(net.query("EVENTS") - e for net, e in zip(nets, e0)) / dt, dt

    log("[bench] batched: all 64 instances, streamed plan")
    net = cx.Network(spec, seed, plan="streamed")
    out["streamed"] = {"tiles": net.query("TILES"), "tile_size": net.query("TILE_SIZE"),
                       "steps_per_sync": net.query("STEPS_PER_SYNC"), "synapses": net.E}
    eps, dt = timed([net])
    out["streamed"].update(events_per_s=eps, wall_s=dt, launches_per_window=1)
    net.close()
    log(f"[bench] batched streamed: {eps:.3e} events/s")
    log("[bench] batched: resident plan, packed")
    groups = _pack_instances(cx, netspec, spec, seed)
    out["resident"] = {"launches": len(groups), "instances_per_launch": [len(g.instances) for g, _ in groups]}
    eps_r, dt_r = timed([net for _, net in groups])
    out["resident"].update(events_per_s=eps_r, wall_s=dt_r)
    for _, net in groups:
        net.close()
    del groups
    log(f"[bench] batched resident: {eps_r:.3e} events/s")
    ev_s, dt_s = 0, 0.0
    for b, inst in enumerate(spec.instances):
        one = netspec.NetSpec(**{**spec.__dict__, "instances": [inst]})
        g = cx.Network(one, seed, plan="resident")
        e, d = timed([g])
        ev_s += e * d
        dt_s += d
        g.close()
    out["sequential_events_per_s"] = ev_s / dt_s
    out["speedup_streamed_vs_sequential"] = eps / (ev_s / dt_s)
    out["speedup_resident_vs_sequential"] = eps_r / (ev_s / dt_s)
    log(f"[bench] one instance per launch: {ev_s / dt_s:.3e} events/s")
    out["adjoint"] = adjoint_all(cx, torch, seed, sim_steps)
    return out


def adjoint_all(cx, torch, seed, sim_steps):
    """The adjoint over all 64 instances: one checkpointed network per
    co-resident group (the adjoint runs on the resident plan), forward then
    the gradient of the voltage loss; the second backward call is timed
    (the first one also allocates its buffers)."""
    import netspec
    spec = netspec.batched_brunel()
    log("[bench] adjoint: forward with checkpoints, per group")
    groups = _pack_instances(cx, netspec, spec, seed)
    specs = [g for g, _ in groups]
    for _, net in groups:
        net.close()
    del groups
    adj = {"instances": 0, "neurons": 0, "synapses": 0, "forward_s": 0.0, "backward_s": 0.0,
           "backward_first_call_s": 0.0, "forward_events": 0, "loss": 0.0, "checkpoint_every_steps": 100,
           "groups": len(specs)}
    for k, sub in enumerate(specs):
        net = cx.Network(sub, seed, ckpt_every=100, adjoint_steps=sim_steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.step(sim_steps)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        vstar = torch.as_tensor(netspec.target_trace(net.N, sim_steps, 10.0, 20.0, seed=seed + 7 + k),
                                dtype=torch.float32, device="cuda")
        grad = torch.empty(net.E, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.backward(vstar, grad)
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, loss = net.backward(vstar, grad)
        torch.cuda.synchronize()
        t_bwd = time.perf_counter() - t0
        log(f"[bench] adjoint group {k}: {len(sub.instances)} instances, forward {t_fwd:.3f}s "
            f"backward {t_bwd:.3f}s (first call {t_first:.3f}s) loss {loss:.4g}")
        adj["instances"] += len(sub.instances)
        adj["neurons"] += net.N
        adj["synapses"] += net.E
        adj["forward_s"] += t_fwd
        adj["backward_s"] += t_bwd
        adj["backward_first_call_s"] += t_first
        adj["forward_events"] += net.query("EVENTS")
        adj["loss"] += loss
        net.close()
        del vstar, grad
        torch.cuda.empty_cache()
    adj["backward_over_forward"] = adj["backward_s"] / adj["forward_s"]
    return adj


def secondary_configs(cx, torch, netspec):
    """Events/s and real-time factor of the 77,169-neuron exp-current
    microcircuit stand-in (FP32, 1 s) and the 1,250-neuron delta-LIF net in
    the FP64 verification mode (100 ms)."""
    out = {}
    for name, spec, seed, steps in (("microcircuit_77k_fp32", netspec.microcircuit_77k(), 3, 10000),
                                    ("brunel_1250_fp64_verify", netspec.brunel_1250_fp64(), 1, 1000)):
        try:
            log(f"[bench] {name}: building")
            t0 = time.perf_counter()
            net = cx.Network(spec, seed)
            torch.cuda.synchronize()
            t_build = time.perf_counter() - t0
            run = timed_run(net, torch, 1, 1, steps, name)
            out[name] = dict(run, neurons=net.N, synapses=net.E, sim_steps=steps, graph_build_s=t_build)
            if spec.precision != "fp64":
                out[name].update(tiles=net.query("TILES"), tile_size=net.query("TILE_SIZE"),
                                 steps_per_sync=net.query("STEPS_PER_SYNC"),
                                 ring_slots=net.query("RING_SLOTS"), record_bytes=net.query("EDGE_BYTES"),
                                 roofline=roofline(net, run, 1, steps))
            net.close()
        except cx.CortexError as e:
            log(f"[bench] {name} failed: {e}")
            out[name] = {"error": str(e)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sim-steps", type=int, default=SIM_STEPS_PER_BENCH_STEP)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--scale", type=float, default=1.0,
                    help="neuron-count scale of the headline network (1.0 = 2,000,000; smaller only for trials)")
    ap.add_argument("--tile-size", type=int, default=0)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--steps-per-sync", type=int, default=0, help="exchange window W (0: tuned or planner)")
    ap.add_argument("--stage-records", type=int, default=0,
                    help="streamed plan: records per tile staged per window (0: automatic, -1: none)")
    ap.add_argument("--autotune", action="store_true",
                    help="measure the candidate launch plans of the timed networks first (minutes for the "
                         "two-million-neuron net) and use the fastest; without it the tuned table is used")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=("brunel_2m_bf16", "brunel_112k_alpha"), default="brunel_2m_bf16",
                    help="the timed network: the two-million-neuron bf16 net (streamed plan, the headline) or "
                         "the 112,500-neuron alpha net (resident persistent plan)")
    ap.add_argument("--cpu-targets", type=int, default=1000)
    ap.add_argument("--cpu-steps", type=int, default=10000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size before the timed region "
                         "(a known-size reference for HBM byte counters)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint over the 64 batched instances and print its figures "
                         "(a profiling aid; not the benchmark line)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import netspec
    import paper_2406_03762_amd as cx

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_all(cx, torch, 4, args.batched_steps)}), flush=True)
        return
    big = args.workload == "brunel_2m_bf16"
    spec = netspec.brunel_2m_bf16(scale_n=args.scale) if big else netspec.brunel_112k_alpha(scale_n=args.scale)
    seed = args.seed if big else 2
    req, plan_source = choose_plan(cx, spec, seed, args)
    log(f"[bench] building the {spec.n_neurons:,}-neuron {spec.model}-LIF network ({spec.weight_dtype} weights), "
        f"plan {req} ({plan_source})")
    t0 = time.perf_counter()
    net = cx.Network(spec, seed, **req)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    log(f"[bench] built: N={net.N} E={net.E} plan={'streamed' if net.query('PLAN') == 2 else 'resident'} "
        f"tiles={net.query('TILES')} T={net.query('TILE_SIZE')} R={net.query('RING_SLOTS')} "
        f"W={net.query('STEPS_PER_SYNC')} BS={net.query('BLOCK_SIZE')} rec={net.query('EDGE_BYTES')}B "
        f"staged={net.query('STAGE_RECORDS')} "
        f"device={net.query('DEVICE_BYTES') / 2**30:.1f} GiB in {t_build:.1f}s")

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {nb} bytes done")
        del src, dst

    streamed = net.query("PLAN") == 2
    run = timed_run(net, torch, args.steps, args.warmup, args.sim_steps, "headline")
    ktimes = net.kernel_times() if streamed else None
    roof = roofline(net, run, args.steps, args.sim_steps, ktimes, model=spec.model)
    rec = "16-bit record + bf16 weight" if spec.weight_dtype == "bf16" else "16-bit record + fp32 weight"
    cfg = {
        "workload": (f"balanced random net, {spec.model}-current LIF, {spec.n_neurons:,} neurons "
                     f"({spec.instances[0].pops[0].size:,} E / {spec.instances[0].pops[1].size:,} I), "
                     "in-degree 9,000 E + 2,250 I, "
                     f"{net.E:.3e} synapses ({rec}, FP32 accumulation), "
                     "weights Normal(J, (0.1J)^2), J = 0.1 mV, g = 5, delays uniform 0.5-3.0 ms, "
                     f"Poisson drive eta = 2, dt 0.1 ms; one step = {args.sim_steps} time steps "
                     f"({args.sim_steps * spec.dt:.0f} ms)"),
        "neurons": net.N, "synapses": net.E, "plan": "streamed" if net.query("PLAN") == 2 else "resident",
        "tiles": net.query("TILES"), "tile_size": net.query("TILE_SIZE"),
        "block_size": net.query("BLOCK_SIZE"), "steps_per_sync": net.query("STEPS_PER_SYNC"),
        "record_bytes": net.query("EDGE_BYTES"), "plan_request": req, "plan_source": plan_source,
    }
    net.close()
    del net
    torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(spec, run["firing_rate_hz"], seed, args.cpu_targets, args.cpu_steps)
        log(f"[bench] cpu baseline {cpu['value']:.3e} events/s")

    secondary = {}
    if not args.no_secondary:
        if big:
            secondary["brunel_112k_alpha_fp32"] = brunel_112k(cx, torch, netspec, args)
        torch.cuda.empty_cache()
        secondary.update(secondary_configs(cx, torch, netspec))
        torch.cuda.empty_cache()
    batched = None
    if not args.no_batched:
        try:
            batched = batched_and_adjoint(cx, torch, 4, args.batched_steps)
        except cx.CortexError as e:
            log(f"[bench] batched/adjoint leg failed: {e}")
            batched = {"error": str(e)}

    out = {
        "metric": "synaptic events/s (1 GPU)",
        "value": run["events_per_s"],
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": run["wall_s"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic (network and Poisson drive generated on device from Philox seeds)",
        "config": cfg,
        "rtf": run["rtf"],
        "firing_rate_hz": run["firing_rate_hz"],
        "events_per_step": run["events"] / args.steps,
        "roofline": roof,
        "cpu_baseline": cpu,
        "graph_build_s": t_build,
        "other_workloads": secondary,
        "batched": batched,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
