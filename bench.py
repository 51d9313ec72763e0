"""Throughput of the LIF + delayed delivery step on one MI355X.

Workload: the 112,500-neuron balanced network with alpha-current LIF neurons,
in-degree 9,000 E + 2,250 I (1.27e9 synapses), delays uniform on 5..30 steps,
FP32, dt = 0.1 ms.  One benchmark step simulates 1 s (10,000 time steps) in
one persistent launch; inputs (graph, state) are resident in HBM before the
timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per synaptic event of the step kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (calibrated against a 1 GiB copy; profiles/step_kernel_brunel112k_alpha.md),
# valid only for the kernel source it was measured on.
TRAFFIC_BYTES_PER_EVENT = (3.0703e7 * 2.0 + 1.8482e6 * 1.0) * 1024 / 9.072019401e9
TRAFFIC_SOURCE_HASH = "4b542c1b14690f92"
SIM_STEPS_PER_BENCH_STEP = 10000      # 1 s of biological time at dt = 0.1 ms


def step_source_hash():
    import hashlib
    p = os.path.join(ROOT, "paper_2406_03762_amd", "csrc", "step.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(spec, rate_hz, seed, n_targets, n_steps):
    """The CPU oracle on a bounded sample of the same workload: every synapse
    into `n_targets` sampled neurons, those neurons' updates, driven for
    `n_steps` by a replayed raster of all sources at the measured rate."""
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


def _pack_instances(cx, netspec, spec, seed):
    """Greedy packing of the instances into as few co-resident launches as the
    device allows: each group is the longest prefix of the remaining
    instances whose plan fits (a plan that does not fit fails before the graph
    is generated)."""
    groups, rest = [], list(spec.instances)
    while rest:
        k = len(rest)
        while True:
            sub = netspec.NetSpec(**{**spec.__dict__, "instances": rest[:k]})
            try:
                net = cx.Network(sub, seed + len(groups))
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
    log-uniform size 1,250-50,000, delta LIF, 1.5 ms delays): the instances
    packed into as few persistent launches as fit the device vs the same
    instances run one after another, and the adjoint (backward) against its
    forward on the first packed group."""
    import netspec
    spec = netspec.batched_brunel()
    out = {"workload": "64 balanced delta-LIF instances, N log-uniform 1,250-50,000 (seeded), "
                       "in-degree 10% of each population, delay 1.5 ms, FP32",
           "sim_steps": sim_steps, "neurons": spec.n_neurons}
    log("[bench] batched: packing 64 instances into co-resident launches")
    groups = _pack_instances(cx, netspec, spec, seed)
    out["launches"] = len(groups)
    out["instances_per_launch"] = [len(g.instances) for g, _ in groups]
    out["synapses"] = int(sum(net.E for _, net in groups))
    log(f"[bench] batched: {len(groups)} launches of {out['instances_per_launch']} instances")
    for i, (_, net) in enumerate(groups):
        log(f"[bench] batched launch {i}: tiles={net.query('TILES')} T={net.query('TILE_SIZE')} "
            f"BS={net.query('BLOCK_SIZE')} W={net.query('STEPS_PER_SYNC')} ring={net.query('RING_BYTES')}B")
    for _, net in groups:
        net.step(200)
    torch.cuda.synchronize()
    e0 = [net.query("EVENTS") for _, net in groups]
    t0 = time.perf_counter()
    for _, net in groups:
        net.step(sim_steps)
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t0
    ev_b = sum(net.query("EVENTS") - e for (_, net), e in zip(groups, e0))
    log(f"[bench] batched: {ev_b / dt_b:.3e} events/s")
    adj_spec = groups[0][0]
    for _, net in groups:
        net.close()
    del groups
    ev_s, dt_s = 0, 0.0
    for b, inst in enumerate(spec.instances):
        one = netspec.NetSpec(**{**spec.__dict__, "instances": [inst]})
        g = cx.Network(one, seed + 1000 + b)
        g.step(200)
        torch.cuda.synchronize()
        e0 = g.query("EVENTS")
        t0 = time.perf_counter()
        g.step(sim_steps)
        torch.cuda.synchronize()
        dt_s += time.perf_counter() - t0
        ev_s += g.query("EVENTS") - e0
        g.close()
    log(f"[bench] one instance per launch: {ev_s / dt_s:.3e} events/s")
    out.update(events_per_s=ev_b / dt_b, sequential_events_per_s=ev_s / dt_s,
               speedup=(ev_b / dt_b) / (ev_s / dt_s), batched_wall_s=dt_b, sequential_wall_s=dt_s)
    # adjoint: checkpointed forward, then the gradient of the voltage loss
    log("[bench] adjoint: forward with checkpoints")
    net = cx.Network(adj_spec, seed, ckpt_every=100, adjoint_steps=sim_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.step(sim_steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    ev_f = net.query("EVENTS")
    vstar = torch.empty((sim_steps, net.N), dtype=torch.float32, device="cuda").uniform_(10.0, 20.0)
    grad = torch.empty(net.E, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, loss = net.backward(vstar, grad)
    torch.cuda.synchronize()
    t_bwd = time.perf_counter() - t0
    log(f"[bench] adjoint: forward {t_fwd:.3f}s backward {t_bwd:.3f}s loss {loss:.4g}")
    out["adjoint"] = {"instances": len(adj_spec.instances), "neurons": net.N, "synapses": net.E,
                      "forward_s": t_fwd, "backward_s": t_bwd, "backward_over_forward": t_bwd / t_fwd,
                      "forward_events": ev_f, "loss": loss, "checkpoint_every_steps": 100}
    net.close()
    return out


def secondary_configs(cx, torch, netspec):
    """Events/s and real-time factor of the other single-GPU workloads: the
    77,169-neuron exp-current microcircuit stand-in (FP32, 1 s) and the
    1,250-neuron delta-LIF net in the FP64 verification mode (100 ms)."""
    out = {}
    for name, spec, seed, steps in (("microcircuit_77k_fp32", netspec.microcircuit_77k(), 3, 10000),
                                    ("brunel_1250_fp64_verify", netspec.brunel_1250_fp64(), 1, 1000)):
        try:
            log(f"[bench] {name}: building")
            t0 = time.perf_counter()
            net = cx.Network(spec, seed)
            torch.cuda.synchronize()
            t_build = time.perf_counter() - t0
            net.step(min(1000, steps))
            torch.cuda.synchronize()
            e0, s0 = net.query("EVENTS"), net.query("SPIKES")
            t0 = time.perf_counter()
            net.step(steps)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            ev, sp = net.query("EVENTS") - e0, net.query("SPIKES") - s0
            sim_s = steps * spec.dt * 1e-3
            out[name] = {"neurons": net.N, "synapses": net.E, "sim_steps": steps,
                         "events_per_s": ev / wall, "rtf": wall / sim_s,
                         "firing_rate_hz": sp / (net.N * sim_s), "graph_build_s": t_build}
            if spec.precision != "fp64":
                out[name].update(tiles=net.query("TILES"), tile_size=net.query("TILE_SIZE"),
                                 steps_per_sync=net.query("STEPS_PER_SYNC"),
                                 ring_slots=net.query("RING_SLOTS"), record_bytes=net.query("EDGE_BYTES"))
            log(f"[bench] {name}: {ev / wall:.3e} events/s, rtf {wall / sim_s:.3f}")
            net.close()
        except cx.CortexError as e:
            log(f"[bench] {name} failed: {e}")
            out[name] = {"error": str(e)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sim-steps", type=int, default=SIM_STEPS_PER_BENCH_STEP)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--tile-size", type=int, default=0)
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--steps-per-sync", type=int, default=0,
                    help="time steps per spike exchange (0 = the planner's choice)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-targets", type=int, default=6000)
    ap.add_argument("--cpu-steps", type=int, default=12000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size before the timed region "
                         "(a known-size reference for HBM byte counters)")
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
    spec = netspec.brunel_112k_alpha()
    log("[bench] building the 112,500-neuron alpha-LIF network")
    t0 = time.perf_counter()
    net = cx.Network(spec, args.seed, tile_size=args.tile_size, block_size=args.block_size,
                     steps_per_sync=args.steps_per_sync)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    E = net.E
    B_rec = net.query("EDGE_BYTES")
    n_tiles = net.query("TILES")
    tile_size = net.query("TILE_SIZE")
    block_size = net.query("BLOCK_SIZE")
    log(f"[bench] built: N={net.N} E={E} tiles={n_tiles} T={net.query('TILE_SIZE')} "
        f"R={net.query('RING_SLOTS')} W={net.query('STEPS_PER_SYNC')} BS={net.query('BLOCK_SIZE')} rec={B_rec}B "
        f"in {t_build:.1f}s")

    if args.copy_calibration_mib > 0:
        nb = args.copy_calibration_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {nb} bytes done")
        del src, dst

    for w in range(args.warmup):
        net.step(args.sim_steps)
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")

    stream = torch.cuda.current_stream()
    ev0 = net.query("EVENTS")
    sp0 = net.query("SPIKES")
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        net.step(args.sim_steps)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev1 = net.query("EVENTS")
    sp1 = net.query("SPIKES")
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    events = ev1 - ev0
    spikes = sp1 - sp0
    sim_s = args.steps * args.sim_steps * spec.dt * 1e-3
    rate_hz = spikes / (net.N * sim_s)
    ev_per_s = events / wall
    avg_kernel_s = float(np.mean(kern_ms)) * 1e-3
    bytes_per_launch = events / args.steps * B_rec
    achieved = bytes_per_launch / avg_kernel_s / 1e9
    offset_bytes = spikes / args.steps * n_tiles * 8
    log(f"[bench] timed {args.steps} x {args.sim_steps} steps: wall {wall:.3f}s, "
        f"kernel avg {avg_kernel_s * 1e3:.2f} ms, rate {rate_hz:.2f} Hz, {ev_per_s:.3e} events/s")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(spec, rate_hz, args.seed, args.cpu_targets, args.cpu_steps)
        log(f"[bench] cpu baseline {cpu['value']:.3e} events/s")

    net.close()
    del net
    secondary = None
    if not args.no_secondary:
        secondary = secondary_configs(cx, torch, netspec)
    batched = None
    if not args.no_batched:
        try:
            batched = batched_and_adjoint(cx, torch, 4, args.batched_steps)
        except cx.CortexError as e:
            log(f"[bench] batched/adjoint leg failed: {e}")
            batched = {"error": str(e)}

    out = {
        "metric": "synaptic events/s (1 GPU)",
        "value": ev_per_s,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic (network and Poisson drive generated on device from Philox seeds)",
        "config": {
            "workload": "balanced random net, alpha-current LIF, 112,500 neurons (90,000 E / 22,500 I), "
                        "in-degree 9,000 E + 2,250 I, 1.27e9 synapses, weights Normal(J, (0.1J)^2) "
                        "as PSP peaks, delays uniform 0.5-3.0 ms, dt 0.1 ms, FP32; "
                        f"one step = {args.sim_steps} time steps ({args.sim_steps * spec.dt:.0f} ms)",
            "neurons": spec.n_neurons,
            "synapses": E,
            "tiles": n_tiles,
            "tile_size": tile_size,
            "block_size": block_size,
            "record_bytes": B_rec,
        },
        "rtf": wall / sim_s,
        "firing_rate_hz": rate_hz,
        "events_per_launch": events / args.steps,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (TRAFFIC_BYTES_PER_EVENT * events / args.steps
                        if step_source_hash() == TRAFFIC_SOURCE_HASH else None),
            "kernel": "step_kernel",
            "algorithmic_bytes_per_launch": bytes_per_launch,
            "offset_bytes_per_launch": offset_bytes,
            "avg_launch_ms": avg_kernel_s * 1e3,
        },
        "cpu_baseline": cpu,
        "graph_build_s": t_build,
        "other_workloads": secondary,
        "batched": batched,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
