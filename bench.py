#!/usr/bin/env python3
"""Benchmark of the domain-decomposed sequential-update kMC hot path.

One step = one schedule sweep of the 1024x1024 periodic Ising lattice cut
into 32x32 domains (1024 domains, 4 colour phases of 256 domains each,
N_I = 1024 ticks per visit, Metropolis, T = 2.269, random start): every
domain visit, class bookkeeping, event selection, clock and the sweep
record.  value = site updates (ticks, null ticks included) per second, with
the sweep run as one dataflow launch (each visit starts once the visits of
its neighbours that precede it in the schedule are done; KMC_F_FLOW).

Extra measurements on the same line: the same workload as four phase
launches per sweep, the batched persistent form (4096 ragged replicas), the
backward score replay and fused score (1024 replicas of 64x64), the
roofline of the dominant kernel, the serial CPU oracle on a bounded sample
of the same workload (one core), and the oracle on the batch with one
process per host core.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Integer lane-operations per tick and per event that the method itself
# requires (see the design notes): one Philox4x32-10 call per tick (20
# 32x32->64 products = 40 multiplies, 40 XORs, 18 key additions) plus the
# slot and 64-bit threshold test; per event the class prefix, the member
# rank, five reclassifications and the count / rate-sum update.
OPS_PER_TICK = 102
OPS_PER_EVENT = 64
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: 32-bit integer lane-operations/s
ALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

# HBM bytes of one launch of each plain-form kernel: rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the
# counter reads for a 1 GiB device copy (profiles/copy_calibration_1GiB.md,
# profiles/k_flow_ising2d_L1024_tile32_plain.md,
# profiles/k_phase_ising2d_L1024_tile32_plain.md).  Valid only for the
# kernel source the counters were taken on; reported as null otherwise.
PLAIN_TRAFFIC = {
    "kernel_source_sha256": "ebae7473953b539bc3255dafa34b7fdd232a7132252188d1983b1111d503e395",
    "fetch_scale": 1048576.0 / 524308.0, "write_scale": 1048576.0 / 1048576.0,
    # k_flow: per sweep (the counter runs launch 40 sweeps per dispatch);
    # k_phase: per launch (one colour phase)
    "kib": {"k_flow<uint32_t,false,false>": (3400.95, 1218.22),
            "k_phase<uint32_t,false,false>": (940.51, 288.0)},
}
# algorithmic bytes per colour phase of the plain workload: each of the 256
# domains reads its 32x32 int8 tile and 4 x 32 halo sites and writes the
# tile back (a one-launch sweep covers four phases)
PLAIN_ALG_BYTES_PER_PHASE = 256 * (2 * 32 * 32 + 4 * 32)


def plain_traffic(kernel, sweeps_per_launch=1.0):
    import hashlib
    t = PLAIN_TRAFFIC
    if kernel not in t["kib"]:
        return None
    src = os.path.join(ROOT, "paper_1403_4674_amd", "csrc", "kmc_device.h")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["kernel_source_sha256"]:
            return None
    fetch, write = t["kib"][kernel]
    per = (fetch * t["fetch_scale"] + write * t["write_scale"]) * 1024.0
    # dataflow launches: the counters are kept per sweep
    return per * (sweeps_per_launch if kernel.startswith("k_flow") else 1.0)


def timed(fn, stream):
    import torch
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3


def plain(args, kmc, workloads, phased=False, steps=None):
    """The 1024^2 lattice, one sweep per step.  Default form: one dataflow
    launch per sweep (KMC_F_FLOW); phased: four colour-phase launches."""
    import torch
    steps = args.steps if steps is None else steps
    seed, descs, _ = workloads.single_1024(2.269)
    d = descs[0]
    lat = kmc.Lattice(descs, seed)
    stream = torch.cuda.current_stream()
    # without a graph, HIP events on the context stream bracket every launch
    # of the hot kernel inside the timed region (KMC_F_TIMING)
    flags = (kmc.F_GRAPH if args.graph else kmc.F_TIMING) | (0 if phased else kmc.F_FLOW)
    lat.run(args.warmup, 1, flags)
    torch.cuda.synchronize()
    if not args.graph:
        lat.timing()
    ev0 = lat.records()[0][-1]["events"] if args.warmup else 0
    sec = timed(lambda: lat.run(steps, 1, flags), stream)
    kernel_ms, launches = (lat.timing() if not args.graph
                           else (None, (4 if phased else 1) * steps))
    rec = lat.records()[0]
    events = int(rec[-1]["events"] - ev0)
    ticks = steps * d["L"] ** 2
    lat.close()
    return dict(sec=sec, ticks=ticks, events=events, launches=launches,
                kernel_sec=None if kernel_ms is None else kernel_ms / 1e3,
                desc=d, seed=seed, phased=phased,
                kernel="k_phase<uint32_t,false,false>" if phased else "k_flow<uint32_t,false,false>")


def parse_tiles(text):
    return {int(a): int(b) for a, b in (kv.split(":") for kv in text.split(","))} if text else None


def batched(args, kmc, workloads):
    import torch
    seed, descs, _ = workloads.batched_4096(tiles=parse_tiles(args.tiles))
    lat = kmc.Lattice(descs, seed)
    stream = torch.cuda.current_stream()
    lat.run(2, 1, kmc.F_PERSISTENT | args.flags)
    ev0 = int(lat.records()["events"][:, -1].sum())
    lat.timing()
    flags = kmc.F_PERSISTENT | kmc.F_TIMING | args.flags
    sec = timed(lambda: lat.run(args.batched_sweeps, args.batched_sweeps, flags), stream)
    kernel_ms, launches = lat.timing()
    events = int(lat.records()["events"][:, -1].sum()) - ev0
    ticks = args.batched_sweeps * sum(x["L"] ** 2 for x in descs)
    lat.close()
    return dict(sec=sec, ticks=ticks, events=events, replicas=len(descs),
                sweeps=args.batched_sweeps, kernel_sec=kernel_ms / 1e3, launches=launches)


def backward(args, kmc, workloads):
    import torch
    seed, descs, _ = workloads.differentiable_1024()
    n = args.grad_sweeps
    lat = kmc.Lattice(descs, seed)
    stream = torch.cuda.current_stream()
    lat.run(2, 1, kmc.F_PERSISTENT)
    fwd = timed(lambda: lat.run(n, 10, kmc.F_PERSISTENT | kmc.F_CHECKPOINT), stream)
    out = torch.empty((len(descs), n // 10, 2), dtype=torch.float64, device="cuda")
    bwd = timed(lambda: lat.score(n // 10, out), stream)
    # the fused form: the forward accumulates the score as it runs
    fused = timed(lambda: lat.run(n, 10, kmc.F_PERSISTENT | kmc.F_SCORE), stream)
    fused_bwd = timed(lambda: lat.score(n // 10, out), stream)
    ticks = n * sum(x["L"] ** 2 for x in descs)
    lat.close()
    return dict(fwd=fwd, bwd=bwd, ticks=ticks, overhead=(fwd + bwd) / fwd - 1.0,
                fused=fused + fused_bwd, fused_overhead=(fused + fused_bwd) / fwd - 1.0,
                replicas=len(descs), sweeps=n)


def parity_prefix(kmc, workloads):
    """Two sweeps of the benchmark workload checked against the oracle."""
    import numpy as np

    from oracle import kmco
    seed, descs, _ = workloads.single_1024(2.269)
    d = descs[0]
    lat = kmc.Lattice(descs, seed)
    lat.run(2, 1)
    g, s = lat.records()[0], lat.spins(0)
    lat.close()
    o = kmco.Replica(d["L"], d["tile"], J=d["J"], h=d["h"], T=d["T"],
                     steps_per_visit=d["steps_per_visit"], seed=seed, replica=0)
    r = o.run(2, 1)
    ok = all(np.array_equal(g[f], r[f]) for f in ("M", "B", "events", "steps"))
    ok = ok and np.array_equal(s, o.spins()) and np.allclose(g["t"], r["t"], rtol=1e-12)
    return bool(ok)


def cpu_baseline(budget_s):
    """The serial oracle, as it stands, on the benchmark workload: sweeps of
    the 1024^2 lattice until about budget_s seconds of one core are used."""
    from oracle import build as ob
    if not os.path.exists(ob.LIB):
        ob.build()
    from oracle import kmco
    from paper_1403_4674_amd import workloads
    seed, descs, _ = workloads.single_1024(2.269)
    d = descs[0]
    o = kmco.Replica(d["L"], d["tile"], J=d["J"], h=d["h"], T=d["T"],
                     steps_per_visit=d["steps_per_visit"], seed=seed, replica=0)
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.run(1, 1)
        n += 1
    sec = time.perf_counter() - t0
    return dict(value=n * d["L"] ** 2 / sec, unit="site-updates/s", cores=1,
                kind="oracle",
                sample=f"{n} sweeps of the 1024x1024 lattice (32x32 domains, N_I=1024, "
                       f"T=2.269) from the random start, serial C oracle, 1 thread, "
                       f"{sec:.1f} s")


def _cpu_batched_worker(job):
    """One host process of cpu_batched: its share of the batch (every n-th
    replica), one sweep of each in turn, until the budget is used."""
    wid, n_workers, budget_s = job
    from oracle import kmco
    from paper_1403_4674_amd import workloads
    seed, descs, _ = workloads.batched_4096()
    mine = []
    for rho in range(wid, len(descs), n_workers):
        d = descs[rho]
        mine.append((kmco.Replica(d["L"], d["tile"], J=d["J"], h=d["h"], T=d["T"],
                                  steps_per_visit=d["steps_per_visit"], seed=seed,
                                  replica=rho), d["L"] ** 2))
    ticks, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        for o, per_sweep in mine:
            o.run(1, 1)
            ticks += per_sweep
            if time.perf_counter() - t0 >= budget_s:
                break
    return ticks, time.perf_counter() - t0


def cpu_batched(budget_s, cores=None):
    """The serial oracle, as it stands, on the batched workload: one process
    per host core (at most 16), each sweeping its share of the 4096 replicas
    one sweep at a time for about budget_s seconds.  Aggregate
    site-updates/s over all processes."""
    import multiprocessing as mp
    from oracle import build as ob
    if not os.path.exists(ob.LIB):
        ob.build()
    n = cores or min(16, len(os.sched_getaffinity(0)))
    # spawned children start fresh interpreters that never touch the GPU
    with mp.get_context("spawn").Pool(n) as pool:
        res = pool.map(_cpu_batched_worker, [(w, n, budget_s) for w in range(n)])
    ticks = sum(r[0] for r in res)
    sec = max(r[1] for r in res)
    return dict(value=ticks / sec, unit="site-updates/s", cores=n, kind="oracle",
                sample=f"{n} processes, each sweeping every {n}-th replica of the 4096-replica "
                       f"batch (one sweep per replica in turn), serial C oracle, "
                       f"{sec:.1f} s")


def copy_probe(nbytes):
    """A plain device copy of known size (PMC byte-counter calibration)."""
    import torch
    x = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1)
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    return nbytes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--graph", action="store_true", help="replay sweeps from a hipGraph")
    ap.add_argument("--phased", action="store_true",
                    help="plain form as four phase launches per sweep (default: one "
                         "dataflow launch per sweep, KMC_F_FLOW)")
    ap.add_argument("--batched-sweeps", type=int, default=40)
    ap.add_argument("--grad-sweeps", type=int, default=200)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--mode", default="all",
                    choices=["all", "plain", "batched", "backward", "copy"],
                    help="all: the full line; the others run one part (for profiling)")
    ap.add_argument("--no-extras", action="store_true", help="same as --mode plain")
    ap.add_argument("--tiles", default="", help="batched workload tiles, e.g. 16:8,24:12")
    ap.add_argument("--flags", type=int, default=0, help="extra kmc_run_schedule flags (batched)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the method's replicas and domains are "
              "run on a single MI355X here; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.no_extras:
        args.mode = "plain"

    import torch

    from paper_1403_4674_amd import kmc, workloads
    torch.cuda.set_device(0)
    # every context of this run is bound to one dedicated stream; the timing
    # events are recorded on that same stream
    torch.cuda.set_stream(torch.cuda.Stream())
    kmc.use_torch_allocator()

    if args.mode == "copy":
        n = copy_probe(1 << 30)
        print(json.dumps({"copy_probe_bytes": n}), flush=True)
        return
    if args.mode == "batched":
        b = batched(args, kmc, workloads)
        print(json.dumps({"batched_site_updates_per_s": b["ticks"] / b["sec"], **b}),
              flush=True)
        return
    if args.mode == "backward":
        g = backward(args, kmc, workloads)
        print(json.dumps({"backward": g}), flush=True)
        return

    p = plain(args, kmc, workloads, phased=args.phased)
    value = p["ticks"] / p["sec"]
    # average duration of one phase-kernel launch: from the HIP events around
    # each launch; with --graph, the timed region over the launch count
    kernel_sec = p["kernel_sec"] if p["kernel_sec"] is not None else p["sec"]
    per_launch = kernel_sec / p["launches"]
    sweeps_per_launch = 0.25 if p["phased"] else args.steps / p["launches"]
    d = p["desc"]
    ops = OPS_PER_TICK * p["ticks"] + OPS_PER_EVENT * p["events"]
    achieved = ops / kernel_sec
    line = {
        "metric": "site-updates/s (plain vs batched replicas) + backward overhead at "
                  "bit-exact oracle match",
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": p["sec"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "ising2d_L1024_tile32_NI1024_T2.269_metropolis_plain",
                   "L": d["L"], "tile": d["tile"], "steps_per_visit": d["steps_per_visit"],
                   "T": d["T"], "seed": p["seed"], "graph": bool(args.graph),
                   "form": "phase_launches" if p["phased"]
                   else "dataflow_launches_of_up_to_64_sweeps"},
        "events_per_s": p["events"] / p["sec"],
        "roofline": {
            "bound": "alu",
            "kernel": p["kernel"],
            "achieved": achieved / 1e12,
            "peak": ALU_PEAK_LANE_OPS / 1e12,
            "unit": "Tlane-op/s",
            "frac": achieved / ALU_PEAK_LANE_OPS,
            "traffic": plain_traffic(p["kernel"], sweeps_per_launch),
            "traffic_unit": "B/launch",
            "algorithmic_bytes_per_launch": PLAIN_ALG_BYTES_PER_PHASE * 4 * sweeps_per_launch,
            "sweeps_per_launch": sweeps_per_launch,
            "per_launch_ms": per_launch * 1e3,
            "launches": p["launches"],
            "ops_per_launch": ops / p["launches"],
            "launch_timing": "hip_events_per_launch" if p["kernel_sec"] is not None
                             else "timed_region_over_launches",
        },
    }
    if args.mode == "all":
        if not args.phased:  # the four-launches-per-sweep form of the same workload
            q = plain(args, kmc, workloads, phased=True, steps=max(args.steps // 2, 1))
            line["plain_phased"] = {"value": q["ticks"] / q["sec"], "unit": "site-updates/s",
                                    "steps": max(args.steps // 2, 1),
                                    "kernel": q["kernel"],
                                    "per_launch_ms": q["kernel_sec"] * 1e3 / q["launches"],
                                    "flow_speedup": value / (q["ticks"] / q["sec"])}
        b = batched(args, kmc, workloads)
        g = backward(args, kmc, workloads)
        b_ops = OPS_PER_TICK * b["ticks"] + OPS_PER_EVENT * b["events"]
        line["batched"] = {"value": b["ticks"] / b["sec"], "unit": "site-updates/s",
                           "replicas": b["replicas"], "sweeps": b["sweeps"],
                           "vs_plain": (b["ticks"] / b["sec"]) / value,
                           "vs_plain_phased": (b["ticks"] / b["sec"])
                           / line.get("plain_phased", {"value": value})["value"],
                           "roofline": {"bound": "alu", "kernel": "k_persistent_multi<false>",
                                        "achieved": b_ops / b["kernel_sec"] / 1e12,
                                        "peak": ALU_PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                                        "frac": b_ops / b["kernel_sec"] / ALU_PEAK_LANE_OPS,
                                        "per_launch_ms": b["kernel_sec"] * 1e3 / b["launches"],
                                        "launches": b["launches"]}}
        line["backward"] = {"fwd_site_updates_per_s": g["ticks"] / g["fwd"],
                            "overhead": g["overhead"], "replicas": g["replicas"],
                            "sweeps": g["sweeps"],
                            "fwd_plus_bwd_vs_plain": (g["ticks"] / (g["fwd"] + g["bwd"]))
                            / value,
                            "fused_overhead": g["fused_overhead"],
                            "fused_site_updates_per_s": g["ticks"] / g["fused"],
                            "fused_vs_plain": (g["ticks"] / g["fused"]) / value,
                            "fused_vs_plain_phased": (g["ticks"] / g["fused"])
                            / line.get("plain_phased", {"value": value})["value"]}
        # the same comparison counted in replicas advanced by one sweep per
        # second (the plain workload is one replica of 1024^2); site-updates/s
        # above is the stricter unit, as the batches hold smaller replicas
        plain_rs = value / (1024 * 1024)
        line["replica_sweeps_per_s"] = {
            "plain": plain_rs,
            "batched": b["replicas"] * b["sweeps"] / b["sec"],
            "fused_score": g["replicas"] * g["sweeps"] / g["fused"],
        }
        line["replica_sweeps_per_s"]["batched_vs_plain"] = (
            line["replica_sweeps_per_s"]["batched"] / plain_rs)
        line["replica_sweeps_per_s"]["fused_score_vs_plain"] = (
            line["replica_sweeps_per_s"]["fused_score"] / plain_rs)
        line["parity_prefix_bit_exact"] = parity_prefix(kmc, workloads)
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        line["cpu_batched"] = cpu_batched(args.cpu_seconds * 2 / 3)
        line["batched"]["vs_cpu_batched"] = line["batched"]["value"] / line["cpu_batched"]["value"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
