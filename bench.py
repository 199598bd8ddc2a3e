#!/usr/bin/env python3
"""Benchmark of the domain-decomposed sequential-update kMC hot path.

One step = one schedule sweep of the 1024x1024 periodic Ising lattice cut
into 32x32 domains (1024 domains, 4 colour phases of 256 domains each,
N_I = 1024 ticks per visit, Metropolis, T = 2.269, random start): every
domain visit, class bookkeeping, event selection, clock and the sweep
record.  value = site updates (ticks, null ticks included) per second over
exactly --steps sweeps, with the sweeps run as dataflow launches (each visit
starts once the visits of its neighbours that precede it in the schedule are
done; KMC_F_FLOW).

Extra legs on the same line (none of them part of `value`):
* plain_steady: the same workload over three 64-sweep launches, the
  reference for every ratio against the plain kernel;
* plain_phased: the same workload as four phase launches per sweep;
* plain_T: the same lattice at T = 1.5 and T = 3.0;
* quench_4096: the 4096x4096 quench lattice (64x64 domains, N_I = 4096);
* small_NI: the 1024x1024 lattice at the paper's visit lengths
  N_I in {1, 2, 5, 10} (Sec. 3, Table 1), where the kernel streams its tiles
  and the HBM roofline is the one that applies;
* batched: the persistent form on 4096 ragged replicas;
* backward: the score replay and the fused score on 1024 replicas of 64x64;
* exact_5x5: exact propagation of the distribution over the 2^25
  configurations of a 5x5 lattice (the verification tool), against the HBM
  roofline;
* parity: the timed plain form and the batched multi-slot form against the
  oracle;
* cpu_baseline / cpu_batched: the serial CPU oracle on bounded samples.
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
# requires (not what the kernel spends): per tick 64 random bits (half a
# Philox4x32-10 call: 10 rounds of one 32x32->64 product (2 multiplies), 2
# XORs and the key additions, ~49 lane-ops) and the 64-bit test x < R (2);
# per event the clock's 53 random bits (another half call, 49), the class
# prefix and compare (~20), the member rank (~12), five reclassifications
# (~20) and the count / rate-sum update (~12).  The FP64 log and divide of
# the clock are not counted.
OPS_PER_TICK = 51
OPS_PER_EVENT = 64 + 49
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: 32-bit integer lane-operations/s
ALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
# MI355X HBM3E
HBM_PEAK = 8.0e12

# HBM bytes per sweep of the plain-form kernels on each plain workload, from
# rocprofv3 counters of the timed dispatch divided by its sweeps: reads are
# 32 n32 + 64 n64 + 128 n128 over the L2-to-memory read requests of each
# size (TCC_EA0_RDREQ_32B/64B/128B_sum; FETCH_SIZE counts a 128-byte request
# as 64 bytes on this GPU), writes are WRITE_SIZE (KiB).  On a 1 GiB device
# copy both give 1 GiB (profiles/copy_calibration_1GiB.md; the per-workload
# summaries in profiles/ name the commands).  Valid only for the kernel
# source the counters were taken on (sha256 of kmc_device.h); null otherwise.
TRAFFIC = {
    "kernel_source_sha256": "54005e3957125d9388ec63381d784c3c2ca20ef3715e67e9a16601db389259cc",
    # workload -> (read bytes, WRITE_SIZE KiB) per sweep
    "per_sweep": {
        # profiles/k_flow_ising2d_L1024_tile32_plain.md
        "ising2d_L1024_tile32_NI1024_T2.269_metropolis_plain": (52562560 / 64, 79994.09 / 64),
        # profiles/k_phase_ising2d_L1024_tile32_plain.md (four launches a sweep)
        "ising2d_L1024_tile32_NI1024_T2.269_metropolis_plain_phased": (4 * 506444.8, 4 * 296.0),
        # profiles/k_flow_ising2d_L1024_tile32_small_NI.md
        "ising2d_L1024_tile32_NI10_T2.269_metropolis_plain": (49081408 / 64, 81076.78 / 64),
        "ising2d_L1024_tile32_NI1_T2.269_metropolis_plain": (48429056 / 64, 79422.59 / 64),
        # profiles/k_flow_ising2d_L4096_tile64_quench.md
        "ising2d_L4096_tile64_NI4096_T1.5_metropolis_plain": (40673024 / 8, 138348.72 / 8),
    },
}


# The same for one tick of exact propagation on the 5 x 5 lattice (both
# passes; profiles/k_exact_tick_L5_one_domain.md), valid for the kernel
# source of kmc_exact.h it was taken on.
EXACT_TRAFFIC = {
    "kernel_source_sha256": "aae916c7b50745228cfb0b7812950f88fdb570f5100354d9bb24cdc4deb413b6",
    # (read bytes, WRITE_SIZE KiB) per tick: k_exact_hi + k_exact_lo
    "per_tick": (268875039 + 536952160, 314743.63 + 262144.08),
}


def kernel_source_sha(name="kmc_device.h"):
    import hashlib
    src = os.path.join(ROOT, "paper_1403_4674_amd", "csrc", name)
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_per_sweep(workload):
    """Calibrated HBM bytes per sweep measured for `workload`, or None."""
    t = TRAFFIC
    if workload not in t["per_sweep"] or t["kernel_source_sha256"] != kernel_source_sha():
        return None
    read, write_kib = t["per_sweep"][workload]
    return read + write_kib * 1024.0


def ticks_per_sweep(d):
    """Site updates (ticks, nulls included) of one sweep of a replica: N_I
    per domain visit."""
    bx = d["tile"]
    by = d.get("tile_rows") or bx
    visits = 2 if d.get("schedule") == 1 else 1
    return (d["L"] // bx) * (d["L"] // by) * (d.get("steps_per_visit") or bx * by) * visits


def alg_bytes_per_sweep(d):
    """Algorithmic HBM bytes of one sweep of a plain lattice: every visit
    reads its int8 tile and the 2 (Bx + By) halo sites and writes the tile
    back (tables, records and counters are negligible)."""
    L, bx = d["L"], d["tile"]
    by = d.get("tile_rows") or bx
    nd = (L // bx) * (L // by)
    return nd * (2 * bx * by + 2 * (bx + by))


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


def workload_name(d, form="flow"):
    T = f"{d['T']:g}"
    return (f"ising2d_L{d['L']}_tile{d['tile']}_NI{d['steps_per_visit']}_T{T}_metropolis_"
            f"{'plain' if form == 'flow' else 'plain_phased'}")


def plain(args, kmc, desc, seed, steps, warmup, phased=False, graph=False):
    """One plain lattice, one sweep per step, in the dataflow form (launches
    of up to 64 sweeps, KMC_F_FLOW) or as four colour-phase launches per
    sweep.  HIP events on the context stream bracket every launch of the hot
    kernel inside the timed region (KMC_F_TIMING), unless graph."""
    import torch
    d = desc
    lat = kmc.Lattice([d], seed)
    stream = torch.cuda.current_stream()
    flags = (kmc.F_GRAPH if graph else kmc.F_TIMING) | (0 if phased else kmc.F_FLOW)
    if warmup:
        lat.run(warmup, warmup, flags)
    torch.cuda.synchronize()
    if not graph:
        lat.timing()
    ev0 = int(lat.records()[0][-1]["events"]) if warmup else 0
    sec = timed(lambda: lat.run(steps, steps, flags), stream)
    kernel_ms, launches = (lat.timing() if not graph
                           else (None, (4 if phased else 1) * steps))
    events = int(lat.records()[0][-1]["events"]) - ev0
    ticks = steps * ticks_per_sweep(d)
    lat.close()
    kernel_sec = kernel_ms / 1e3 if kernel_ms is not None else sec
    kern = ("k_phase" if phased else "k_flow") + (
        "<uint64_t,false,false>" if d["tile"] > 32 else "<uint32_t,false,false>")
    return dict(sec=sec, ticks=ticks, events=events, launches=launches, steps=steps,
                kernel_sec=kernel_sec, timing="hip_events_per_launch" if kernel_ms is not None
                else "timed_region_over_launches", desc=d, seed=seed, phased=phased,
                kernel=kern, workload=workload_name(d, "phased" if phased else "flow"))


def roofline(p):
    """Both rooflines of a plain leg: the lane-op count of the method (ALU)
    and its algorithmic HBM bytes, over the summed duration of the timed
    launches of its kernel."""
    ops = OPS_PER_TICK * p["ticks"] + OPS_PER_EVENT * p["events"]
    alg = alg_bytes_per_sweep(p["desc"]) * p["steps"]
    tr = traffic_per_sweep(p["workload"])
    ks = p["kernel_sec"]
    return {
        "kernel": p["kernel"],
        "per_launch_ms": ks * 1e3 / p["launches"],
        "launches": p["launches"],
        "sweeps_per_launch": p["steps"] / p["launches"],
        "launch_timing": p["timing"],
        "alu": {"achieved": ops / ks / 1e12, "peak": ALU_PEAK_LANE_OPS / 1e12,
                "unit": "Tlane-op/s", "frac": ops / ks / ALU_PEAK_LANE_OPS,
                "ops_per_launch": ops / p["launches"]},
        "hbm": {"achieved": alg / ks / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": alg / ks / HBM_PEAK, "algorithmic_bytes_per_launch": alg / p["launches"],
                "traffic": None if tr is None else tr * p["steps"] / p["launches"],
                "traffic_unit": "B/launch"},
    }


def leg(p, extra=None):
    out = {"value": p["ticks"] / p["sec"], "unit": "site-updates/s", "steps": p["steps"],
           "ms_per_step": p["sec"] * 1e3 / p["steps"], "events_per_s": p["events"] / p["sec"],
           "workload": p["workload"], "roofline": roofline(p)}
    out.update(extra or {})
    return out


def exact(kmc, sweeps=2, L=5):
    """Exact propagation of the distribution over the 2^(L^2) configurations
    of an L x L lattice (one domain of L^2 sites, N_I = L^2 ticks a sweep)
    through `sweeps` sweeps (the verification tool, Sec. 3.1).  A tick is two
    launches over tiles of 2^14 states in LDS (k_exact_hi: the states that
    share bits 3..13; k_exact_lo: consecutive states), algorithmically a
    read of the 2^N doubles and a write of 2^N (every flip partner is an
    entry of the same vector); the two passes move 40 bytes a state (p twice,
    the partial sums written and read, p' written).  HBM roofline over the
    timed sweeps (the last tick of a sweep writes p itself)."""
    import torch
    N = L * L
    n = 1 << N
    d = dict(L=L, tile=L, T=2.5, h=0.1)
    p = torch.zeros(n, dtype=torch.float64, device="cuda")
    p[0] = 1.0
    work = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    kmc.kmc_exact_sweeps(d, p, work, 1)  # warm-up
    stream = torch.cuda.current_stream()
    sec = timed(lambda: kmc.kmc_exact_sweeps(d, p, work, sweeps), stream)
    total = float(p.sum().item())
    ticks = sweeps * N
    alg = ticks * 2 * 8 * n
    traffic = None
    if L == 5 and EXACT_TRAFFIC["kernel_source_sha256"] == kernel_source_sha("kmc_exact.h"):
        read, write_kib = EXACT_TRAFFIC["per_tick"]
        traffic = read + write_kib * 1024.0
    return {"value": ticks * n / sec, "unit": "state-ticks/s", "sweeps": sweeps,
            "states": n, "ticks": ticks, "ms_per_sweep": sec * 1e3 / sweeps,
            "probability_sum": total, "workload": f"exact_L{L}_one_domain_NI{N}",
            "roofline": {"bound": "hbm", "kernel": "k_exact_lo + k_exact_hi (one tick)",
                         "achieved": alg / sec / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": alg / sec / HBM_PEAK, "algorithmic_bytes_per_tick": 16 * n,
                         "traffic": traffic, "traffic_unit": "bytes_per_tick",
                         "timing": "timed_region_over_the_sweeps"}}


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
    ticks = args.batched_sweeps * sum(ticks_per_sweep(x) for x in descs)
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
    ticks = n * sum(ticks_per_sweep(x) for x in descs)
    lat.close()
    return dict(fwd=fwd, bwd=bwd, ticks=ticks, overhead=(fwd + bwd) / fwd - 1.0,
                fused=fused + fused_bwd, fused_overhead=(fused + fused_bwd) / fwd - 1.0,
                replicas=len(descs), sweeps=n)


def parity(kmc, workloads):
    """The timed forms against the oracle: two sweeps of the plain workload as
    one dataflow launch (KMC_F_FLOW), and three sweeps of the 4096-replica
    batch in the persistent form the batched leg times, with one replica of
    each lattice side compared."""
    import numpy as np

    from oracle import kmco

    def oracle(d, seed, rho):
        return kmco.Replica(d["L"], d["tile"], J=d["J"], h=d["h"], T=d["T"],
                            steps_per_visit=d["steps_per_visit"], seed=seed, replica=rho,
                            tile_rows=d.get("tile_rows", 0))

    def same(g, r, sg, so):
        ok = all(np.array_equal(g[f], r[f]) for f in ("sweep", "M", "B", "events", "steps"))
        return bool(ok and np.array_equal(sg, so) and np.allclose(g["t"], r["t"], rtol=1e-12))

    seed, descs, _ = workloads.single_1024(2.269)
    lat = kmc.Lattice(descs, seed)
    lat.run(2, 1, kmc.F_FLOW)
    o = oracle(descs[0], seed, 0)
    ok_plain = same(lat.records()[0], o.run(2, 1), lat.spins(0), o.spins())
    lat.close()
    seed, descs, _ = workloads.batched_4096()
    lat = kmc.Lattice(descs, seed)
    lat.run(3, 1, kmc.F_PERSISTENT)
    rec = lat.records()
    picks = sorted({d["L"]: rho for rho, d in enumerate(descs)}.values())
    ok_batch = True
    for rho in picks:
        o = oracle(descs[rho], seed, rho)
        ok_batch = ok_batch and same(rec[rho], o.run(3, 1), lat.spins(rho), o.spins())
    lat.close()
    return {"plain_flow_2_sweeps": ok_plain,
            f"batched_persistent_3_sweeps_{len(picks)}_replicas": ok_batch,
            "bit_exact": ok_plain and ok_batch}


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
                                  replica=rho, tile_rows=d.get("tile_rows", 0)),
                     ticks_per_sweep(d)))
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


# the paper's visit lengths (Sec. 3, Table 1)
SMALL_NI = (1, 2, 5, 10)


def small_ni_desc(d, ni):
    return dict(d, steps_per_visit=ni)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--graph", action="store_true", help="replay sweeps from a hipGraph")
    ap.add_argument("--phased", action="store_true",
                    help="plain form as four phase launches per sweep (default: dataflow "
                         "launches of up to 64 sweeps, KMC_F_FLOW)")
    ap.add_argument("--batched-sweeps", type=int, default=40)
    ap.add_argument("--grad-sweeps", type=int, default=200)
    ap.add_argument("--exact-sweeps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--mode", default="all",
                    choices=["all", "plain", "small_ni", "quench", "batched", "backward", "exact",
                             "copy"],
                    help="all: the full line; the others run one part (for profiling)")
    ap.add_argument("--ni", type=int, default=0,
                    help="--mode small_ni: run only this N_I (default: 1, 2, 5, 10)")
    ap.add_argument("--L", type=int, default=1024, choices=[1024, 4096],
                    help="--mode small_ni: the 1024^2 lattice or the 4096^2 one")
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

    seed2, d2s, _ = workloads.single_1024(2.269)
    d2 = d2s[0]
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
    if args.mode == "small_ni":
        if args.L == 4096:
            seed3, d3s, _ = workloads.quench_4096()
            d, sd = d3s[0], seed3
        else:
            d, sd = d2, seed2
        for ni in ([args.ni] if args.ni else SMALL_NI):
            p = plain(args, kmc, small_ni_desc(d, ni), sd, args.steps, args.warmup)
            print(json.dumps({f"NI{ni}": leg(p)}), flush=True)
        return
    if args.mode == "exact":
        print(json.dumps({"exact_5x5": exact(kmc, args.exact_sweeps)}), flush=True)
        return
    if args.mode == "quench":
        seed3, d3s, _ = workloads.quench_4096()
        p = plain(args, kmc, d3s[0], seed3, args.steps, args.warmup)
        print(json.dumps({"quench_4096": leg(p)}), flush=True)
        return

    p = plain(args, kmc, d2, seed2, args.steps, args.warmup, phased=args.phased,
              graph=args.graph)
    value = p["ticks"] / p["sec"]
    rl = roofline(p)
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
                   "L": d2["L"], "tile": d2["tile"], "steps_per_visit": d2["steps_per_visit"],
                   "T": d2["T"], "seed": seed2, "graph": bool(args.graph),
                   "form": "phase_launches" if p["phased"]
                   else "dataflow_launches_of_up_to_64_sweeps"},
        "events_per_s": p["events"] / p["sec"],
        # the dominant kernel is bound by its serial event chain (instruction
        # issue and latency): "alu", with the HBM fraction of its algorithmic
        # bytes beside it
        "roofline": {"bound": "alu", "kernel": p["kernel"],
                     "achieved": rl["alu"]["achieved"], "peak": rl["alu"]["peak"],
                     "unit": rl["alu"]["unit"], "frac": rl["alu"]["frac"],
                     "traffic": rl["hbm"]["traffic"], "traffic_unit": "B/launch",
                     "hbm_frac": rl["hbm"]["frac"], "hbm_achieved_GBps": rl["hbm"]["achieved"],
                     "algorithmic_bytes_per_launch": rl["hbm"]["algorithmic_bytes_per_launch"],
                     "ops_per_launch": rl["alu"]["ops_per_launch"],
                     "per_launch_ms": rl["per_launch_ms"], "launches": rl["launches"],
                     "sweeps_per_launch": rl["sweeps_per_launch"],
                     "launch_timing": rl["launch_timing"]},
    }
    if args.mode == "all":
        # the reference for every ratio: the same workload at its steady state
        # (three full 64-sweep launches after the warm-up)
        st = plain(args, kmc, d2, seed2, 3 * kmc.FLOW_MAX_SWEEPS, max(args.warmup, 40))
        plain_ref = st["ticks"] / st["sec"]
        line["plain_steady"] = leg(st)
        q = plain(args, kmc, d2, seed2, 64, 16, phased=True)
        line["plain_phased"] = leg(q, {"flow_speedup": plain_ref / (q["ticks"] / q["sec"])})
        line["plain_T"] = {}
        for T in (1.5, 3.0):
            sT, dTs, _ = workloads.single_1024(T)
            line["plain_T"][f"T{T:g}"] = leg(plain(args, kmc, dTs[0], sT, 128, 16))
        seed3, d3s, _ = workloads.quench_4096()
        line["quench_4096"] = leg(plain(args, kmc, d3s[0], seed3, 20, 4))
        line["small_NI"] = {}
        for ni in SMALL_NI:
            line["small_NI"][f"NI{ni}"] = leg(
                plain(args, kmc, small_ni_desc(d2, ni), seed2, 3 * kmc.FLOW_MAX_SWEEPS, 16))
        # the same visit length on the 4096^2 lattice: 16 times the visits per
        # sweep for the same dependency depth of the schedule
        line["small_NI"]["NI10_L4096"] = leg(
            plain(args, kmc, small_ni_desc(d3s[0], 10), seed3, 64, 16))
        line["exact_5x5"] = exact(kmc, args.exact_sweeps)
        b = batched(args, kmc, workloads)
        g = backward(args, kmc, workloads)
        b_ops = OPS_PER_TICK * b["ticks"] + OPS_PER_EVENT * b["events"]
        line["batched"] = {"value": b["ticks"] / b["sec"], "unit": "site-updates/s",
                           "replicas": b["replicas"], "sweeps": b["sweeps"],
                           "vs_plain_steady": (b["ticks"] / b["sec"]) / plain_ref,
                           "vs_plain_phased": (b["ticks"] / b["sec"]) / (q["ticks"] / q["sec"]),
                           "roofline": {"bound": "alu", "kernel": "k_persistent_multi<false>",
                                        "achieved": b_ops / b["kernel_sec"] / 1e12,
                                        "peak": ALU_PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                                        "frac": b_ops / b["kernel_sec"] / ALU_PEAK_LANE_OPS,
                                        "per_launch_ms": b["kernel_sec"] * 1e3 / b["launches"],
                                        "launches": b["launches"]}}
        line["backward"] = {"fwd_site_updates_per_s": g["ticks"] / g["fwd"],
                            "overhead": g["overhead"], "replicas": g["replicas"],
                            "sweeps": g["sweeps"],
                            "fwd_plus_bwd_vs_plain_steady": (g["ticks"] / (g["fwd"] + g["bwd"]))
                            / plain_ref,
                            "fused_overhead": g["fused_overhead"],
                            "fused_site_updates_per_s": g["ticks"] / g["fused"],
                            "fused_vs_plain_steady": (g["ticks"] / g["fused"]) / plain_ref,
                            "fused_vs_plain_phased": (g["ticks"] / g["fused"])
                            / (q["ticks"] / q["sec"])}
        # the same comparison counted in replicas advanced by one sweep per
        # second (the plain workload is one replica of 1024^2); site-updates/s
        # above is the stricter unit, as the batches hold smaller replicas
        plain_rs = plain_ref / (1024 * 1024)
        line["replica_sweeps_per_s"] = {
            "plain_steady": plain_rs,
            "batched": b["replicas"] * b["sweeps"] / b["sec"],
            "fused_score": g["replicas"] * g["sweeps"] / g["fused"],
        }
        line["parity"] = parity(kmc, workloads)
        line["parity_prefix_bit_exact"] = line["parity"]["bit_exact"]
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        line["cpu_batched"] = cpu_batched(args.cpu_seconds * 2 / 3)
        line["batched"]["vs_cpu_batched"] = line["batched"]["value"] / line["cpu_batched"]["value"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
