"""GPU vs oracle parity through the C-ABI (needs an MI355X).

Lattice states, per-domain and total event counts, step counts and the
integer observables must be bit-identical to the serial oracle; simulated
time (FP64 sums of -ln(u)/R) within 1e-12 relative.  Sizes: the full
16x16 workload, the 1024^2 and 4096^2 lattices at their real domain shapes
for a prefix of sweeps, and ragged batches of the batched workload.
"""
import numpy as np
import pytest

from paper_1403_4674_amd import kmc, workloads
from tests.gpu_helpers import (assert_records_equal, assert_replica_equal, assert_score_close,
                               oracle_for, oracle_score, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU test on a host without a GPU"
    return torch


def run_both(kmco, descs, seed, sweeps, record_every=1, flags=0, given=None, chunks=None):
    lat = kmc.Lattice(descs, seed, given_spins=given)
    for n in (chunks or [sweeps]):
        lat.run(n, record_every, flags)
    g_rec = lat.records()
    oras, o_recs = [], []
    for rho, d in enumerate(descs):
        o = oracle_for(kmco, d, seed, rho, None if given is None else given[rho])
        o_recs.append(o.run(sweeps, record_every) if not chunks else
                      np.concatenate([o.run(n, record_every) for n in chunks]))
        oras.append(o)
    return lat, g_rec, oras, o_recs


def test_single_16_full_run(torch_cuda, oracle_lib):
    cases, run = workloads.single_16()
    for seed, descs in cases:
        say(f"16x16 seed {seed} {run['sweeps']} sweeps")
        lat, g, oras, o = run_both(oracle_lib, descs, seed, run["sweeps"], run["record_every"])
        assert_replica_equal(lat, 0, oras[0], g[0], o[0], f"seed {seed}")
        lat.close()


@pytest.mark.parametrize("flags", [kmc.F_PERSISTENT, kmc.F_GRAPH])
def test_paths_are_bit_identical(torch_cuda, oracle_lib, flags):
    descs = [dict(L=16, tile=8, T=2.5, steps_per_visit=64),
             dict(L=24, tile=12, T=1.9, h=0.2),
             dict(L=32, tile=8, T=3.1, h=-0.1, steps_per_visit=10),
             dict(L=64, tile=16, T=2.2, h=0.05),
             dict(L=128, tile=64, T=2.6, steps_per_visit=700),
             dict(L=48, tile=24, T=1.6, h=0.4)]
    say(f"ragged batch, flags {flags}")
    a = kmc.Lattice(descs, 77)
    b = kmc.Lattice(descs, 77)
    a.run(37, 4)
    b.run(37, 4, flags)
    ra, rb = a.records(), b.records()
    for f in ("sweep", "M", "B", "events", "steps"):
        assert np.array_equal(ra[f], rb[f]), f
    np.testing.assert_allclose(ra["t"], rb["t"], rtol=1e-13)
    for rho in range(len(descs)):
        assert np.array_equal(a.spins(rho), b.spins(rho)), rho
    # and against the oracle, every replica
    for rho, d in enumerate(descs):
        o = oracle_for(oracle_lib, d, 77, rho)
        orec = o.run(37, 4)
        assert_replica_equal(b, rho, o, rb[rho], orec, f"replica {rho}")


@pytest.mark.parametrize("T", [1.5, 2.269, 3.0])
def test_single_1024_prefix(torch_cuda, oracle_lib, T):
    seed, descs, _ = workloads.single_1024(T)
    say(f"1024^2 T={T}, 3 sweeps")
    lat, g, oras, o = run_both(oracle_lib, descs, seed, 3, 1)
    assert_replica_equal(lat, 0, oras[0], g[0], o[0], f"1024 T={T}")


def oracle_in_chunks(o, sweeps, every, chunk, what):
    """Oracle records of a long run, in chunks of `chunk` sweeps (a multiple
    of `every`) with a progress line after each."""
    out = []
    for k in range(0, sweeps, chunk):
        out.append(o.run(min(chunk, sweeps - k), every))
        say(f"{what}: oracle at sweep {k + min(chunk, sweeps - k)}")
    return np.concatenate(out)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("T,sweeps", [(2.269, 200), (1.5, 20), (3.0, 20)])
def test_single_1024_timed_form(torch_cuda, oracle_lib, T, sweeps):
    """The 1024^2 workload in the form the benchmark times (dataflow launches
    of up to 64 sweeps, records every 10 sweeps as the workload defines)."""
    seed, descs, run = workloads.single_1024(T)
    every = run["record_every"]
    say(f"1024^2 T={T}, {sweeps} sweeps, dataflow form")
    lat = kmc.Lattice(descs, seed)
    lat.run(sweeps, every, kmc.F_FLOW)
    g = lat.records()
    o = oracle_for(oracle_lib, descs[0], seed, 0)
    orec = oracle_in_chunks(o, sweeps, every, 20, f"1024^2 T={T}")
    assert_replica_equal(lat, 0, o, g[0], orec, f"1024 T={T} flow")


@pytest.mark.timeout(900)
def test_quench_4096_timed_form(torch_cuda, oracle_lib):
    """The 4096^2 quench at its full shape (64 x 64 domains, N_I = 4096) in
    the dataflow form, 50 sweeps with records every 10."""
    seed, descs, run = workloads.quench_4096()
    sweeps, every = 50, run["record_every"]
    say(f"4096^2 T=1.5, {sweeps} sweeps at N_I=4096, dataflow form")
    lat = kmc.Lattice(descs, seed)
    lat.run(sweeps, every, kmc.F_FLOW)
    g = lat.records()
    o = oracle_for(oracle_lib, descs[0], seed, 0)
    orec = oracle_in_chunks(o, sweeps, every, 10, "4096^2 quench")
    assert_replica_equal(lat, 0, o, g[0], orec, "4096 quench flow")


def test_quench_4096_short_visits(torch_cuda, oracle_lib):
    seed, descs, _ = workloads.quench_4096()
    descs = [dict(descs[0], steps_per_visit=64)]
    say("4096^2 T=1.5, 4 sweeps at N_I=64")
    lat, g, oras, o = run_both(oracle_lib, descs, seed, 4, 2)
    assert_replica_equal(lat, 0, oras[0], g[0], o[0], "4096 N_I=64")


def test_batched_sample_persistent(torch_cuda, oracle_lib):
    seed, descs, _ = workloads.batched_4096(n=96)
    say("96 ragged replicas, persistent, 12 sweeps")
    lat, g, oras, o = run_both(oracle_lib, descs, seed, 12, 3, kmc.F_PERSISTENT)
    Ls = {d["L"] for d in descs}
    assert Ls == {16, 24, 32, 48, 64, 128}
    for rho in range(len(descs)):
        assert_replica_equal(lat, rho, oras[rho], g[rho], o[rho], f"replica {rho}")


@pytest.mark.parametrize("variant", ["palindrome", "barker", "given", "all_up"])
def test_schedule_rate_and_init_variants(torch_cuda, oracle_lib, variant):
    d = dict(L=32, tile=8, T=2.1, h=0.1, steps_per_visit=50)
    given = None
    if variant == "palindrome":
        d["schedule"] = kmc.SCHED_PALINDROME
    elif variant == "barker":
        d["rate_model"] = kmc.RATE_BARKER
    elif variant == "all_up":
        d["init"] = kmc.INIT_ALL_UP
    else:
        d["init"] = kmc.INIT_GIVEN
        rng = np.random.default_rng(8)
        given = [np.where(rng.random((32, 32)) < 0.3, 1, -1).astype(np.int8)]
    say(f"variant {variant}")
    lat, g, oras, o = run_both(oracle_lib, [d], 11, 25, 5, given=given)
    assert_replica_equal(lat, 0, oras[0], g[0], o[0], variant)


def test_resume_and_determinism(torch_cuda, oracle_lib):
    descs = [dict(L=32, tile=16, T=2.4, h=0.05), dict(L=16, tile=4, T=2.0)]
    say("resume: 7 + 13 sweeps vs 20")
    lat, g, oras, o = run_both(oracle_lib, descs, 5, 20, 1, chunks=[7, 13])
    for rho in range(2):
        assert_replica_equal(lat, rho, oras[rho], g[rho], o[rho], f"resume {rho}")
    b = kmc.Lattice(descs, 5)
    b.run(20, 1)
    rb = b.records()
    for f in ("M", "B", "events"):
        assert np.array_equal(rb[f], g[f])


MULTI_MIX = (
    # four-replica groups (one domain per colour), a partial group
    [dict(L=16, tile=8, T=2.3 + 0.1 * i, h=0.05 * i) for i in range(6)]
    + [dict(L=24, tile=12, T=2.0 + 0.2 * i, h=-0.1) for i in range(5)]
    + [dict(L=32, tile=16, T=3.0, h=0.2, rate_model=kmc.RATE_BARKER) for _ in range(3)]
    # one replica split over the slots of a wavefront (4 and 9 per colour)
    + [dict(L=32, tile=8, T=2.6, h=0.0), dict(L=48, tile=8, T=1.8, h=0.3),
       dict(L=64, tile=16, T=2.4, h=-0.2, schedule=kmc.SCHED_PALINDROME)]
    # over the slots of a workgroup (16 per colour)
    + [dict(L=128, tile=16, T=2.269, h=0.0), dict(L=64, tile=8, T=3.3, h=0.1)]
)


def test_multi_slot_form_is_bit_identical(torch_cuda, oracle_lib):
    descs = MULTI_MIX
    say(f"multi-slot form, {len(descs)} replicas")
    a = kmc.Lattice(descs, 123)
    b = kmc.Lattice(descs, 123)
    a.run(9, 3, kmc.F_PERSISTENT | kmc.F_NO_MULTI)
    b.run(9, 3, kmc.F_PERSISTENT | kmc.F_MULTI)
    ra, rb = a.records(), b.records()
    for f in ("sweep", "M", "B", "events", "steps"):
        assert np.array_equal(ra[f], rb[f]), f
    np.testing.assert_allclose(ra["t"], rb["t"], rtol=1e-13)
    for rho in range(len(descs)):
        assert np.array_equal(a.spins(rho), b.spins(rho)), rho
        sa, ca, ea = a.domain_state(rho)
        sb, cb, eb = b.domain_state(rho)
        assert np.array_equal(ea, eb)
        np.testing.assert_allclose(sa + ca, sb + cb, rtol=1e-13)
    for rho in (0, 6, 11, 14, 15, 16, 17, 18):
        o = oracle_for(oracle_lib, descs[rho], 123, rho)
        orec = o.run(9, 3)
        assert_replica_equal(b, rho, o, rb[rho], orec, f"multi replica {rho}")


def test_persistent_graph_replays(torch_cuda, oracle_lib):
    """Persistent chunks replayed from one captured graph, several runs with
    reads of the results (synchronising host work) between the replays; every
    replay is checked against eager launches."""
    descs = MULTI_MIX[:6] + [dict(L=32, tile=16, T=2.2), dict(L=64, tile=32, T=2.8, h=0.1)]
    say("persistent + graph, 3 runs x 4 replays")
    a = kmc.Lattice(descs, 31)
    b = kmc.Lattice(descs, 31)
    for run in range(3):
        a.run(8, 2, kmc.F_PERSISTENT)
        b.run(8, 2, kmc.F_PERSISTENT | kmc.F_GRAPH)
        ra, rb = a.records(), b.records()
        assert ra.shape == rb.shape == (len(descs), 4 * (run + 1))
        for f in ("sweep", "M", "B", "events", "steps"):
            assert np.array_equal(ra[f], rb[f]), (run, f)
        np.testing.assert_allclose(ra["t"], rb["t"], rtol=1e-13)
        for rho in range(len(descs)):
            assert np.array_equal(a.spins(rho), b.spins(rho)), (run, rho)
    b.run(5, 2, kmc.F_PERSISTENT | kmc.F_GRAPH)  # two replays and a remainder
    a.run(5, 2, kmc.F_PERSISTENT)
    assert np.array_equal(a.records(), b.records())
    o = oracle_for(oracle_lib, descs[6], 31, 6)
    orec = o.run(29, 2)
    assert_replica_equal(b, 6, o, b.records()[6], orec, "graph replica 6")


def test_timing_instrumentation_changes_nothing(torch_cuda):
    """KMC_F_TIMING only brackets the hot-kernel launches with events: one
    pair per phase launch (four per sweep here), results unchanged."""
    descs = [dict(L=64, tile=16, T=2.3, h=0.1)]
    say("timing flag")
    a = kmc.Lattice(descs, 9)
    b = kmc.Lattice(descs, 9)
    a.run(6, 2)
    b.run(6, 2, kmc.F_TIMING)
    ms, n = b.timing()
    assert n == 4 * 6 and ms > 0.0
    assert b.timing() == (0.0, 0)
    b.run(3, 3, kmc.F_PERSISTENT | kmc.F_TIMING)
    a.run(3, 3, kmc.F_PERSISTENT)
    ms, n = b.timing()
    assert n >= 1 and ms > 0.0
    assert np.array_equal(a.records(), b.records())
    assert np.array_equal(a.spins(0), b.spins(0))


FLOW_MIX = [dict(L=16, tile=8, T=2.5, steps_per_visit=64),
            dict(L=24, tile=12, T=1.9, h=0.2),
            dict(L=32, tile=8, T=3.1, h=-0.1, steps_per_visit=10),
            dict(L=64, tile=16, T=2.2, h=0.05, schedule=kmc.SCHED_PALINDROME),
            dict(L=128, tile=64, T=2.6, steps_per_visit=700),
            dict(L=48, tile=24, T=1.6, h=0.4),
            dict(L=8, tile=4, T=2.0, schedule=kmc.SCHED_PALINDROME)]


@pytest.mark.parametrize("graph", [False, True])
def test_one_launch_sweeps_are_bit_identical(torch_cuda, oracle_lib, graph):
    """KMC_F_FLOW (one launch per sweep, visits ordered by per-domain
    counters) against the phase launches and the oracle: both row widths,
    the palindrome, odd domains, 2x2 domains."""
    say(f"one-launch sweeps, graph={graph}")
    a = kmc.Lattice(FLOW_MIX, 44)
    b = kmc.Lattice(FLOW_MIX, 44)
    a.run(21, 3)
    b.run(21, 3, kmc.F_FLOW | (kmc.F_GRAPH if graph else 0))
    b.run(19, 1, kmc.F_FLOW | (kmc.F_GRAPH if graph else 0))  # a second run: counters restart
    a.run(19, 1)
    ra, rb = a.records(), b.records()
    assert np.array_equal(ra, rb)
    for rho in range(len(FLOW_MIX)):
        assert np.array_equal(a.spins(rho), b.spins(rho)), rho
        assert np.array_equal(a.domain_state(rho)[2], b.domain_state(rho)[2])
    for rho in (0, 3, 4, 6):
        o = oracle_for(oracle_lib, FLOW_MIX[rho], 44, rho)
        orec = np.concatenate([o.run(21, 3), o.run(19, 1)])
        assert_replica_equal(b, rho, o, rb[rho], orec, f"flow replica {rho}")


def test_dataflow_windows_of_many_sweeps(torch_cuda, oracle_lib):
    """Runs longer than one dataflow launch (kmc.FLOW_MAX_SWEEPS sweeps):
    sweeps of a window overlap, records every 7 sweeps straddle the window
    boundaries, and the result still equals the phase launches bit for bit
    (records, lattices, per-domain clocks); the fused score over the windows
    matches the phase form's within the score tolerance."""
    G = kmc.FLOW_MAX_SWEEPS
    descs = FLOW_MIX[:4] + [FLOW_MIX[6]]
    n1 = 2 * G + 22
    say(f"dataflow windows: {n1} sweeps, records every 7")
    a = kmc.Lattice(descs, 91)
    b = kmc.Lattice(descs, 91)
    a.run(n1, 7)
    b.run(n1, 7, kmc.F_FLOW | kmc.F_TIMING)
    ms, n = b.timing()
    assert n == 3 and ms > 0  # G + G + 22 sweeps
    assert np.array_equal(a.records(), b.records())
    for rho in range(len(descs)):
        assert np.array_equal(a.spins(rho), b.spins(rho)), rho
        for x, y in zip(a.domain_state(rho), b.domain_state(rho)):
            assert np.array_equal(x, y), rho
    o = oracle_for(oracle_lib, descs[2], 91, 2)
    assert_records_equal(b.records()[2], o.run(n1, 7), "oracle")
    n2 = G + 50
    say(f"dataflow windows: fused score, {n2} sweeps")
    a.run(n2, 10, kmc.F_SCORE)
    b.run(n2, 10, kmc.F_FLOW | kmc.F_SCORE)
    nb = -(-n2 // 10)
    sa, sb = a.score(nb), b.score(nb)
    assert np.array_equal(a.records(), b.records())
    for rho, d in enumerate(descs):
        _, _, sc, mag = oracle_score(oracle_lib, d, 91, rho, n2, 10, pre=n1)
        assert_score_close(sa[rho], sc, mag, f"phase form {rho}")
        assert_score_close(sb[rho], sc, mag, f"dataflow form {rho}")


@pytest.mark.parametrize("which", ["1024", "4096"])
def test_one_launch_sweeps_full_shapes(torch_cuda, oracle_lib, which):
    if which == "1024":
        seed, descs, _ = workloads.single_1024(2.269)
        sweeps = 3
    else:
        seed, descs, _ = workloads.quench_4096()
        descs = [dict(descs[0], steps_per_visit=256)]
        sweeps = 2
    say(f"one-launch sweeps on {which}^2, {sweeps} sweeps")
    lat, g, oras, o = run_both(oracle_lib, descs, seed, sweeps, 1, kmc.F_FLOW | kmc.F_TIMING)
    ms, n = lat.timing()
    assert n == -(-sweeps // kmc.FLOW_MAX_SWEEPS) and ms > 0  # sweeps share launches
    assert_replica_equal(lat, 0, oras[0], g[0], o[0], f"flow {which}")


def test_one_launch_score_replay(torch_cuda, oracle_lib):
    descs = FLOW_MIX[:4]
    say("one-launch sweeps: score replay")
    lat = kmc.Lattice(descs, 8)
    lat.run(12, 4, kmc.F_FLOW | kmc.F_CHECKPOINT)
    sc = lat.score(3)
    for rho, d in enumerate(descs):
        _, orec, osc, mag = oracle_score(oracle_lib, d, 8, rho, 12, 4)
        assert_records_equal(lat.records()[rho], orec, f"flow score replica {rho}")
        assert_score_close(sc[rho], osc, mag, f"flow score replica {rho}")


def test_one_launch_rejects_persistent(torch_cuda):
    lat = kmc.Lattice([dict(L=16, tile=8, T=2.0)], 1)
    with pytest.raises(kmc.KmcError) as e:
        lat.run(2, 1, kmc.F_FLOW | kmc.F_PERSISTENT)
    assert e.value.status == kmc.KMC_EINVAL


def test_dataflow_wait_timeout_is_reported(torch_cuda):
    """The failure path, forced from the host: with a bound of 0 polls every
    wait that finds a neighbour unfinished gives up at once, so the launch
    still ends, and the run is reported as failed (and stays so); a fresh
    context with the default bound runs clean.  A replay that times out is
    reported by kmc_backward_score; the forward run's records stay valid."""
    d = [dict(L=128, tile=16, T=2.3, steps_per_visit=256)]
    say("dataflow wait timeout")
    lat = kmc.Lattice(d, 3)
    lat.set_wait_limit(0)
    lat.run(40, 40, kmc.F_FLOW)
    for _ in range(2):
        with pytest.raises(kmc.KmcError) as e:
            lat.records()
        assert e.value.status == kmc.KMC_EDEVICE
    # the lattice and the domain state of a void run are refused as well
    for getter in (lambda: lat.spins(0), lambda: lat.domain_state(0),
                   lambda: lat.domain_clocks(0)):
        with pytest.raises(kmc.KmcError) as e:
            getter()
        assert e.value.status == kmc.KMC_EDEVICE
    lat.close()
    # and the score a void dataflow run accumulated (fused score)
    fz = kmc.Lattice(d, 3)
    fz.set_wait_limit(0)
    fz.run(40, 20, kmc.F_FLOW | kmc.F_SCORE)
    with pytest.raises(kmc.KmcError) as e:
        fz.score(2)
    assert e.value.status == kmc.KMC_EDEVICE
    fz.close()
    ok = kmc.Lattice(d, 3)
    ok.run(40, 40, kmc.F_FLOW)
    assert ok.records().shape == (1, 1)
    ok.run(40, 20, kmc.F_FLOW | kmc.F_CHECKPOINT)
    ok.set_wait_limit(0)
    with pytest.raises(kmc.KmcError) as e:
        ok.score(2)
    assert e.value.status == kmc.KMC_EDEVICE
    assert ok.records().shape == (1, 3)
    ok.close()
