"""The benchmark's traffic and byte accounting (host side, no GPU)."""
import bench


def test_algorithmic_bytes_and_ticks():
    d = dict(L=1024, tile=32, steps_per_visit=1024)
    assert bench.alg_bytes_per_sweep(d) == 1024 * (2 * 1024 + 128) == 2228224
    assert bench.ticks_per_sweep(d) == 1024 * 1024
    assert bench.ticks_per_sweep(dict(L=64, tile=16, tile_rows=8, steps_per_visit=10)) == \
        32 * 10
    assert bench.alg_bytes_per_sweep(dict(L=64, tile=16, tile_rows=8)) == 32 * (2 * 128 + 48)


def test_traffic_is_tied_to_the_kernel_source(monkeypatch):
    name = "ising2d_L1024_tile32_NI1024_T2.269_metropolis_plain"
    assert bench.workload_name(dict(L=1024, tile=32, steps_per_visit=1024, T=2.269)) == name
    t = bench.traffic_per_sweep(name)
    if bench.TRAFFIC["kernel_source_sha256"] == bench.kernel_source_sha():
        assert t is not None and 0.5 < t / 2228224 < 1.3
    monkeypatch.setitem(bench.TRAFFIC, "kernel_source_sha256", "0" * 64)
    assert bench.traffic_per_sweep(name) is None
    assert bench.traffic_per_sweep("no such workload") is None


def test_exact_traffic_constant():
    # the two tick passes move 40 bytes a state against the 16 of one read
    # and one write of the 2^25 doubles; the constant names the source of
    # kmc_exact.h it was taken on (the benchmark reports null for another)
    read, write_kib = bench.EXACT_TRAFFIC["per_tick"]
    ratio = (read + write_kib * 1024.0) / (16 << 25)
    assert 2.0 < ratio < 3.0
    assert len(bench.EXACT_TRAFFIC["kernel_source_sha256"]) == 64
