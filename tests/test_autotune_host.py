"""Host logic of the partition / visit-length autotuner (timing stubbed, no
GPU)."""
import json

from paper_1403_4674_amd import autotune, workloads


def test_valid_tiles_and_shapes():
    assert autotune.valid_tiles(16) == [8]
    assert autotune.valid_tiles(24) == [12]
    assert autotune.valid_tiles(48) == [8, 12, 24]
    assert autotune.valid_tiles(64) == [8, 16, 32]
    assert autotune.valid_tiles(128) == [8, 16, 32]
    for L in (16, 24, 32, 48, 64, 128, 1024):
        for bx, by in autotune.valid_shapes(L, 64, 4):
            for B in (bx, by):  # an even number of domains along each axis
                assert L % B == 0 and (L // B) % 2 == 0 and B % 4 == 0
            assert max(bx, by) <= 2 * min(bx, by)
    assert (8, 16) in autotune.valid_shapes(64) and (16, 8) in autotune.valid_shapes(64)
    assert (8, 32) not in autotune.valid_shapes(64)  # aspect 4


def test_visit_lengths():
    # 12 x 12 domains run 16 ticks per batch: 144 = 9 batches already
    assert autotune.visit_lengths(12, 12) == [32, 36, 48, 64, 72, 80, 144]
    # 24 x 24 run 64 per batch: 576 = 9 batches; 144 and 288 rounded both ways
    assert autotune.visit_lengths(24, 24) == [128, 144, 192, 256, 288, 320, 576]
    # the cap: never above nu_max * n_d
    assert max(autotune.visit_lengths(8, 16, nu_max=0.5)) <= 64
    assert autotune.visit_lengths(4, 4) == [4, 8, 16]


def test_ticks_per_sweep():
    assert autotune.ticks_per_sweep(dict(L=64, tile=16)) == 64 * 64
    assert autotune.ticks_per_sweep(dict(L=64, tile=16, tile_rows=8, steps_per_visit=100)) == \
        32 * 100
    assert autotune.ticks_per_sweep(dict(L=32, tile=8, schedule=1)) == 2 * 32 * 32


def test_coordinate_descent_picks_fastest(tmp_path, monkeypatch):
    # stub rate: prefers 16 x 8 domains with N_I = 64 for L = 64, 12 x 12 for
    # L = 48, and the longest visits otherwise
    want = {64: (16, 8, 64), 48: (12, 12, 144), 16: (8, 8, 64)}

    def fake_rate(descs, seed, sweeps):
        r = 1e9
        for d in descs:
            bx, by, ni = d["tile"], d.get("tile_rows") or d["tile"], d["steps_per_visit"]
            w = want[d["L"]]
            r -= 10 * (abs(bx - w[0]) + abs(by - w[1])) + abs(ni - w[2]) / 16
        return r

    monkeypatch.setattr(autotune, "_rate", fake_rate)
    descs = [dict(L=64, tile=32, T=2.0), dict(L=48, tile=24, T=2.5), dict(L=16, tile=8, T=3)]
    path = tmp_path / "tiles.json"
    got = autotune.tune_batch("w", descs, 1, path=str(path))
    assert got == want
    table = json.loads(path.read_text())
    assert table["w"]["shapes"] == {"16": [8, 8, 64], "48": [12, 12, 144], "64": [16, 8, 64]}
    assert autotune.shapes_for("w", str(path)) == want
    assert autotune.shapes_for("missing", str(path)) is None
    assert len(table["w"]["trials"]) > 6
    # the descriptors the tuned workload builds carry the shape and N_I
    d = autotune.apply(descs, got)
    assert d[0]["tile"] == 16 and d[0]["tile_rows"] == 8 and d[0]["steps_per_visit"] == 64
    assert d[1]["tile_rows"] == 0 and d[1]["steps_per_visit"] == 144


def test_workloads_take_tuned_shapes(monkeypatch, tmp_path):
    path = tmp_path / "t.json"
    path.write_text(json.dumps({
        "batched_4096": {"shapes": {"16": [8, 8, 48], "24": [12, 12, 144], "32": [16, 8, 128],
                                    "48": [12, 12, 144], "64": [16, 16, 256],
                                    "128": [16, 16, 256]}},
        "differentiable_1024": {"tiles": {"64": 8}}}))
    monkeypatch.setattr(workloads, "TUNED_TILES", str(path))
    _, descs, _ = workloads.batched_4096(n=200)
    for d in descs:
        if d["L"] == 32:
            assert (d["tile"], d["tile_rows"], d["steps_per_visit"]) == (16, 8, 128)
        if d["L"] == 16:
            assert (d["tile"], d["tile_rows"], d["steps_per_visit"]) == (8, 0, 48)
    # a table entry of the square-only format: N_I = B^2
    _, descs, _ = workloads.differentiable_1024(n=4)
    assert (descs[0]["tile"], descs[0]["steps_per_visit"]) == (8, 64)
