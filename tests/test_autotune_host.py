"""Host logic of the tile autotuner (timing stubbed, no GPU)."""
import json

from paper_1403_4674_amd import autotune


def test_valid_tiles():
    assert autotune.valid_tiles(16) == [8]
    assert autotune.valid_tiles(24) == [12]
    assert autotune.valid_tiles(48) == [8, 12, 24]
    assert autotune.valid_tiles(64) == [8, 16, 32]
    assert autotune.valid_tiles(128) == [8, 16, 32]
    for L in (16, 24, 32, 48, 64, 128, 1024):
        for B in autotune.valid_tiles(L, 64, 4):
            assert L % B == 0 and (L // B) % 2 == 0 and B % 4 == 0


def test_coordinate_descent_picks_fastest(tmp_path, monkeypatch):
    # stub rate: prefers tile 16 for L=64 and 12 for L=48
    want = {64: 16, 48: 12, 16: 8}  # reachable from either start

    def fake_rate(descs, seed, sweeps):
        return 1e9 - sum(abs(d["tile"] - want[d["L"]]) for d in descs)

    monkeypatch.setattr(autotune, "_rate", fake_rate)
    descs = [dict(L=64, tile=32, T=2.0), dict(L=48, tile=24, T=2.5), dict(L=16, tile=8, T=3)]
    path = tmp_path / "tiles.json"
    got = autotune.tune_batch("w", descs, 1, path=str(path))
    assert got == want
    table = json.loads(path.read_text())
    assert table["w"]["tiles"] == {"16": 8, "48": 12, "64": 16}
    assert autotune.tiles_for("w", str(path)) == want
    assert autotune.tiles_for("missing", str(path)) is None
