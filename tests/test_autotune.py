"""Host logic of the tile autotuner: shape classes, table lookup, JSON round trip."""
import json

import pytest


def test_shape_class_buckets():
    from paper_1510_02148_amd import autotune
    assert autotune.shape_class(32 ** 3) == 15
    assert autotune.shape_class(96 ** 3) == 20           # 884736 = 2^19.75
    assert autotune.shape_class(64 * 64 * 64) == 18
    assert autotune.shape_class(1) == 0


def test_tiles_for_uses_class_entries():
    from paper_1510_02148_amd import autotune
    table = {"batch-f64:15": {"tile_cells": 256}, "batch-f64:20": {"tile_cells": 384},
             "single-f32:20": {"tile_cells": 1024}}
    got = autotune.tiles_for([(32, 32, 32), (96, 96, 96), (64, 64, 64)], table)
    assert got == [256, 384, None]
    assert autotune.tiles_for([(32, 32, 32)], table, precision="f32") == [None]
    assert autotune.tiles_for([(128, 128, 64)], table, precision="f32", kind="single") == [1024]
    assert autotune.tiles_for([(128, 128, 64)], table, precision="f64", kind="single") == [None]


def test_table_round_trip(tmp_path, monkeypatch):
    from paper_1510_02148_amd import autotune
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    path = str(tmp_path / "t.json")
    autotune.save_table({"batch-f64:17": {"tile_cells": 512, "ms": {"512": 1.0}}}, path)
    autotune.save_table({"single-f32:18": {"tile_cells": 384, "ms": {}}}, path)
    assert set(autotune.load_table(path)) == {"batch-f64:17", "single-f32:18"}
    with open(path) as f:
        assert list(json.load(f)) == ["gfx950"]


def test_committed_table_is_well_formed():
    from paper_1510_02148_amd import autotune
    with open(autotune.TABLE_PATH) as f:
        data = json.load(f)
    for arch_entries in data.values():
        for key, e in arch_entries.items():
            kp, cls = key.split(":")
            kind, prec = kp.split("-")
            assert kind in ("batch", "single") and prec in ("f64", "f32") and int(cls) >= 0
            assert 64 <= e["tile_cells"] <= 2048
            assert str(e["tile_cells"]) in e["ms"]
