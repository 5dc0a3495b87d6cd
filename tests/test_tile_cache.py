"""Host logic of the tile autotuner's cache file (no GPU)."""
import json

import pytest

torch = pytest.importorskip("torch")
hh = pytest.importorskip("paper_1712_08740_amd.hh")


def test_key_names_precision_batch_and_levels():
    k = hh.tile_cache_key([(201, 401), (101, 201), (51, 101)], False, 1)
    assert k == "c128/rhs1/201x401,101x201,51x101"
    assert hh.tile_cache_key([(3, 5)], True, 32) == "c64/rhs32/3x5"


def test_cache_round_trip_keeps_other_entries(tmp_path):
    path = str(tmp_path / "t.json")
    assert hh.read_tile_cache(path) == {}
    hh.write_tile_cache(path, "a", [(0, 2), (1, 0)])
    hh.write_tile_cache(path, "b", [(1, 1)])
    data = hh.read_tile_cache(path)
    assert data == {"a": [[0, 2], [1, 0]], "b": [[1, 1]]}
    hh.write_tile_cache(path, "a", [(1, 2), (0, 0)])
    assert hh.read_tile_cache(path)["a"] == [[1, 2], [0, 0]]
    assert sorted(p.name for p in tmp_path.iterdir()) == ["t.json"]


def test_cache_rejects_a_file_that_is_not_a_mapping(tmp_path):
    path = tmp_path / "bad.json"
    path.write_text(json.dumps([1, 2]))
    with pytest.raises(ValueError):
        hh.read_tile_cache(str(path))


def test_tile_constants_match_the_header():
    import re
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "helmholtz.h")).read()
    consts = dict(re.findall(r"#define (HH_TILE_\w+) \(?(-?\d+)\)?", hdr))
    assert int(consts["HH_TILE_DEFAULT"]) == hh.HH_TILE_DEFAULT
    assert int(consts["HH_TILE_DOWN_COUNT"]) == hh.HH_TILE_DOWN_COUNT == len(hh.TILE_DOWN_SHAPES)
    assert int(consts["HH_TILE_UP_COUNT"]) == hh.HH_TILE_UP_COUNT == len(hh.TILE_UP_SHAPES)
