"""The autotune cache's host logic: round trip, and every kind of damaged
file or entry read as a miss (the solver then tunes again)."""
import json

from paper_1210_7774_amd import tunecache as T


def test_roundtrip_and_keys(tmp_path):
    p = str(tmp_path / "tune.json")
    k1 = T.key("MI355X", "f32|rbgs|nu2,2", "diffusion2d-batch", [127, 255])
    k2 = T.key("MI355X", "f64|rbgs|nu2,2", "diffusion2d-batch", [127, 255])
    assert k1 != k2
    assert T.load(p, k1) is None  # no file
    c1 = {255: (64, False), 127: (32, True)}
    T.store(p, k1, c1)
    assert T.load(p, k1) == c1
    assert T.load(p, k2) is None
    c2 = {255: (8, False)}
    T.store(p, k2, c2)
    assert T.load(p, k1) == c1 and T.load(p, k2) == c2
    T.store(p, k1, {255: (16, False)})  # replaces the entry only
    assert T.load(p, k1) == {255: (16, False)} and T.load(p, k2) == c2
    assert [f.name for f in tmp_path.iterdir()] == ["tune.json"]  # no temporary left


def test_damaged_cache_is_a_miss(tmp_path):
    p = tmp_path / "tune.json"
    k = T.key("dev", "f64|rbgs|nu2,2", "poisson2d", [1023])
    for text in ("", "{", "[1, 2]", "null", json.dumps({k: [1, 2]}), json.dumps({k: {}}),
                 json.dumps({k: {"1023": [64]}}), json.dumps({k: {"1023": [1, False]}}),
                 json.dumps({k: {"1023": [512, False]}}), json.dumps({k: {"x": [64, False]}}),
                 json.dumps({k: {"1023": [64, 1]}}), json.dumps({k: {"0": [64, False]}})):
        p.write_text(text)
        assert T.load(str(p), k) is None, text
    # a damaged file is replaced by a good one on the next store
    p.write_text("{")
    T.store(str(p), k, {1023: (64, False)})
    assert T.load(str(p), k) == {1023: (64, False)}
