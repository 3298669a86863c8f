"""The autotuner's persistent cache (CPU only; the search itself needs a GPU)."""
import json

from paper_2107_13500_amd import binding as B
from paper_2107_13500_amd import tune


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(path) == {}
    tune.save_entry("gfx950|hip7|f64|a", {"tuning": {"chunk": 512, "seg": 64}, "ms": 1.5}, path)
    tune.save_entry("gfx950|hip7|f64|b", {"tuning": {"chunk": 256, "seg": 8}, "ms": 0.5}, path)
    data = tune.load_cache(path)
    assert data["gfx950|hip7|f64|a"]["tuning"]["seg"] == 64
    assert set(data) == {"gfx950|hip7|f64|a", "gfx950|hip7|f64|b"}


def test_corrupt_cache_reads_as_empty(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    assert tune.load_cache(str(p)) == {}
    p.write_text(json.dumps([1, 2]))
    assert tune.load_cache(str(p)) == {}


def test_shape_keys_distinguish_storage_and_batches():
    s1 = [B.PwShape(64, 64, 64, 0, 64, 66 * 64)]
    s2 = [B.PwShape(64, 64, 64, 0, 64, 66 * 64), B.PwShape(16, 20, 96, 0, 96, 22 * 96)]
    assert tune.shape_key(B.F64, s1) != tune.shape_key(B.F32, s1)
    assert tune.shape_key(B.F64, s1).startswith("f64|")
    assert "batch2" in tune.shape_key(B.F64, s2)
    assert tune.shape_key(B.F64, s2) == tune.shape_key(B.F64, list(s2))


def test_cache_path_env(monkeypatch, tmp_path):
    monkeypatch.setenv("PW_TUNE_CACHE", str(tmp_path / "x.json"))
    assert tune.cache_path() == str(tmp_path / "x.json")


def test_library_key_follows_the_built_library(tmp_path, monkeypatch):
    lib = tmp_path / "libx.so"
    lib.write_bytes(b"one build")
    monkeypatch.setattr(B, "LIBRARY", str(lib))
    k1 = tune.library_key()
    assert k1 == tune.library_key()
    lib.write_bytes(b"another build")
    assert tune.library_key() != k1
