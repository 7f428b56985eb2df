"""Host-side parts of the autotuner: graph signatures and the cache file."""
import numpy as np

from paper_2411_19901_amd import inputs, tune


def test_signature_separates_shapes():
    a = inputs.rmat(12)
    c = inputs.grid(64, 64, 0.05, 0.01, seed=1)
    assert tune.signature(a.row_ptr, "async", 8) == tune.signature(a.row_ptr.copy(), "async", 8)
    assert tune.signature(a.row_ptr, "async", 8) != tune.signature(c.row_ptr, "async", 8)
    assert tune.signature(a.row_ptr, "async", 8) != tune.signature(a.row_ptr, "det", 8)
    assert tune.signature(np.zeros(1, np.int32), "det", 8)  # empty graph


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert tune.load_cache(path) == {}
    cache = {"x": 1024, "y": 256}
    tune.save_cache(cache, path)
    assert tune.load_cache(path) == cache
