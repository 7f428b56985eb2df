"""Host-side parts of the autotuner: graph signatures and the cache file."""
import numpy as np

from paper_2411_19901_amd import inputs, tune


def test_signature_separates_shapes():
    a = inputs.rmat(12)
    c = inputs.grid(64, 64, 0.05, 0.01, seed=1)
    assert tune.signature(a.row_ptr, "async", 8) == tune.signature(a.row_ptr.copy(), "async", 8)
    assert tune.signature(a.row_ptr, "async", 8) != tune.signature(c.row_ptr, "async", 8)
    assert tune.signature(a.row_ptr, "async", 8) != tune.signature(a.row_ptr, "det", 8)
    # decisions are kept per GPU architecture
    assert (tune.signature(a.row_ptr, "async", 8, arch="gfx950")
            != tune.signature(a.row_ptr, "async", 8, arch="gfx942"))
    assert tune.signature(np.zeros(1, np.int32), "det", 8)  # empty graph


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    assert tune.load_cache(path) == {}
    cache = {"x": {"lane_max_degree": 1024, "move_blocks_per_cu": 0, "ranked": False},
             "y": {"lane_max_degree": 256, "move_blocks_per_cu": 2, "ranked": True}}
    tune.save_cache(cache, path)
    assert tune.load_cache(path) == cache
