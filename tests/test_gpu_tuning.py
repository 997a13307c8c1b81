"""The autotuner's persistent cache (lbm_autotune_cached) on the GPU."""
import json

import numpy as np
import pytest

from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def _lines(path):
    return [json.loads(x) for x in path.read_text().splitlines() if x.strip()]


@pytest.mark.parametrize("lattice,N,grid,storage", [("D2Q37", 4, (512, 64, 1), "fp32_dev"),
                                                    ("D2Q16-GH", 3, (300, 40, 1), "fp32_dev"),
                                                    ("D3Q39", 4, (256, 8, 6), "bf16_dev")])
def test_cache_miss_stores_and_hit_reuses_without_timing(tmp_path, lattice, N, grid, storage):
    """A miss tunes (as lbm_autotune does), leaves the state alone and writes one JSON line; a
    simulation of the same class then hits: same tile, the stored time, nothing re-timed.  A
    line whose tile description no longer matches the library is a miss, and is replaced."""
    lbm = need_gpu()
    path = tmp_path / "tune.jsonl"
    axis = 2 if lattice == "D3Q39" else 1
    kw = dict(storage=storage, stochastic_round=storage == "bf16_dev", sr_seed=1)
    with lbm.Sim(lattice, N, 0.9, grid, **kw) as s:
        s.set_shear_wave(1e-3, axis, rho_noise=1e-6, seed=3)
        before = s.save_state()
        t1, ms1, hit1 = s.autotune_cached(path, 2)
        assert not hit1 and 0 <= t1 < s.tile_count() and ms1 > 0
        assert np.array_equal(s.save_state(), before)
        entries = _lines(path)
        assert len(entries) == 1 and entries[0]["tile"] == t1
        key = entries[0]["key"]
        say(f"{lattice}: miss -> tile {t1}, {ms1:.4f} ms, key {key}")
        assert "gfx" in key and f"N{N}" in key
        # same class: ny nz rounded up to the same power of two
        g2 = (grid[0], grid[1] - 3, 1) if grid[2] == 1 else (grid[0], grid[1], grid[2] - 1)
        with lbm.Sim(lattice, N, 0.7, g2, **kw) as s2:
            t2, ms2, hit2 = s2.autotune_cached(path, 2)
            assert hit2 and t2 == t1 and ms2 == pytest.approx(ms1, rel=1e-5)
        # a stale description of the tile: miss, re-tuned, the line replaced
        entries[0]["shape"] = "stale"
        path.write_text(json.dumps(entries[0]) + "\n")
        t3, _, hit3 = s.autotune_cached(path, 2)
        assert not hit3
        again = _lines(path)
        assert len(again) == 1 and again[0]["key"] == key and again[0]["shape"] != "stale" and again[0]["tile"] == t3
        assert not list(tmp_path.glob("*.tmp.*"))


def test_cache_errors(tmp_path):
    lbm = need_gpu()
    with lbm.Sim("D2Q9", 2, 0.8, (64, 16, 1), storage="fp64") as s:
        with pytest.raises(lbm.LbmError) as e:
            s.autotune_cached(tmp_path / "no" / "dir" / "tune.jsonl", 1)
        assert e.value.code == lbm.LBM_EINVAL
        with pytest.raises(lbm.LbmError) as e:
            s.autotune_cached(tmp_path / "t.jsonl", 0)
        assert e.value.code == lbm.LBM_EINVAL
