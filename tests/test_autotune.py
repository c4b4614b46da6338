"""Column-tile autotuner: selection and cache logic on the host; timing on the GPU."""
import numpy as np
import pytest

from paper_1507_05988_amd import autotune
from paper_1507_05988_amd import workloads as wl


def test_select_picks_fastest_measurable_tile():
    times = {(4, 8): 3.0, (4, 16): None, (8, 8): 1.5, (16, 8): 1.5, (32, 8): 2.0}
    best, table = autotune.select(list(times), lambda w, l: times[(w, l)])
    assert best == (8, 8)  # ties keep the earlier candidate
    assert "4x16" not in table and table["32x8"] == 2.0
    with pytest.raises(RuntimeError):
        autotune.select([(4, 8)], lambda w, l: None)


def test_fits_matches_the_workgroup_limit():
    assert autotune.fits(4, 8, 1024)        # 4 * 128 = 512
    assert not autotune.fits(8, 8, 1024)    # 1024 threads
    assert autotune.fits(32, 8, 128)
    assert not autotune.fits(32, 8, 129)


def test_shape_key_is_order_independent(tmp_path):
    a = [wl.config_small(nr=64, nt=256), wl.config_small(nr=40, nt=512)]
    assert autotune.shape_key(a, "fp32") == autotune.shape_key(a[::-1], "fp32")
    assert autotune.shape_key(a, "fp32") != autotune.shape_key(a, "fp64")
    path = tmp_path / "cache.json"
    autotune.store_cache(str(path), {"k": {"col_tile": 8, "col_rows": 16}})
    assert autotune.load_cache(str(path))["k"]["col_rows"] == 16
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}


@pytest.mark.gpu
def test_tuned_plan_runs_and_is_cached(tmp_path):
    import oracle
    from paper_1507_05988_amd import fcn
    insts = [wl.config_small(nr=64, nt=256), wl.config_small(nr=120, nt=512)]
    cache = str(tmp_path / "tiles.json")
    r = autotune.tune(insts, "fp64", steps=5, repeats=2, cache_path=cache)
    assert not r["cached"] and r["table"] and r["col_ms"] > 0
    assert autotune.tune(insts, "fp64", cache_path=cache)["cached"]
    plan = autotune.tuned_plan(insts, "fp64", cache_path=cache)
    assert plan.tiles()[:2] == (r["col_tile"], r["col_rows"])
    fields = [wl.gaussian_field(i) for i in insts]
    f = plan.pack(fields)
    plan.step(f, 3)
    plan.sync()
    for got, inst, a0 in zip(plan.unpack(f), insts, fields):
        want = oracle.propagate(inst, a0, 3)
        assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))
