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


def test_shape_key_is_order_independent():
    a = [wl.config_small(nr=64, nt=256), wl.config_small(nr=40, nt=512)]
    assert autotune.shape_key(a, "fp32") == autotune.shape_key(a[::-1], "fp32")
    assert autotune.shape_key(a, "fp32") != autotune.shape_key(a, "fp64")


def test_tune_cache_text_round_trip(tmp_path):
    path = str(tmp_path / "tiles.txt")
    cache = {("fp32", 512): (8, 16, 101.5), ("fp32_cn64", 1024): (4, 8, 362.0)}
    autotune.store_cache(path, cache)
    assert autotune.load_cache(path) == cache
    assert autotune.load_cache(str(tmp_path / "missing.txt")) == {}
    with open(path) as fh:
        assert "fp32_cn64 col 1024 4 8 362.00" in fh.read()


def _create(lib, insts, precision, cache):
    import ctypes
    from paper_1507_05988_amd import fcn
    arr = (fcn.Instance * len(insts))(*[fcn.make_instance(i) for i in insts])
    o = fcn.Options(precision=fcn.PRECISIONS[precision], adaptive=0, max_phase=0.05, dz_min=1e-6, dz_max=1e-2,
                    use_graph=0, col_tile=0, col_rows=0, lanes=0, tune_cache=cache.encode() if cache else None)
    h = ctypes.c_void_p()
    rc = lib.fcn_plan_create(arr, len(insts), ctypes.byref(o), ctypes.byref(h))
    return rc, h


def test_library_reads_the_tune_cache(tmp_path):
    """The library (fcn_plan_create) takes each nr bucket's column tile from the cache file, for
    the plan's precision only; an unreadable or malformed cache is refused (no GPU call)."""
    import ctypes
    from paper_1507_05988_amd import fcn
    lib = fcn.load_library()
    path = str(tmp_path / "tiles.txt")
    autotune.store_cache(path, {("fp32", 200): (16, 16, 1.0), ("fp64", 200): (2, 8, 1.0)})
    insts = [wl.config_small(nr=200, nt=256)]
    for prec, want in (("fp32", (16, 16)), ("fp64", (2, 8)), ("fp32_storage", (4, 8))):
        rc, h = _create(lib, insts, prec, path)
        assert rc == fcn.FCN_OK
        w, l, e = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert lib.fcn_plan_tiles(h, ctypes.byref(w), ctypes.byref(l), ctypes.byref(e)) == 0
        assert (w.value, l.value) == want, prec
        lib.fcn_plan_destroy(h)
    assert _create(lib, insts, "fp32", str(tmp_path / "missing.txt"))[0] == fcn.FCN_E_ARG
    with open(path, "a") as fh:
        fh.write("fp32 col 300 oops\n")
    assert _create(lib, insts, "fp32", path)[0] == fcn.FCN_E_ARG


@pytest.mark.gpu
def test_tuned_plan_per_bucket_tiles_and_cache(tmp_path):
    """Per-nr tiles on a ragged batch: every bucket gets its own fastest tile, the cache answers
    the second call, the tuned plan matches the oracle, and each instance of it equals, bit for
    bit, the instance run alone with its bucket's tile given explicitly."""
    import oracle
    from paper_1507_05988_amd import fcn
    insts = [wl.config_small(nr=64, nt=256), wl.config_small(nr=300, nt=512), wl.config_small(nr=64, nt=512)]
    cache = str(tmp_path / "tiles.txt")
    r = autotune.tune(insts, "fp64", steps=5, repeats=2, cache_path=cache)
    assert not r["cached"] and set(r["per_nr"]) == {64, 300}
    assert all(v["table"] and v["us"] > 0 for v in r["per_nr"].values())
    assert autotune.tune(insts, "fp64", cache_path=cache)["cached"]
    plan = fcn.Plan(insts, precision="fp64", tune_cache=cache)
    fields = [wl.gaussian_field(i) for i in insts]
    f = plan.pack(fields)
    plan.step(f, 3)
    plan.sync()
    for got, inst, a0 in zip(plan.unpack(f), insts, fields):
        want = oracle.propagate(inst, a0, 3)
        assert np.max(np.abs(got - want)) < 1e-10 * np.max(np.abs(want))
        t = r["per_nr"][inst["nr"]]
        alone = fcn.Plan(inst, precision="fp64", col_tile=t["col_tile"], col_rows=t["col_rows"])
        g = alone.pack(a0)
        alone.step(g, 3)
        alone.sync()
        assert np.array_equal(alone.unpack(g)[0].view(np.uint64), got.view(np.uint64))
