"""Host logic of the autotuner's JSON cache (no GPU): the key names every
shape the kernel times depend on, and the file round-trips atomically."""
import json
import os

from paper_1508_02897_amd import autotune
from paper_1508_02897_amd import hddm as H


def test_key_separates_every_shape_parameter():
    base = dict(device_name="AMD Instinct MI355X", precision=H.HDDM_MIXED_C64, factor_format=0,
                nbx=32, nby=32, max_mx=176, max_my=176, block=True)
    k0 = autotune.cache_key(**base)
    assert k0 == "AMD Instinct MI355X|c64|format0|boxes32x32|box176x176|block"
    variants = [dict(device_name="other"), dict(precision=H.HDDM_PLAIN_C128),
                dict(factor_format=2), dict(nbx=16), dict(nby=16), dict(max_mx=168),
                dict(max_my=168), dict(block=False)]
    keys = {autotune.cache_key(**dict(base, **v)) for v in variants}
    assert len(keys) == len(variants) and k0 not in keys


def test_cache_round_trip_is_atomic(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load_cache(path) == {}
    assert autotune.load_cache(None) == {}
    entries = {"k1": {"choice": {"block_variant": 1, "factor_variant": 0},
                      "block_sweep_ms": {"three_mfma_lds_transpose": 11.9}}}
    autotune.save_cache(path, entries)
    assert autotune.load_cache(path) == entries
    entries["k2"] = {"choice": {"sweep_variant": 0, "sweep_threads": 0, "factor_variant": 0}}
    autotune.save_cache(path, entries)
    assert set(json.load(open(path))) == {"k1", "k2"}
    # no temporary files left beside the cache
    assert os.listdir(os.path.dirname(path)) == ["tune.json"]
