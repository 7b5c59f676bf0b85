"""Host logic of the NS tile autotuner: cache keys, masks from a cache, and
the bucket list (no GPU)."""
import json

import numpy as np
import pytest


def test_buckets_and_bits(box64):
    from paper_2104_08245_amd import autotune as at
    n = 6 * np.diff(box64.K.row_ptr)
    assert at.buckets_of(box64) == sorted(set(((n + 63) // 64 * 64).tolist()))
    assert at.bit_of(64) == 1 and at.bit_of(192) == 4 and at.bit_of(1536) == 1 << 23


def test_mask_from_cache(tmp_path, box64):
    from paper_2104_08245_amd import autotune as at, _lib as L
    d = L.default_opts("fp16").ns_small_tile_mask
    bk = at.buckets_of(box64)
    assert bk == [192, 256]
    # no cache: the default, nothing tuned
    assert at.mask_for(box64, "fp16", True, cache=str(tmp_path / "none.json")) == (d, [], bk)
    table = {at.key("fp16", True, 192): 128, at.key("fp16", True, 256): 64,
             at.key("fp16", False, 256): 128, at.key("bf16", True, 192): 64,
             at.key("fp16", True, 1024): 64}          # a bucket this system lacks
    f = tmp_path / "t.json"
    f.write_text(json.dumps(table))
    mask, tuned, _ = at.mask_for(box64, "fp16", True, cache=str(f))
    assert tuned == [192, 256]
    assert mask == (d & ~at.bit_of(192)) | at.bit_of(256)
    assert not mask & at.bit_of(1024)
    # other variant and precision read their own keys
    assert at.mask_for(box64, "fp16", False, cache=str(f))[:2] == (d & ~at.bit_of(256), [256])
    assert at.mask_for(box64, "bf16", True, cache=str(f))[:2] == (d | at.bit_of(192), [192])
    f.write_text(json.dumps({at.key("fp16", True, 192): 96}))
    with pytest.raises(ValueError):
        at.mask_for(box64, "fp16", True, cache=str(f))


def test_committed_cache_is_well_formed():
    from paper_2104_08245_amd import autotune as at, _lib as L
    import os
    if not os.path.exists(at.CACHE):
        pytest.skip("no tile cache committed")
    for k, v in at.load_table().items():
        arch, prec, variant, npd = k.split("/")
        assert arch == at.ARCH and prec in ("fp16", "bf16") and variant in ("sym", "plain")
        assert int(npd) % 64 == 0 and 64 <= int(npd) <= L.MAX_ROWS and v in (64, 128)
