"""Host-only checks of the C-ABI library: it loads, exports every function
include/frustration.h declares, and its pure host calls behave (no GPU)."""
import ctypes
import os
import re

import pytest

from paper_2311_00869_amd import frustration as fr

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "frustration.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fi_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = fr.load_library()
    names = _declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(fr.SYMBOLS)


def test_strerror_and_workspace_arithmetic():
    lib = fr.load_library()
    assert lib.fi_strerror(0) == b"ok"
    assert b"symmetric" in lib.fi_strerror(-2)
    size = ctypes.c_size_t()
    assert lib.fi_graph_workspace_size(1000, 10000, 1000, ctypes.byref(size)) == 0
    small = size.value
    assert lib.fi_graph_workspace_size(2000, 20000, 1000, ctypes.byref(size)) == 0
    assert size.value > small > 1000 * 12
    assert lib.fi_graph_workspace_size(-1, 0, 0, ctypes.byref(size)) == -1
    assert lib.fi_graph_workspace_size(10, 2**31, 0, ctypes.byref(size)) == -6


def test_bounded_cloud_sizing_is_host_arithmetic():
    lib = fr.load_library()
    size = ctypes.c_size_t()
    assert lib.fi_bcloud_workspace_size(1000, 256, ctypes.byref(size)) == 0
    one = size.value
    assert lib.fi_bcloud_workspace_size(2000, 256, ctypes.byref(size)) == 0
    assert size.value > one > 1000 * 128  # two entry arrays and the index
    for fmax, staging in ((0, 16), (-1, 16), (2**31 + 1, 16), (8, 0), (8, 8193)):
        assert lib.fi_bcloud_workspace_size(fmax, staging, ctypes.byref(size)) == -1
    # F_max from a memory cap (Alg. alg-scale): the largest table that fits
    fmax = ctypes.c_int64()
    for cap in (1 << 20, 10 << 20, 1 << 30):
        assert lib.fi_bcloud_fmax_for(cap, 1024, ctypes.byref(fmax)) == 0
        assert lib.fi_bcloud_workspace_size(fmax.value, 1024, ctypes.byref(size)) == 0
        assert size.value <= cap
        assert lib.fi_bcloud_workspace_size(fmax.value + 1, 1024, ctypes.byref(size)) == 0
        assert size.value > cap
    assert lib.fi_bcloud_fmax_for(1000, 1024, ctypes.byref(fmax)) == -12
    assert lib.fi_bcloud_create(0, 16, None, 0, None, ctypes.byref(ctypes.c_void_p())) == -1
    assert lib.fi_bcloud_create(8, 16, None, 0, None, ctypes.byref(ctypes.c_void_p())) == -12
    assert b"order" in lib.fi_strerror(-13)


def test_create_rejects_bad_arguments_without_touching_the_device():
    lib = fr.load_library()
    out = ctypes.c_void_p()
    # null output pointer, negative sizes and a missing workspace fail before any HIP call
    assert lib.fi_graph_create(4, 8, None, None, None, 16, None, 0, None, None) == -1
    assert lib.fi_graph_create(-1, 0, None, None, None, 16, None, 0, None, ctypes.byref(out)) == -1
    assert lib.fi_graph_create(4, 2**31, None, None, None, 16, None, 0, None, ctypes.byref(out)) == -6


def test_product_path_has_no_oracle_import():
    pkg = os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_2311_00869_amd")
    for root, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h")):
                text = open(os.path.join(root, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f


def test_default_schedule_crossover(monkeypatch, tmp_path):
    # one tree per workgroup in LDS, then in workspace slots while n + m/2 stays
    # at or below 135,000 (256 threads up to average degree 10), then 128 trees
    # per pass
    from paper_2311_00869_amd import tune
    monkeypatch.setattr(tune, "CACHE", str(tmp_path / "none.json"))
    assert tune.default_schedule(1000, 10000)["block"] == 256
    assert tune.default_schedule(3000, 30000)["block"] == 512
    assert tune.default_schedule(10000, 100000) == dict(path=1, block=1024, grid=0, heavy=512, batch=1)
    assert tune.default_schedule(60000, 2 * 150000) == dict(path=2, block=256, grid=0, heavy=512, batch=1)
    assert tune.default_schedule(30000, 2 * 210000)["block"] == 1024   # 30,000 + 105,000
    assert tune.default_schedule(30000, 2 * 210002)["path"] == 5
    assert tune.default_schedule(60000, 2 * 480000)["path"] == 5
    assert tune.default_schedule(16000000, 2 * 64000000)["path"] == 5


def test_autotune_candidates_cover_every_path_and_multi_grids():
    from paper_2311_00869_amd import tune
    small = tune.candidates(5000, 50000)
    assert {c["path"] for c in small} == {1, 2, 3, 4, 5}
    assert {c["grid"] for c in small if c["path"] == 5} == {0, 64, 128}
    large = tune.candidates(16000000, 128000000)
    assert {c["path"] for c in large} == {3, 4, 5}


def test_clean_no_alloc_rejects_sizes_on_the_host():
    # argument and size checks come before any device work
    lib = fr.load_library()
    counts = (ctypes.c_int64 * 5)()
    big = fr.CLEAN_NO_ALLOC_MAX_ENTRIES + 1
    fake = ctypes.c_void_p(256)
    assert lib.fi_clean_no_alloc(10, big, fake, fake, fake, fake, fake, fake, counts, None) == -6
    assert lib.fi_clean_no_alloc(-1, 0, None, None, None, fake, None, None, counts, None) == -1
    assert lib.fi_clean_no_alloc(10, 5, None, fake, fake, fake, fake, fake, counts, None) == -1
    hdr = open(HEADER).read()
    assert f"#define FI_CLEAN_NO_ALLOC_MAX_ENTRIES {fr.CLEAN_NO_ALLOC_MAX_ENTRIES}" in hdr


def test_gather_probe_rejects_bad_arguments_on_the_host():
    # the measurement aid checks its arguments before any device work, and an
    # empty probe is a no-op
    lib = fr.load_library()
    fake = ctypes.c_void_p(256)
    assert lib.fi_probe_gather(fake, -1, fake, 4, fake, None) == -1
    assert lib.fi_probe_gather(fake, 8, fake, 0, fake, None) == -1
    assert lib.fi_probe_gather(fake, 8, fake, 2**31 + 1, fake, None) == -1
    assert lib.fi_probe_gather(None, 8, fake, 4, fake, None) == -1
    assert lib.fi_probe_gather(fake, 8, fake, 4, None, None) == -1
    assert lib.fi_probe_gather(None, 0, None, 4, fake, None) == 0
