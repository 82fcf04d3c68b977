"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before touching the device."""
from __future__ import annotations

import ctypes
import os
import subprocess

import pytest

from paper_2411_09859_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_skip():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libskltlt.so not built")
    return binding.lib()


def test_exports_every_header_function():
    _lib_or_skip()
    names = binding.header_functions()
    assert "skltlt_factor" in names and "skltlt_pfaffian" in names and "skltlt_batched" in names
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], check=True,
                         capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_status_strings():
    L = _lib_or_skip()
    for st in (0, -1, -2, -3, -4, 7):
        assert L.skltlt_status_string(st)


def test_workspace_size_queries():
    _lib_or_skip()
    a = binding.workspace_size(256, 32)
    b = binding.workspace_size(16384, 128)
    assert 0 < a < b
    with pytest.raises(binding.SkltltError) as e:
        binding.workspace_size(-1)
    assert e.value.status == binding.SKLTLT_EINVAL
    with pytest.raises(binding.SkltltError) as e:
        binding.workspace_size(64, 0, precision=7)
    assert e.value.status == binding.SKLTLT_EINVAL
    with pytest.raises(binding.SkltltError) as e:
        binding.workspace_size(64, 1000)
    assert e.value.status == binding.SKLTLT_ENOTSUP


def test_default_block_sizes():
    _lib_or_skip()
    for n in (1, 100, 1000, 5000, 16384):
        b = binding.default_block_size(n)
        assert 1 <= b <= 256


def test_factor_rejects_bad_arguments_without_device_work():
    L = _lib_or_skip()
    vp = ctypes.c_void_p
    fake = vp(0x1000)
    # negative n
    assert L.skltlt_factor(-1, fake, 1, fake, fake, 0, 0, fake, 1 << 20, None) == -1
    # lda < n
    assert L.skltlt_factor(8, fake, 4, fake, fake, 0, 0, fake, 1 << 20, None) == -1
    # unknown precision
    assert L.skltlt_factor(8, fake, 8, fake, fake, 0, 3, fake, 1 << 20, None) == -1
    # null pointers
    assert L.skltlt_factor(8, None, 8, fake, fake, 0, 0, fake, 1 << 20, None) == -1
    assert L.skltlt_factor(8, fake, 8, None, fake, 0, 0, fake, 1 << 20, None) == -1
    # workspace too small / misaligned
    assert L.skltlt_factor(8, fake, 8, fake, fake, 0, 0, fake, 16, None) == -1
    assert L.skltlt_factor(8, fake, 8, fake, fake, 0, 0, vp(0x1008), 1 << 20, None) == -1
    # n = 0 is a no-op
    assert L.skltlt_factor(0, None, 1, None, None, 0, 0, None, 0, None) == 0
    # pfaffian needs its outputs
    assert L.skltlt_pfaffian(8, fake, 8, fake, fake, None, fake, 0, 0, fake, 1 << 20, None) == -1


def test_batched_workspace_size():
    """The queue counter (256 bytes) and the processing order (4 bytes per
    matrix, rounded up to 256 bytes); a shorter workspace is refused before
    anything is enqueued."""
    L = _lib_or_skip()
    sz = ctypes.c_size_t(0)
    assert L.skltlt_batched_workspace_size(-1, ctypes.byref(sz)) == -1
    for batch, want in ((0, 256), (1, 512), (64, 512), (65, 768), (4096, 256 + 4 * 4096)):
        assert L.skltlt_batched_workspace_size(batch, ctypes.byref(sz)) == 0
        assert sz.value == want
    fake = ctypes.c_void_p(0x1000)
    for batch in (1, 4096):
        L.skltlt_batched_workspace_size(batch, ctypes.byref(sz))
        assert L.skltlt_batched(batch, fake, fake, fake, fake, fake, None, None, None, 16, 0, 0,
                                fake, sz.value - 4, None) == binding.SKLTLT_EINVAL


def test_batched_argument_checks():
    """Argument checks of skltlt_batched run before anything is enqueued."""
    L = _lib_or_skip()
    # panel width above the supported 16
    for bs in (17, 33):
        assert L.skltlt_batched(1, None, None, None, None, None, None, None, None, 16, bs, 0, None,
                                0, None) == binding.SKLTLT_ENOTSUP
    # negative batch, orders above the kernel's 256
    assert L.skltlt_batched(-1, None, None, None, None, None, None, None, None, 16, 0, 0, None, 0,
                            None) == binding.SKLTLT_EINVAL
    assert L.skltlt_batched(1, None, None, None, None, None, None, None, None, 257, 0, 0, None, 0,
                            None) == binding.SKLTLT_ENOTSUP


def test_noalloc_batched_limits():
    """The allocation-free batched call states its limit and refuses larger
    batches (and bad arguments) before touching the device."""
    L = _lib_or_skip()
    mx = L.skltlt_batched_noalloc_max_batch()
    assert mx == 1 << 18
    fake = 256  # never dereferenced: the call returns before any device work
    assert L.skltlt_batched_noalloc(mx + 1, fake, fake, fake, fake, fake, None, None, None,
                                    16, 0, 0, None) == binding.SKLTLT_ENOTSUP
    assert L.skltlt_batched_noalloc(-1, fake, fake, fake, fake, fake, None, None, None,
                                    16, 0, 0, None) == binding.SKLTLT_EINVAL
    assert L.skltlt_batched_noalloc(4, fake, fake, fake, fake, fake, None, None, None,
                                    16, 0, 1, None) == binding.SKLTLT_ENOTSUP
    assert L.skltlt_batched_noalloc(0, None, None, None, None, None, None, None, None,
                                    16, 0, 0, None) == binding.SKLTLT_OK


def test_tuner_tables_match_their_measurements(tmp_path):
    """The compiled-in tables are what the tuners write from the committed
    measurements: regenerating the headers from the JSON files gives the
    headers in csrc/ byte for byte, and the library's default widths follow
    the single-matrix table."""
    import json
    import math

    from paper_2411_09859_amd import tune_batched, tune_factor
    _lib_or_skip()
    pkg = os.path.dirname(binding.LIB_PATH)
    fm = json.load(open(os.path.join(pkg, "tune_factor.json")))["orders"]
    ftable = [(int(n), int(v["best"])) for n, v in sorted(fm.items(), key=lambda kv: int(kv[0]))]
    for n, v in fm.items():  # the best is the fastest measured width
        assert int(v["best"]) == int(min(v["ms"], key=v["ms"].get))
    tune_factor.write_outputs(ftable, fm, out_dir=str(tmp_path))
    assert (tmp_path / "factor_table.h").read_text() == \
        open(os.path.join(pkg, "csrc", "factor_table.h")).read()
    bm = json.load(open(os.path.join(pkg, "tune_batched.json")))["classes"]
    btable = []
    for cls, v in sorted(bm.items(), key=lambda kv: int(kv[0].split("-")[1])):
        hi = int(cls.split("-")[1])
        assert v["best_width"] == int(min(v["ms"], key=v["ms"].get).split("x")[0])
        mixed = v["mixed_16_to_hi_ms_by_wgpc"]
        assert v["best_wgpc"] == int(min(mixed, key=mixed.get))
        btable.append((hi, v["best_width"], v["best_wgpc"]))
    tune_batched.write_outputs(btable, bm, out_dir=str(tmp_path))
    assert (tmp_path / "batched_table.h").read_text() == \
        open(os.path.join(pkg, "csrc", "batched_table.h")).read()
    L = binding.lib()
    for k, (n, b) in enumerate(ftable):
        assert L.skltlt_default_block_size(n) == b
        if k + 1 < len(ftable):  # just below the next class boundary
            edge = int(math.sqrt(n * ftable[k + 1][0]))
            assert L.skltlt_default_block_size(edge) == b
