"""CPU-side checks of the C ABI library: it loads, exports every symbol the
header declares, and its host-only helpers and argument checks behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xeng.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xeng_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("xeng_plan", "xeng_correlate", "xeng_dump", "xeng_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1904_07778_amd import xeng
    lib = ctypes.CDLL(xeng.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_helpers():
    from paper_1904_07778_amd import xeng as X
    assert X.xeng_nbaselines(0) == 0 and X.xeng_nbaselines(-1) == -1
    assert X.xeng_nbaselines(192) == 18528
    k = 0
    for i in range(20):
        for j in range(i + 1):
            assert X.xeng_baseline_index(i, j) == k
            k += 1
        assert X.xeng_baseline_index(i, i + 1) == -1
    assert X.xeng_strerror(X.XENG_EOVERFLOW)
    assert X.xeng_strerror(12345) == "unknown status"


@pytest.mark.parametrize("desc", [(0, 4, 10), (257, 4, 10), (8, 0, 10), (8, 4, 0), (8, 4, 16_777_216),
                                  (256, 8_388_608, 10)])   # F * N = 2^31: a time row past 32-bit offsets
def test_plan_rejects_bad_shapes_before_touching_the_device(desc):
    from paper_1904_07778_amd import xeng as X
    with pytest.raises(X.XengError) as e:
        X.xeng_plan([desc])
    assert e.value.status == X.XENG_EINVAL


def test_null_arguments():
    from paper_1904_07778_amd import xeng as X
    lib = X._lib
    assert lib.xeng_plan(None, None, 1, 0, None) == X.XENG_EINVAL
    assert lib.xeng_correlate(None, None, None) == X.XENG_EINVAL
    assert lib.xeng_dump(None, 0, None, 0, None) == X.XENG_EINVAL
    lib.xeng_destroy(None)
    assert X.xeng_integrated(None, 0) == -1


def test_null_arguments_of_batch_and_serving_calls():
    from paper_1904_07778_amd import xeng as X
    lib = X._lib
    assert lib.xeng_attach(None, None, None) == X.XENG_EINVAL
    assert lib.xeng_detach(None, 0) == X.XENG_EINVAL
    assert lib.xeng_autotune(None, None, None, 1, None) == X.XENG_EINVAL
    assert X.xeng_slots(None) == -1


def test_accumulator_bytes():
    from paper_1904_07778_amd import xeng as X
    assert X.xeng_accumulator_bytes(192, 1024) == 1024 * 18528 * 8
    assert X.xeng_accumulator_bytes(1, 1) == 8
    assert X.xeng_accumulator_bytes(0, 5) == -1 and X.xeng_accumulator_bytes(5, 0) == -1


def test_plan_flags_and_empty_plans():
    from paper_1904_07778_amd import xeng as X
    with pytest.raises(X.XengError) as e:
        X.xeng_plan([])                       # an empty plan must be a batched one
    assert e.value.status == X.XENG_EINVAL
    with pytest.raises(X.XengError) as e:
        X.xeng_plan([(8, 4, 10)], flags=1 << 5)   # unknown flag
    assert e.value.status == X.XENG_EINVAL


def test_requantize_argument_checks_without_device():
    from paper_1904_07778_amd import xeng as X
    lib = X._lib
    assert lib.xeng_requantize(None, None, None, 1, 1, 1, None) == X.XENG_EINVAL
    assert lib.xeng_requantize(8, 4, 16, -1, 1, 1, None) == X.XENG_EINVAL     # n_time < 0
    assert lib.xeng_requantize(8, 4, 16, 1, 0, 1, None) == X.XENG_EINVAL      # no channels
    assert lib.xeng_requantize(9, 4, 16, 1, 1, 1, None) == X.XENG_EINVAL      # words misaligned
    assert lib.xeng_requantize(8, 6, 16, 1, 1, 1, None) == X.XENG_EINVAL      # gains misaligned
    assert lib.xeng_requantize(8, 4, 16, 0, 1, 1, None) == X.XENG_OK          # nothing to do


def test_ingest_argument_checks_without_device():
    from paper_1904_07778_amd import xeng as X
    lib = X._lib
    ok = dict(n_packets=1, stride=8 + 8 * 32 * 32, mcnt0=0, blocks=1, boards=1, chans=32, xid=0)
    def call(pk=8, idx=4, out=8, **kw):
        a = dict(ok, **kw)
        return lib.xeng_ingest(pk, a["n_packets"], a["stride"], a["mcnt0"], a["blocks"], a["boards"],
                               a["chans"], a["xid"], idx, out, None)
    assert call(idx=None) == X.XENG_EINVAL
    assert call(stride=8 + 8 * 32 * 32 - 8) == X.XENG_EINVAL      # payload does not fit
    assert call(stride=8 + 8 * 32 * 32 + 4) == X.XENG_EINVAL      # not a multiple of 8
    assert call(boards=9) == X.XENG_EINVAL                        # 288 inputs
    assert call(xid=256) == X.XENG_EINVAL
    assert call(mcnt0=1 << 48) == X.XENG_EINVAL
    assert call(pk=12) == X.XENG_EINVAL                           # misaligned packets
    assert call(blocks=65536) == X.XENG_EINVAL


def test_channelise_sizes_and_checks_without_device():
    from paper_1904_07778_amd import xeng as X
    lib = X._lib
    assert lib.xeng_channelise_spectra(2048 * 10, 1024) == 7
    assert lib.xeng_channelise_spectra(2048 * 3, 1024) == 0
    assert lib.xeng_channelise_table_floats(1024) == 4 * 2048 + 2048
    assert lib.xeng_channelise(8, 2048, 3, 1024, 16, 16, None) == X.XENG_EINVAL   # odd input count
    assert lib.xeng_channelise(8, 2048, 2, 1000, 16, 16, None) == X.XENG_EINVAL   # not a power of two
    assert lib.xeng_channelise(8, 2048, 2, 2048, 16, 16, None) == X.XENG_EINVAL   # FFT too long
    assert lib.xeng_channelise(8, 2044, 2, 1024, 16, 16, None) == X.XENG_EINVAL   # samples % 8
    assert lib.xeng_channelise(8, 2048, 2, 1024, 24, 16, None) == X.XENG_EINVAL   # out misaligned


def test_stats_and_load_argument_checks():
    from paper_1904_07778_amd import xeng as X
    lib = X._lib
    assert lib.xeng_stats(None, None) == X.XENG_EINVAL
    assert lib.xeng_load_acc(None, 0, None, 0) == X.XENG_EINVAL


def test_correlate_dump_argument_checks():
    from paper_1904_07778_amd import xeng as X
    assert X._lib.xeng_correlate_dump(None, None, None, None, None) == X.XENG_EINVAL


def test_tune_cache_file_round_trip(tmp_path):
    """The tuning cache reads and writes its text form without a GPU;
    malformed lines are skipped and reported."""
    from paper_1904_07778_amd import xeng as X
    X.xeng_tune_cache_clear()
    src = tmp_path / "tune.txt"
    src.write_text("# comment\n"
                   "gfx950 0 192 10 13 0 2 0\n"
                   "gfx950 1 32 10 11 1 1 1\n"
                   "gfx950 1 0 0 4 0 4 0\n"        # a batched plan's items per workgroup
                   "gfx950 0 0 0 4 0 4 0\n"        # N = 0 is for batched plans only
                   "gfx950 0 999 10 13 0 2 0\n"     # N out of range
                   "garbage line\n")
    with pytest.raises(X.XengError) as ei:
        X.xeng_tune_cache_load(str(src))
    assert ei.value.status == X.XENG_EINVAL
    out = tmp_path / "saved.txt"
    X.xeng_tune_cache_save(str(out))
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert sorted(lines) == ["gfx950 0 192 10 13 0 2 0", "gfx950 1 0 0 4 0 4 0", "gfx950 1 32 10 11 1 1 1"]
    X.xeng_tune_cache_clear()
    X.xeng_tune_cache_save(str(out))
    assert [l for l in out.read_text().splitlines() if not l.startswith("#")] == []
    with pytest.raises(X.XengError):
        X.xeng_tune_cache_load(str(tmp_path / "missing.txt"))
