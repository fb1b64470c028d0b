"""The seeded input generator: determinism, chunk independence, value range."""
import numpy as np
import pytest

import synth


@pytest.mark.parametrize("recipe", synth.RECIPES)
def test_deterministic_and_chunk_independent(recipe):
    full = synth.voltages(recipe, 11, 24, 9, 64, threads=4)
    again = synth.voltages(recipe, 11, 24, 9, 64, threads=1)
    np.testing.assert_array_equal(full, again)
    part = synth.voltages(recipe, 11, 24, 9, 64, chans=[7, 2], threads=1)
    np.testing.assert_array_equal(part, full[:, [7, 2]])
    other = synth.voltages(recipe, 12, 24, 9, 64)
    assert not np.array_equal(full, other)


@pytest.mark.parametrize("recipe", synth.RECIPES)
def test_range_never_minus8(recipe):
    v = synth.voltages(recipe, 3, 16, 4, 512)
    hi, lo = v >> 4, v & 0xF
    assert not np.any(hi == 8) and not np.any(lo == 8)   # requantiser range is +-7


def test_blocks_differ_and_shapes():
    a = synth.voltages("sources", 5, 8, 3, 32, array=1, block=0)
    b = synth.voltages("sources", 5, 8, 3, 32, array=1, block=1)
    assert a.shape == (32, 3, 8) and not np.array_equal(a, b)
    assert synth.voltages("noise", 1, 8, 3, 0).shape == (0, 3, 8)


def test_pack_layout_and_range():
    assert synth.pack(np.array([1]), np.array([2]))[0] == 0x12
    assert synth.pack(np.array([-1]), np.array([-8]))[0] == 0xF8
    with pytest.raises(ValueError):
        synth.pack(np.array([8]), np.array([0]))


def test_workload_shapes():
    assert [a["n_inputs"] for a in synth.batch_arrays()] == [a["n_inputs"] for a in synth.batch_arrays()]
    arrs = synth.batch_arrays()
    assert len(arrs) == 12
    assert all(a["n_inputs"] in (16, 32, 48, 64, 96, 192) for a in arrs)
    assert all(a["n_chans"] in (256, 512, 1024) for a in arrs)
    assert all(a["n_time"] in (2048, 4096, 8192) for a in arrs)
    subs = synth.stream_subarrays()
    assert [(s["n_inputs"], s["n_chans"]) for s in subs] == [(192, 1024), (96, 1024), (32, 1024), (32, 256)]
    assert all(8192 <= s["dump_len"] <= 65536 for s in subs)
