"""Pins of the requantiser oracle (paper Sec. 2.1, equaliser), on the CPU.

The oracle rounds with integer shifts and masks; these checks restate the
rule independently: exact rational rounding half to even (Python's round()
on fractions.Fraction), closed forms at unit gain, the two's-complement
field layout of the PFB word, saturation, and the 4-bit RMS band the paper
aims for (Eq. 3)."""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import requant as R


def ref_code(d: int, g: int) -> int:
    q = round(Fraction(d * g, 1 << 21))      # exact; ties to even
    return max(-7, min(7, q))


def test_random_products_against_exact_rounding():
    rng = np.random.default_rng(1)
    d = rng.integers(-(1 << 17), 1 << 17, size=4000)
    g = rng.integers(0, 1 << 18, size=4000)
    d[:1000] = rng.integers(-3000, 3000, size=1000)          # mostly unsaturated
    g[:1000] = rng.integers(0, 1500, size=1000)
    got = R.requantize_value(d, g)
    want = np.array([ref_code(int(a), int(b)) for a, b in zip(d, g)])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("m", range(-9, 9))
def test_ties_round_to_even(m):
    # d * g = (2m + 1) * 2^20 is exactly half-way between codes m and m + 1
    d, g = (2 * m + 1) << 4, 1 << 16
    assert ref_code(d, g) == max(-7, min(7, m + (m & 1)))  # the restatement itself
    assert R.requantize_value(d, g) == max(-7, min(7, m if m % 2 == 0 else m + 1))


def test_unit_gain_closed_form():
    # gain 1.0 (fix_18_7: 128) on k/8 (fix_18_17: k * 2^14) gives code k, saturated at 7
    k = np.arange(-20, 21)
    assert np.array_equal(R.requantize_value(k << 14, 128), np.clip(k, -7, 7))
    # gain 2.0 doubles, gain 0 gives 0
    assert np.array_equal(R.requantize_value(k << 14, 256), np.clip(2 * k, -7, 7))
    assert not R.requantize_value(k << 14, 0).any()


def test_word_layout_and_ignored_bits():
    re, im = -(1 << 17), (1 << 17) - 1                       # the 18-bit extremes
    w = np.uint64(((0xABCDEF1 << 36) | ((re & 0x3FFFF) << 18) | (im & 0x3FFFF)))
    r, i = R.unpack_word(np.array([w]))
    assert (int(r[0]), int(i[0])) == (re, im)
    # gain bits above 18 are ignored
    assert R.requantize_value(1 << 14, (1 << 20) | 128) == 1


def test_packing_real_in_high_nibble():
    words = np.array([[[((3 << 14) << 18) | ((-2 << 14) & 0x3FFFF)]]], dtype=np.uint64)
    out = R.requantize(words, np.array([[128]], dtype=np.uint32))
    assert out[0, 0, 0] == 0x3E                                 # re 3, im -2


def test_paper_rms_band():
    # Sec. 2.1: a sigma of 2^14 with the default gains (~2.5) lands in the 2..3 RMS band
    w = synth.pfb_words(3, 8, 16, 2048)
    g = synth.eq_gains(3, 8, 16)
    out = R.requantize(w, g)
    re = ((out >> 4).astype(np.int16) ^ 8) - 8
    im = ((out & 15).astype(np.int16) ^ 8) - 8
    rms = np.sqrt(0.5 * np.mean(re.astype(float) ** 2 + im.astype(float) ** 2))
    assert 2.0 < rms < 3.0
