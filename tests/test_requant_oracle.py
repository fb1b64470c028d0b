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


def test_eq_update_exact_rounding_and_closed_form():
    from fractions import Fraction
    import math
    rng = np.random.default_rng(9)
    F, N, T = 3, 5, 4096
    vis = np.zeros((F, N * (N + 1) // 2, 2), dtype=np.int32)
    gains = rng.integers(1, 1 << 18, size=(F, N)).astype(np.uint32)
    P = rng.integers(1, 128 * T, size=(F, N))
    for i in range(N):
        vis[:, i * (i + 1) // 2 + i, 0] = P[:, i]
    vis[1, 2 * 3 // 2 + 2, 0] = 0                      # a silent input keeps its gain
    got = R.eq_update(vis, T, gains, 40)               # target 2.5
    for f in range(F):
        for i in range(N):
            p = int(vis[f, i * (i + 1) // 2 + i, 0])
            if p == 0:
                assert got[f, i] == gains[f, i]
                continue
            # restatement: nearest integer to G t sqrt(2 N / P), from exact
            # rational bounds (no float): k minimises |k^2 ... |, checked by
            # bracketing (k - 1/2)^2 <= (G t)^2 2N/P < (k + 1/2)^2
            x2 = Fraction(int(gains[f, i]) ** 2 * 25 * 2 * T, 4 * p)
            k = int(got[f, i])
            if 1 < k < (1 << 18) - 1:
                assert Fraction(2 * k - 1, 2) ** 2 <= x2 < Fraction(2 * k + 1, 2) ** 2
    # closed form: RMS already at the target -> gain unchanged
    g0 = np.full((1, 1), 320, dtype=np.uint32)
    v0 = np.zeros((1, 1, 2), dtype=np.int32)
    v0[0, 0, 0] = 2 * 1000 * (5 * 5) // 4             # RMS = 2.5 exactly over N = 1000
    assert R.eq_update(v0, 1000, g0, 40)[0, 0] == 320
    # RMS twice the target -> gain halves
    v0[0, 0, 0] = 2 * 1000 * 25                        # RMS = 5
    assert R.eq_update(v0, 1000, g0, 40)[0, 0] == 160
