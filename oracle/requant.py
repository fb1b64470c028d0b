"""CPU oracle of the equaliser / 4-bit requantiser (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg use it, and it
imports nothing from the product path.

Paper Sec. 2.1 (equaliser): each 18-bit real and imaginary part of a PFB
output word is multiplied by a per-channel scale factor, an unsigned
fix_18_7 number; the fix_36_24 product is rounded half to even at the
fix_4_3 least significant bit and kept as a 4-bit fix_4_3 number whose
range is 1.001b .. 0.111b, i.e. -7/8 .. 7/8; the two 4-bit parts are
re-packed into one byte.  Readings (the bit numbering of the printed text
is garbled): the PFB parts are fix_18_17 (17 fraction bits, so that 17 + 7 =
24 fraction bits in the product); rounding is at product bit 21 (2^-3 =
2^21 / 2^24); out-of-range values saturate to -7 / +7 (the stated range);
the PFB word carries the real part in bits 35..18 and the imaginary part in
bits 17..0 (the real part first, Sec. 2.1), higher bits ignored; the scale
factor is the low 18 bits of its word; the byte has the real part in the
high nibble (the reading used by the X-engine).
"""
from __future__ import annotations

import numpy as np

FRAC_SHIFT = 21            # 24 fraction bits of the product - 3 of fix_4_3
HALF = 1 << (FRAC_SHIFT - 1)


def sext18(x):
    """Two's-complement value of the low 18 bits."""
    x = np.asarray(x, dtype=np.int64) & 0x3FFFF
    return x - ((x >> 17) << 18)


def unpack_word(w):
    """PFB output word -> (real, imaginary) fix_18_17 integers."""
    w = np.asarray(w, dtype=np.uint64)
    return sext18((w >> np.uint64(18)).astype(np.int64)), sext18((w & np.uint64(0x3FFFF)).astype(np.int64))


def requantize_value(d, g):
    """One fix_18_17 part times one fix_18_7 gain -> 4-bit code in [-7, 7]."""
    p = np.asarray(d, dtype=np.int64) * (np.asarray(g, dtype=np.int64) & 0x3FFFF)
    base = p >> FRAC_SHIFT                    # floor(p / 2^21)
    rem = p - (base << FRAC_SHIFT)            # in [0, 2^21)
    up = (rem > HALF) | ((rem == HALF) & ((base & 1) == 1))
    return np.clip(base + up.astype(np.int64), -7, 7)


def requantize(words: np.ndarray, gains: np.ndarray) -> np.ndarray:
    """uint64 words [T][F][N] and uint32 gains [F][N] -> packed bytes [T][F][N]."""
    re, im = unpack_word(words)
    g = np.asarray(gains).astype(np.int64)[None, :, :]
    qr, qi = requantize_value(re, g), requantize_value(im, g)
    return (((qr & 0xF) << 4) | (qi & 0xF)).astype(np.uint8)


def eq_update(vis: np.ndarray, n_integrated: int, gains: np.ndarray, target_x16: int) -> np.ndarray:
    """New equaliser gains from the autocorrelations (paper Sec. 2.1, Eq. 3).

    RMS_i = sqrt(P_i / (2 N)) with P_i the integrated auto power of input i
    (Re V_ii) over N samples.  The 4-bit RMS scales with the gain, so the
    gain that brings it to the target t = target_x16 / 16 is
    G' = G t / RMS = G t sqrt(2 N / P).  G' is rounded to the nearest
    integer (fix_18_7 units, halves up) exactly: with M = 8 G^2 t^2 N / P,
    round(sqrt(M) / 2) = (isqrt(floor(M)) + 1) // 2; then clamped to
    [1, 2^18 - 1].  Inputs with P = 0 keep their gain."""
    import math
    F, nbl, _ = vis.shape
    N = int((math.isqrt(8 * nbl + 1) - 1) // 2)
    out = np.array(gains, dtype=np.uint32, copy=True)
    for f in range(F):
        for i in range(N):
            P = int(vis[f, i * (i + 1) // 2 + i, 0])
            G = int(gains[f, i]) & 0x3FFFF
            if P <= 0:
                continue
            M = (8 * G * G * target_x16 * target_x16 * n_integrated) // (P * 256)
            k = (math.isqrt(M) + 1) // 2
            out[f, i] = min(max(k, 1), (1 << 18) - 1)
    return out
