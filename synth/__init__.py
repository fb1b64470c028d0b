"""Seeded synthetic channelised voltages for the X-engine.

This module is the only code shared by the CPU oracle and the HIP path: it
produces the *input* bytes and nothing else. It holds none of the X-engine's
arithmetic (no decoding, no products, no sums over time).

What it stands in for. The correlator's X-engine receives, for every time
sample and frequency channel, one byte per input: a complex sample with a
4-bit two's-complement real part and a 4-bit imaginary part, in the order
[time, channel, input] (paper, Sec. 2.3, description of the packet payload
and of the order the correlation code expects). The F-engine's equaliser
produces 4-bit values in the range -7..+7 with an RMS of 2-3 (paper,
Sec. 2.1, equaliser description and Eq. 3). The paper's own data are
hardware observations that are not available, so seeded synthetic
voltages with the paper's shapes stand in for them:

* ``uniform``  re, im iid uniform integers in [-7, 7].
* ``tone``     Q(sigma*(g + j g') + 0.5*sigma*exp(j phi_i)*exp(j(2 pi 0.01 t + theta_f)))
* ``sources``  Q(sigma*(g + j g') + sum_k A_k exp(j phi_ik) s_k(f, t)),
               A = (0.5, 0.35, 0.25)*sigma (first ``n_src`` of them),
               s_k iid unit-power complex Gaussian shared by all inputs.
* ``noise``    Q(sigma*(g + j g'))

with sigma = 2.5, g, g' iid standard normal, phases uniform in [0, 2 pi),
and Q(z) = clip(round_half_even(z), -7, 7) per component (the requantiser
range of the paper's equaliser). Packing puts the real part in the high
nibble and the imaginary part in the low nibble of each byte.

Seeding. Every (array, block, channel) has its own PCG64 stream derived with
``SeedSequence(seed, spawn_key=(1, array, block, channel))`` and every array
its own parameter stream ``spawn_key=(0, array)``, so the bytes of a channel
do not depend on how channels are chunked or threaded, and block ``b`` of a
stream is reproducible on its own.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

SIGMA = 2.5
SOURCE_AMPS = (0.5, 0.35, 0.25)
TONE_AMP = 0.5
TONE_FREQ = 0.01  # cycles per sample

RECIPES = ("uniform", "tone", "sources", "noise")


def _rng(seed: int, key: tuple) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=key)))


def quantise(z: np.ndarray) -> np.ndarray:
    """Requantise one real component: round half to even, clip to [-7, 7]."""
    return np.clip(np.rint(z), -7, 7).astype(np.int8)


def pack(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Pack 4-bit two's-complement (re, im) into one byte, re in the high nibble."""
    re = np.asarray(re)
    im = np.asarray(im)
    if re.size and (re.min() < -8 or re.max() > 7 or im.min() < -8 or im.max() > 7):
        raise ValueError("4-bit components must lie in [-8, 7]")
    re8 = re.astype(np.int8).view(np.uint8)
    im8 = im.astype(np.int8).view(np.uint8)
    return ((re8 << 4) | (im8 & 0xF)).astype(np.uint8)


@dataclass(frozen=True)
class ArrayParams:
    """Per-array draws that are fixed across channels and blocks."""
    phi_tone: np.ndarray      # [N] tone phase per input
    phi_src: np.ndarray       # [N, 3] source phase per input


def array_params(seed: int, n_inputs: int, array: int = 0) -> ArrayParams:
    r = _rng(seed, (0, array))
    phi_tone = r.uniform(0.0, 2 * np.pi, size=n_inputs)
    phi_src = r.uniform(0.0, 2 * np.pi, size=(n_inputs, len(SOURCE_AMPS)))
    return ArrayParams(phi_tone, phi_src)


def _channel(recipe: str, seed: int, n_inputs: int, n_time: int, f: int,
             array: int, block: int, params: ArrayParams, n_src: int) -> np.ndarray:
    """One channel's packed bytes, shape [T, N]."""
    r = _rng(seed, (1, array, block, f))
    if recipe == "uniform":
        v = r.integers(-7, 8, size=(n_time, n_inputs, 2), dtype=np.int8)
        return pack(v[..., 0], v[..., 1])
    g = r.standard_normal(size=(n_time, n_inputs, 2), dtype=np.float32)
    g *= np.float32(SIGMA)
    re, im = g[..., 0], g[..., 1]
    if recipe == "tone":
        # exp(j(2 pi nu t + theta_f + phi_i)) = exp(j(2 pi nu t + theta_f)) * exp(j phi_i)
        theta_f = r.uniform(0.0, 2 * np.pi)
        t = np.arange(n_time, dtype=np.float64) + float(block) * n_time
        pt = np.exp(1j * (2 * np.pi * TONE_FREQ * t + theta_f)).astype(np.complex64)
        pi_ = (TONE_AMP * SIGMA * np.exp(1j * params.phi_tone)).astype(np.complex64)
        z = pt[:, None] * pi_[None, :]
        re += z.real
        im += z.imag
    elif recipe == "sources":
        k = max(0, min(n_src, len(SOURCE_AMPS)))
        s = r.standard_normal(size=(n_time, k, 2), dtype=np.float32) * np.float32(np.sqrt(0.5))
        sc = (s[..., 0] + 1j * s[..., 1]).astype(np.complex64)               # [T, k]
        gain = np.asarray(SOURCE_AMPS[:k]) * SIGMA                             # [k]
        mix = (gain[None, :] * np.exp(1j * params.phi_src[:, :k])).astype(np.complex64)  # [N, k]
        z = sc @ mix.T                                                         # [T, N]
        re += z.real
        im += z.imag
    elif recipe != "noise":
        raise ValueError(f"unknown recipe {recipe!r}")
    return pack(quantise(re), quantise(im))


def voltages(recipe: str, seed: int, n_inputs: int, n_chans: int, n_time: int,
             array: int = 0, block: int = 0, chans=None, n_src: int = 3,
             threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Packed 4+4-bit voltages, uint8 [T, F, N] (time, channel, input).

    ``chans`` restricts generation to a subset of channels; the returned array
    then has shape [T, len(chans), N] and holds exactly the bytes those
    channels have in the full array.
    """
    if recipe not in RECIPES:
        raise ValueError(f"unknown recipe {recipe!r}")
    chans = list(range(n_chans)) if chans is None else list(chans)
    params = array_params(seed, n_inputs, array)
    if out is None:
        out = np.empty((n_time, len(chans), n_inputs), dtype=np.uint8)
    if n_time == 0 or not chans or n_inputs == 0:
        return out

    def work(idx):
        out[:, idx, :] = _channel(recipe, seed, n_inputs, n_time, chans[idx], array,
                                  block, params, n_src)

    nthr = threads or min(16, os.cpu_count() or 1)
    if nthr <= 1 or len(chans) == 1:
        for i in range(len(chans)):
            work(i)
    else:
        with ThreadPoolExecutor(nthr) as ex:
            list(ex.map(work, range(len(chans))))
    return out


# Workload shapes of the paper's two arrays (Sec. 1: 16 dual-pol dishes = 32
# inputs; 96 dual-pol cylinder feeds = 192 inputs; Sec. 2.1: 512/1024-point
# FFT).  Named by what they are.
WORKLOADS = {
    "dish_tiny": dict(recipe="uniform", seed=1, n_inputs=32, n_chans=64, n_time=4096, calls=1),
    "dish": dict(recipe="tone", seed=2, n_inputs=32, n_chans=1024, n_time=16384, calls=8),
    "cylinder": dict(recipe="sources", seed=3, n_inputs=192, n_chans=1024, n_time=8192, calls=1),
}


def batch_arrays(seed: int = 4, n_arrays: int = 12):
    """Shapes of the batched workload: N, F, T drawn per array from the seed."""
    r = _rng(seed, (2,))
    ns = r.choice([16, 32, 48, 64, 96, 192], size=n_arrays)
    fs = r.choice([256, 512, 1024], size=n_arrays)
    ts = r.choice([2048, 4096, 8192], size=n_arrays)
    return [dict(n_inputs=int(n), n_chans=int(f), n_time=int(t)) for n, f, t in zip(ns, fs, ts)]


def stream_subarrays(seed: int = 5):
    """Sub-arrays of the streaming workload with their dump lengths (samples)."""
    shapes = [(192, 1024), (96, 1024), (32, 1024), (32, 256)]
    r = _rng(seed, (3,))
    dumps = r.choice([8192, 16384, 32768, 65536], size=len(shapes))
    return [dict(n_inputs=n, n_chans=f, dump_len=int(d)) for (n, f), d in zip(shapes, dumps)]


def pfb_words(seed: int, n_inputs: int, n_chans: int, n_time: int, sigma: float = 2.0 ** 14) -> np.ndarray:
    """F-engine output words, uint64 [T][F][N]: 18-bit two's-complement real
    part in bits 35..18, imaginary part in bits 17..0 (fix_18_17 integers),
    Gaussian with the given sigma, clipped to the 18-bit range; bits 36..63
    carry seeded junk, which the equaliser ignores."""
    r = _rng(seed, (4,))
    z = r.normal(0.0, sigma, size=(n_time, n_chans, n_inputs, 2))
    v = np.clip(np.rint(z), -(1 << 17), (1 << 17) - 1).astype(np.int64) & 0x3FFFF
    junk = r.integers(0, 1 << 28, size=(n_time, n_chans, n_inputs), dtype=np.int64)
    return ((junk << 36) | (v[..., 0] << 18) | v[..., 1]).astype(np.uint64)


def eq_gains(seed: int, n_inputs: int, n_chans: int, center: float = 320.0, spread: float = 0.2) -> np.ndarray:
    """Equaliser scale factors, uint32 [F][N], unsigned fix_18_7 integers
    around `center` (320 = 2.5: a fix_18_17 sigma of 2^14 then lands at an
    RMS of 2.5 codes), +-spread relative."""
    r = _rng(seed, (5,))
    g = center * (1.0 + r.uniform(-spread, spread, size=(n_chans, n_inputs)))
    return np.clip(np.rint(g), 0, (1 << 18) - 1).astype(np.uint32)


def packets(block: np.ndarray, mcnt0: int, xid: int, stride: int | None = None) -> np.ndarray:
    """Cut a voltage block uint8 [8 M][F][32 B] into the F engine's packets
    (one per time block of 8 samples and board of 32 inputs), each an 8-byte
    header (6-byte big-endian counter, board id, band id) followed by the
    [8][F][32] payload, padded to `stride` bytes.  Packets are in (counter,
    board) order; tests shuffle, drop and duplicate them."""
    T, F, N = block.shape
    M, B = T // 8, N // 32
    pay = 8 * F * 32
    stride = stride or 8 + pay
    out = np.zeros((M * B, stride), dtype=np.uint8)
    for m in range(M):
        for b in range(B):
            row = out[m * B + b]
            row[:6] = np.frombuffer((mcnt0 + m).to_bytes(6, "big"), dtype=np.uint8)
            row[6], row[7] = b, xid
            row[8:8 + pay] = block[8 * m:8 * m + 8, :, 32 * b:32 * b + 32].reshape(-1)
    return out
