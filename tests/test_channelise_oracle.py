"""Pins of the channeliser oracle (paper Sec. 2.1, Eq. 1-2), on the CPU:
Eq. 2 against separate real transforms, the polyphase frames against a
direct FIR sum, tone placement, and the one-tap rectangular case."""
import numpy as np

from oracle import channelise as C


def test_two_real_trick_equals_separate_transforms():
    rng = np.random.default_rng(1)
    F = 64
    x = rng.integers(-128, 128, size=(4, 2 * F * 9)).astype(np.int8)
    X = C.channelise(x, F)
    v = C.frames(x, 2 * F)
    for i in range(4):
        direct = np.fft.rfft(v[i], axis=-1)[:, :F]        # a real transform per input
        assert np.allclose(X[:, :, i], direct, rtol=0, atol=1e-9 * np.abs(direct).max())


def test_frames_are_the_fir_sum():
    rng = np.random.default_rng(2)
    L, taps = 32, 4
    x = rng.integers(-128, 128, size=(2, L * 10)).astype(np.int8)
    h = C.coefficients(L, taps)
    v = C.frames(x, L, taps)
    s, n = 3, 17
    want = sum(h[p * L + n] * float(x[1, s * L + p * L + n]) for p in range(taps))
    assert abs(v[1, s, n] - want) < 1e-12
    assert v.shape == (2, C.n_spectra(x.shape[1], L, taps), L)


def test_coefficients_shape_and_symmetry():
    h = C.coefficients(256)
    assert h.shape == (1024,)
    m = np.arange(1024)
    w = 0.54 - 0.46 * np.cos(2 * np.pi * m / 1023)       # symmetric Hamming, length PL
    assert np.allclose(w, w[::-1]) and abs(w[0] - 0.08) < 1e-12
    sinc_part = h / w
    # the sinc is centred on PL/2 = 512, zero at every other multiple of L = 256
    assert np.allclose(sinc_part[1:], sinc_part[1:][::-1], atol=1e-12)
    assert abs(sinc_part[512] - 1) < 1e-12 and np.allclose(sinc_part[[0, 256, 768]], 0, atol=1e-12)


def test_tone_lands_in_its_channel():
    F, k0 = 128, 37
    L = 2 * F
    n = np.arange(L * 12)
    x = np.stack([np.round(60 * np.cos(2 * np.pi * k0 * n / L)),
                  np.round(60 * np.sin(2 * np.pi * (k0 + 5) * n / L))]).astype(np.int8)
    X = C.channelise(x, F)
    assert np.argmax(np.abs(X[2, :, 0])) == k0
    assert np.argmax(np.abs(X[2, :, 1])) == k0 + 5


def test_one_tap_rectangular_is_a_plain_fft():
    rng = np.random.default_rng(3)
    F = 16
    x = rng.integers(-128, 128, size=(2, 2 * F * 3)).astype(np.int8)
    h1 = C.coefficients(2 * F, taps=1)
    v = C.frames(x, 2 * F, taps=1)
    assert np.allclose(v, x.reshape(2, 3, 2 * F) * h1[None, None, :])
