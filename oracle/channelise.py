"""CPU oracle of the F-stage channeliser (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

Paper Sec. 2.1: each real input stream is channelised by a polyphase filter
bank with a Hamming window, FFT length 512 or 1024 (1024 or 2048 real
samples per spectrum here: F channels from 2F real samples), and two real
streams go through one complex FFT as y = x1 + j x2 (Eq. 1), their spectra
recovered from Y as (Eq. 2)
    X1[k] = (Y[k] + conj(Y[-k])) / 2,    X2[k] = (Y[k] - conj(Y[-k])) / (2j).
Readings (the paper gives no tap count or coefficients): P = 4 taps, the
usual polyphase prototype h[m] = w[m] sinc((m - PL/2) / L) with w the
symmetric Hamming window of length PL; spectrum s uses samples
[sL, sL + PL) of each stream, v_s[n] = sum_p h[pL + n] x[sL + pL + n]; the
F channels are k = 0 .. F-1 (the Nyquist bin is dropped); the two inputs
of a complex FFT are 2q and 2q + 1.  Float64 throughout; the FFT is
numpy's (a library step).
"""
from __future__ import annotations

import numpy as np

TAPS = 4


def coefficients(L: int, taps: int = TAPS) -> np.ndarray:
    m = np.arange(taps * L, dtype=np.float64)
    w = 0.54 - 0.46 * np.cos(2.0 * np.pi * m / (taps * L - 1))
    return w * np.sinc((m - taps * L / 2.0) / L)


def n_spectra(n_samples: int, L: int, taps: int = TAPS) -> int:
    return max(0, n_samples // L - taps + 1)


def frames(x: np.ndarray, L: int, taps: int = TAPS) -> np.ndarray:
    """x [N][S] real -> polyphase frames v [N][S'][L]."""
    h = coefficients(L, taps).reshape(taps, L)
    S = n_spectra(x.shape[1], L, taps)
    blocks = x[:, : (S + taps - 1) * L].astype(np.float64).reshape(x.shape[0], S + taps - 1, L)
    v = np.zeros((x.shape[0], S, L))
    for p in range(taps):
        v += h[p][None, None, :] * blocks[:, p:p + S, :]
    return v


def channelise(x: np.ndarray, F: int, taps: int = TAPS) -> np.ndarray:
    """int8 ADC samples x [N][S] (N even) -> complex spectra [S'][F][N]."""
    L = 2 * F
    v = frames(x, L, taps)                                 # [N][S'][L]
    y = v[0::2] + 1j * v[1::2]                             # Eq. 1: inputs 2q, 2q + 1
    Y = np.fft.fft(y, axis=-1)                             # [N/2][S'][L]
    Yr = np.conj(np.roll(Y[..., ::-1], 1, axis=-1))        # conj(Y[-k])
    X1 = (Y + Yr) / 2.0                                    # Eq. 2
    X2 = (Y - Yr) / 2.0j
    out = np.empty((x.shape[0], v.shape[1], F), dtype=np.complex128)
    out[0::2], out[1::2] = X1[..., :F], X2[..., :F]
    return np.ascontiguousarray(out.transpose(1, 2, 0))    # [S'][F][N]
