"""CPU oracle of the X-engine (test infrastructure).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The product path
(the HIP library and its Python binding) never imports it, and it imports
nothing from the product path; the two share only the seeded input
generator in ``synth``.

The arithmetic lives in ``xeng_oracle.c`` (plain loops, int64 sums); this file
compiles it with gcc on first use and wraps it with ctypes. Every function
states the passage of the paper it follows:

* ``decode``        Sec. 2.1 (equaliser output: 4-bit two's-complement real
                    and imaginary parts re-packed into one byte) and Sec. 2.3
                    (one byte per complex sample); real part = high nibble.
* ``accumulate``    Sec. 2 (FX: cross-multiply spectra of each pair at the
                    same frequency, integrate over a chosen duration), Sec. 2.2
                    (complex multiply-accumulate), Sec. 2.3 (natural order:
                    fix one input, run over all inputs including itself).
* ``Engine``        the same, with the integration spanning every call since
                    the last dump, and a dump that narrows to int32.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xeng_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# Largest integration (samples since the last dump) whose sums are
# guaranteed to fit int32: |Re|, |Im| <= 128 per sample (all codes -8).
T_MAX_EXACT = (2**31 - 1) // 128


# gcc flags of the oracle library (integer arithmetic: the optimisation level
# changes the speed, not the results)
BUILD_FLAGS = "-O3 -fopenmp"


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3, OpenMP) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *BUILD_FLAGS.split(), "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = ctypes.CDLL(build())
            u8p = ctypes.POINTER(ctypes.c_uint8)
            L.oracle_decode.argtypes = [ctypes.c_uint8, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]
            L.oracle_nbaselines.argtypes = [ctypes.c_int32]
            L.oracle_nbaselines.restype = ctypes.c_int64
            L.oracle_baseline_index.argtypes = [ctypes.c_int32, ctypes.c_int32]
            L.oracle_baseline_index.restype = ctypes.c_int64
            L.oracle_accumulate_i4.argtypes = [u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_int]
            L.oracle_accumulate_i4.restype = ctypes.c_int
            L.oracle_accumulate_c128.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                                 ctypes.c_int32, ctypes.c_void_p, ctypes.c_int]
            L.oracle_accumulate_c128.restype = ctypes.c_int
            L.oracle_to_int32.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
            L.oracle_to_int32.restype = ctypes.c_int64
            L.oracle_max_threads.restype = ctypes.c_int
            _lib = L
    return _lib


def max_threads() -> int:
    """OpenMP threads the oracle uses when nthreads = 0."""
    return int(lib().oracle_max_threads())


def decode(byte: int) -> tuple[int, int]:
    re, im = ctypes.c_int32(), ctypes.c_int32()
    lib().oracle_decode(ctypes.c_uint8(byte), ctypes.byref(re), ctypes.byref(im))
    return re.value, im.value


def nbaselines(n: int) -> int:
    return int(lib().oracle_nbaselines(n))


def baseline_index(i: int, j: int) -> int:
    return int(lib().oracle_baseline_index(i, j))


def accumulate(v: np.ndarray, acc: np.ndarray | None = None, chans=None,
               nthreads: int = 0) -> np.ndarray:
    """Integrate packed voltages v (uint8 [T, F, N]) into int64 acc [F', nbl, 2].

    ``chans`` = (f0, f1) restricts the work to channels f0..f1-1; acc then has
    f1 - f0 rows.
    """
    v = np.ascontiguousarray(v, dtype=np.uint8)
    if v.ndim != 3:
        raise ValueError("voltages must be [T, F, N]")
    T, F, N = v.shape
    f0, f1 = (0, F) if chans is None else chans
    nbl = N * (N + 1) // 2
    if acc is None:
        acc = np.zeros((f1 - f0, nbl, 2), dtype=np.int64)
    if acc.dtype != np.int64 or acc.shape != (f1 - f0, nbl, 2) or not acc.flags.c_contiguous:
        raise ValueError("acc must be C-contiguous int64 [F', nbl, 2]")
    if N == 0 or f1 == f0:
        return acc
    rc = lib().oracle_accumulate_i4(v.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), T, F, N,
                                    f0, f1, acc.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError("oracle_accumulate_i4 rejected its arguments")
    return acc


def accumulate_c128(x: np.ndarray, acc: np.ndarray | None = None, nthreads: int = 0) -> np.ndarray:
    """Float64 form: x complex [T, F, N] -> acc complex [F, nbl] (sum x_i conj x_j)."""
    x = np.asarray(x, dtype=np.complex128)
    T, F, N = x.shape
    xr = np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1))
    nbl = N * (N + 1) // 2
    out = np.zeros((F, nbl, 2), dtype=np.float64)
    rc = lib().oracle_accumulate_c128(xr.ctypes.data, T, F, N, out.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError("oracle_accumulate_c128 rejected its arguments")
    res = out[..., 0] + 1j * out[..., 1]
    return res if acc is None else acc + res


def to_int32(acc: np.ndarray) -> np.ndarray:
    """Narrow int64 sums to int32; raises OverflowError if any does not fit."""
    acc = np.ascontiguousarray(acc, dtype=np.int64)
    out = np.empty(acc.shape, dtype=np.int32)
    bad = lib().oracle_to_int32(acc.ctypes.data, acc.size, out.ctypes.data)
    if bad:
        raise OverflowError(f"{bad} visibilities exceed int32")
    return out


def correlate(v: np.ndarray, chans=None, nthreads: int = 0) -> np.ndarray:
    """One integration over v: int32 [F', nbl, 2] visibilities."""
    return to_int32(accumulate(v, chans=chans, nthreads=nthreads))


class Engine:
    """Oracle with the boundary's integration semantics.

    The integration spans every ``correlate`` call since the last ``dump``;
    ``dump`` returns the int32 visibilities and the number of samples
    integrated, then (unless ``keep``) starts a new integration.
    """

    def __init__(self, n_inputs: int, n_chans: int, nthreads: int = 0):
        self.n_inputs, self.n_chans, self.nthreads = n_inputs, n_chans, nthreads
        self.acc = np.zeros((n_chans, n_inputs * (n_inputs + 1) // 2, 2), dtype=np.int64)
        self.n_integrated = 0

    def correlate(self, v: np.ndarray) -> None:
        if v.shape[1:] != (self.n_chans, self.n_inputs):
            raise ValueError("voltage block shape does not match the engine")
        accumulate(v, self.acc, nthreads=self.nthreads)
        self.n_integrated += v.shape[0]

    def dump(self, keep: bool = False):
        vis, n = to_int32(self.acc), self.n_integrated
        if not keep:
            self.acc[...] = 0
            self.n_integrated = 0
        return vis, n
