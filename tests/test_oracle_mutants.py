"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle's C source, plants one plausible mistake (a
dropped term, a wrong sign, a swapped nibble, a transposed index ...),
every one of them keeping its memory accesses in bounds,
compiles it on the CPU and checks that the hand-worked examples or the
brute-force comparison reject it.  The product path is not involved.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests.golden.fixtures import hand_examples
from tests.test_oracle_pins import brute_force, full_matrix, random_bytes

SRC = os.path.join(os.path.dirname(oracle.__file__), "xeng_oracle.c")

MUTANTS = {
    "im_sign": ("(b[i] * a[j] - a[i] * b[j])", "(a[i] * b[j] - b[i] * a[j])"),
    "dropped_bb": ("(a[i] * a[j] + b[i] * b[j])", "(a[i] * a[j])"),
    "nibbles_swapped": ("*re = sext4((byte >> 4) & 0xF);\n    *im = sext4(byte & 0xF);",
                        "*im = sext4((byte >> 4) & 0xF);\n    *re = sext4(byte & 0xF);"),
    "no_sign_extend": ("return (code & 0x8) ? code - 16 : code;", "return code;"),
    "no_autos": ("for (int32_t j = 0; j <= i; ++j) {\n                        vi[2 * j]",
                 "for (int32_t j = 0; j < i; ++j) {\n                        vi[2 * j]"),
    # row start i(i-1)/2 instead of i(i+1)/2: every index stays in bounds
    "index_off": ("return (int64_t)i * (i + 1) / 2 + j;", "return (int64_t)i * (i - 1) / 2 + j;"),
    "row_stride": ("const uint8_t *row = v + (t * F + f) * (int64_t)N;",
                   "const uint8_t *row = v + (f * T + t) * (int64_t)N;"),
    "conj_on_i": ("vi[2 * j + 1] += (int64_t)(b[i] * a[j] - a[i] * b[j]);",
                  "vi[2 * j + 1] += (int64_t)(a[i] * b[j] - b[i] * a[j]);"),
}


def build_mutant(tmp_path, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", str(so), str(path)])
    L = ctypes.CDLL(str(so))
    L.oracle_accumulate_i4.argtypes = [ctypes.POINTER(ctypes.c_uint8), ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                       ctypes.c_int]
    return L


def run(L, v):
    T, F, N = v.shape
    acc = np.zeros((F, N * (N + 1) // 2, 2), dtype=np.int64)
    v = np.ascontiguousarray(v)
    L.oracle_accumulate_i4(v.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), T, F, N, 0, F,
                           acc.ctypes.data, 1)
    return acc


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, rng, name):
    L = build_mutant(tmp_path, name)
    caught = []
    for ex_name, v, expect in hand_examples():
        if not np.array_equal(run(L, v), expect):
            caught.append(ex_name)
    v = random_bytes(rng, 24, 3, 6)
    T, F, N = v.shape
    if not np.array_equal(full_matrix(run(L, v), N), brute_force(v)):
        caught.append("brute_force")
    assert caught, f"mutant {name} survived every pin"
