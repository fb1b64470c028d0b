"""Planted mistakes in the F-stage oracles must be caught by their pins.

Each case copies one oracle module's source (channeliser, requantiser and
gain update, packet ingest), plants one plausible mistake (a wrong window,
a reversed tap order, a missing conjugate, a sign, an index off by one,
rounding half up, a swapped field or nibble, a lost filter), loads the copy
as a module and runs that oracle's pin tests against it: at least one pin
must fail.  CPU only; the product path is not involved.
"""
import inspect
import os
import types

import pytest

import oracle
from tests import test_channelise_oracle as TC
from tests import test_ingest_oracle as TI
from tests import test_requant_oracle as TR

ORACLE_DIR = os.path.dirname(oracle.__file__)

# (source file, pin module, name the pins use for the oracle module, mutations)
CASES = {
    "channelise": ("channelise.py", TC, "C", {
        "hann_window": ("w = 0.54 - 0.46 * np.cos(", "w = 0.5 - 0.5 * np.cos("),
        "sinc_off_centre": ("np.sinc((m - taps * L / 2.0) / L)", "np.sinc((m - taps * L / 2.0 + 1) / L)"),
        "taps_reversed": ("v += h[p][None, None, :] * blocks[:, p:p + S, :]",
                          "v += h[taps - 1 - p][None, None, :] * blocks[:, p:p + S, :]"),
        "one_spectrum_short": ("return max(0, n_samples // L - taps + 1)", "return max(0, n_samples // L - taps)"),
        "eq1_inputs_swapped": ("y = v[0::2] + 1j * v[1::2]", "y = v[1::2] + 1j * v[0::2]"),
        "eq2_no_conjugate": ("Yr = np.conj(np.roll(Y[..., ::-1], 1, axis=-1))", "Yr = np.roll(Y[..., ::-1], 1, axis=-1)"),
        "eq2_mirror_off_by_one": ("Yr = np.conj(np.roll(Y[..., ::-1], 1, axis=-1))",
                                  "Yr = np.conj(np.roll(Y[..., ::-1], 0, axis=-1))"),
        "eq2_sign": ("X2 = (Y - Yr) / 2.0j", "X2 = (Yr - Y) / 2.0j"),
        "channels_shifted": ("out[0::2], out[1::2] = X1[..., :F], X2[..., :F]",
                             "out[0::2], out[1::2] = X1[..., 1:F + 1], X2[..., 1:F + 1]"),
    }),
    "requant": ("requant.py", TR, "R", {
        "round_half_up": ("up = (rem > HALF) | ((rem == HALF) & ((base & 1) == 1))", "up = rem >= HALF"),
        "saturate_at_minus8": ("return np.clip(base + up.astype(np.int64), -7, 7)",
                               "return np.clip(base + up.astype(np.int64), -8, 7)"),
        "lsb_one_bit_low": ("FRAC_SHIFT = 21 ", "FRAC_SHIFT = 20 "),
        "nibbles_swapped": ("(((qr & 0xF) << 4) | (qi & 0xF))", "(((qi & 0xF) << 4) | (qr & 0xF))"),
        "word_fields_swapped": (
            "return sext18((w >> np.uint64(18)).astype(np.int64)), sext18((w & np.uint64(0x3FFFF)).astype(np.int64))",
            "return sext18((w & np.uint64(0x3FFFF)).astype(np.int64)), sext18((w >> np.uint64(18)).astype(np.int64))"),
        "no_sign_extension": ("return x - ((x >> 17) << 18)", "return x"),
        "gain_high_bits_kept": ("p = np.asarray(d, dtype=np.int64) * (np.asarray(g, dtype=np.int64) & 0x3FFFF)",
                                "p = np.asarray(d, dtype=np.int64) * np.asarray(g, dtype=np.int64)"),
        "eq_update_rms_without_2": ("M = (8 * G * G * target_x16 * target_x16 * n_integrated) // (P * 256)",
                                    "M = (4 * G * G * target_x16 * target_x16 * n_integrated) // (P * 256)"),
        "eq_update_rounds_down": ("k = (math.isqrt(M) + 1) // 2", "k = math.isqrt(M) // 2"),
    }),
    "ingest": ("ingest.py", TI, "I", {
        "mcnt_little_endian": ('return int.from_bytes(h[:6], "big"), h[6], h[7]',
                               'return int.from_bytes(h[:6], "little"), h[6], h[7]'),
        "fid_xid_swapped": ('return int.from_bytes(h[:6], "big"), h[6], h[7]',
                            'return int.from_bytes(h[:6], "big"), h[7], h[6]'),
        "first_duplicate_wins": ("        idx[m - mcnt0, fid] = p\n",
                                 "        if idx[m - mcnt0, fid] < 0:\n            idx[m - mcnt0, fid] = p\n"),
        "other_bands_kept": ("if x != xid or fid >= n_boards or", "if fid >= n_boards or"),
        "window_one_past": ("not (mcnt0 <= m < mcnt0 + n_blocks)", "not (mcnt0 <= m <= mcnt0 + n_blocks)"),
        "payload_channel_input_swapped": (
            "data = packets[p, HEADER:HEADER + pay].reshape(TIMES, n_chans, BOARD_INPUTS)",
            "data = packets[p, HEADER:HEADER + pay].reshape(TIMES, BOARD_INPUTS, n_chans).transpose(0, 2, 1)"),
    }),
}


def mutant_module(oracle_name, mutation):
    fname, _, _, muts = CASES[oracle_name]
    old, new = muts[mutation]
    with open(os.path.join(ORACLE_DIR, fname)) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"mutation site of {mutation} not found exactly once"
    mod = types.ModuleType(f"mutant_{oracle_name}_{mutation}")
    exec(compile(src.replace(old, new), f"<{mutation}>", "exec"), mod.__dict__)
    return mod


def pin_calls(pins):
    """Every pin test of a module, parametrised ones over their cases."""
    calls = []
    for name in sorted(n for n in dir(pins) if n.startswith("test_")):
        fn = getattr(pins, name)
        params = list(inspect.signature(fn).parameters)
        if not params:
            calls.append((name, fn))
        elif params == ["m"]:
            marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
            for v in marks[0].args[1]:
                calls.append((f"{name}[{v}]", lambda fn=fn, v=v: fn(v)))
        else:
            raise AssertionError(f"pin {name} takes parameters this harness does not supply")
    return calls


@pytest.mark.parametrize("oracle_name,mutation",
                         [(o, m) for o, case in CASES.items() for m in sorted(case[3])])
def test_fstage_mutant_is_caught(monkeypatch, oracle_name, mutation):
    _, pins, attr, _ = CASES[oracle_name]
    monkeypatch.setattr(pins, attr, mutant_module(oracle_name, mutation))
    caught = []
    for name, call in pin_calls(pins):
        try:
            call()
        except Exception:      # an assertion or a shape error: the pin rejects the mutant
            caught.append(name)
    assert caught, f"{oracle_name} mutant {mutation} survived every pin"


@pytest.mark.parametrize("oracle_name", sorted(CASES))
def test_unmutated_oracle_passes_every_pin(oracle_name):
    """The harness itself: the oracle as committed passes all its pins."""
    _, pins, _, _ = CASES[oracle_name]
    for name, call in pin_calls(pins):
        call()
