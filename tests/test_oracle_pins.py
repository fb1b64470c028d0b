"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: a hand-worked example, an
exhaustive enumeration, brute force through an independent decoder and
numpy, an exact algebraic invariant of the definition, the FX == XF identity
the paper states, the paper's delay experiment (Eq. 5) reproduced on
synthetic data, or the RMS relation of Eq. 3.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.golden.fixtures import hand_examples


# ---------------------------------------------------------------- helpers
def independent_decode(v):
    """4-bit two's complement via int8 arithmetic shifts (no table, no oracle)."""
    v = np.asarray(v, dtype=np.uint8)
    re = v.view(np.int8) >> 4
    im = (v << 4).astype(np.uint8).view(np.int8) >> 4
    return re.astype(np.int64), im.astype(np.int64)


def brute_force(v):
    """Full Hermitian matrix by numpy einsum over complex values, per channel."""
    re, im = independent_decode(v)
    x = re + 1j * im
    return np.einsum("tfi,tfj->fij", x, np.conj(x))


def full_matrix(tri, n):
    """Lower-triangle natural-order visibilities -> full N x N complex matrix."""
    F = tri.shape[0]
    m = np.zeros((F, n, n), dtype=np.complex128)
    k = 0
    for i in range(n):
        for j in range(i + 1):
            m[:, i, j] = tri[:, k, 0] + 1j * tri[:, k, 1]
            m[:, j, i] = np.conj(m[:, i, j])
            k += 1
    return m


def random_bytes(rng, T, F, N, allow_minus8=True):
    lo = -8 if allow_minus8 else -7
    re = rng.integers(lo, 8, size=(T, F, N))
    im = rng.integers(lo, 8, size=(T, F, N))
    return synth.pack(re, im)


# ---------------------------------------------------------- golden values
@pytest.mark.parametrize("name,v,expect", hand_examples(), ids=lambda x: x if isinstance(x, str) else "")
def test_hand_worked_examples(name, v, expect):
    got = oracle.accumulate(v)
    np.testing.assert_array_equal(got, expect, err_msg=name)


def test_decode_exhaustive_256_codes():
    # Two's complement of a 4-bit code c: c for c < 8, c - 16 otherwise
    # (fix_4_3 range 1.000b..0.111b in units of 1/8, Sec. 2.1).
    def tc4(c):
        return c if c < 8 else c - 16
    for b in range(256):
        assert oracle.decode(b) == (tc4(b >> 4), tc4(b & 0xF)), hex(b)


def test_baseline_index_enumeration():
    # Natural order of Sec. 2.3: input i against inputs 0..i, rows in turn.
    k = 0
    for i in range(40):
        for j in range(i + 1):
            assert oracle.baseline_index(i, j) == k
            k += 1
        assert oracle.nbaselines(i + 1) == k
        assert oracle.baseline_index(i, i + 1) == -1
    assert oracle.nbaselines(192) == 18528


# -------------------------------------------------------------- brute force
@pytest.mark.parametrize("T,F,N", [(1, 1, 1), (7, 3, 5), (64, 4, 8), (33, 2, 7)])
def test_brute_force_einsum(rng, T, F, N):
    v = random_bytes(rng, T, F, N)
    got = full_matrix(oracle.accumulate(v), N)
    want = brute_force(v)
    np.testing.assert_array_equal(got, want)


def test_channel_subset_matches_full(rng):
    v = random_bytes(rng, 40, 6, 5)
    full = oracle.accumulate(v)
    part = oracle.accumulate(v, chans=(2, 5))
    np.testing.assert_array_equal(part, full[2:5])


# ----------------------------------------------------------- invariants
def test_autos_real_nonnegative_and_hermitian(rng):
    N = 9
    v = random_bytes(rng, 50, 3, N)
    tri = oracle.accumulate(v)
    for i in range(N):
        k = oracle.baseline_index(i, i)
        assert np.all(tri[:, k, 1] == 0)
        assert np.all(tri[:, k, 0] >= 0)
    m = full_matrix(tri, N)
    np.testing.assert_array_equal(m, np.conj(np.swapaxes(m, 1, 2)))


def test_identical_inputs_closed_form(rng):
    # x_i == x_j  =>  V_ij = V_ii = V_jj = sum_t |x|^2 (a closed form).
    T, F, N = 37, 2, 4
    v = random_bytes(rng, T, F, N)
    v[:, :, 2] = v[:, :, 0]
    tri = oracle.accumulate(v)
    re, im = independent_decode(v[:, :, 0])
    power = (re * re + im * im).sum(axis=0)                      # [F]
    for k in (oracle.baseline_index(0, 0), oracle.baseline_index(2, 0), oracle.baseline_index(2, 2)):
        np.testing.assert_array_equal(tri[:, k, 0], power)
        np.testing.assert_array_equal(tri[:, k, 1], 0)


def test_linearity_over_split_integration(rng):
    v = random_bytes(rng, 90, 3, 6)
    e = oracle.Engine(6, 3)
    e.correlate(v[:31])
    e.correlate(v[31:])
    vis, n = e.dump()
    assert n == 90
    np.testing.assert_array_equal(vis, oracle.correlate(v))
    vis2, n2 = e.dump()
    assert n2 == 0 and not vis2.any()


def test_permutation_equivariance(rng):
    N = 7
    v = random_bytes(rng, 20, 2, N)
    perm = rng.permutation(N)
    m = full_matrix(oracle.accumulate(v), N)
    mp = full_matrix(oracle.accumulate(v[:, :, perm]), N)
    np.testing.assert_array_equal(mp, m[:, perm][:, :, perm])


def test_rotation_by_j_and_global_negation(rng):
    # Inputs in [-7, 7] so that rotation and negation stay representable.
    N, p = 6, 3
    v = random_bytes(rng, 25, 2, N, allow_minus8=False)
    re, im = independent_decode(v)
    m = full_matrix(oracle.accumulate(v), N)
    # x_p -> j x_p, i.e. (a, b) -> (-b, a)
    re2, im2 = re.copy(), im.copy()
    re2[:, :, p], im2[:, :, p] = -im[:, :, p], re[:, :, p]
    mr = full_matrix(oracle.accumulate(synth.pack(re2, im2)), N)
    want = m.copy()
    want[:, p, :] *= 1j          # V_pj = x_p conj(x_j) gains a factor j
    want[:, :, p] *= -1j         # V_ip = x_i conj(x_p) gains a factor -j
    np.testing.assert_array_equal(mr, want)
    mn = full_matrix(oracle.accumulate(synth.pack(-re, -im)), N)
    np.testing.assert_array_equal(mn, m)


def test_int32_bound_of_the_integration():
    # All codes -8 add 128 per sample to an auto: T = floor((2^31-1)/128)
    # samples still fit int32, one more does not.
    tmax = oracle.T_MAX_EXACT
    assert tmax == 16_777_215
    v = np.full((tmax, 1, 1), 0x88, dtype=np.uint8)
    acc = oracle.accumulate(v)
    assert acc[0, 0, 0] == 128 * tmax
    oracle.to_int32(acc)
    acc = oracle.accumulate(v[:1], acc)
    with pytest.raises(OverflowError):
        oracle.to_int32(acc)


def test_integer_and_float_forms_agree(rng):
    v = random_bytes(rng, 30, 3, 5)
    re, im = independent_decode(v)
    c = oracle.accumulate_c128(re + 1j * im)
    i = oracle.accumulate(v)
    np.testing.assert_array_equal(c.real, i[..., 0])
    np.testing.assert_array_equal(c.imag, i[..., 1])


# --------------------------------------------------------------- FX == XF
def test_fx_equals_xf_float64(rng):
    """Sec. 2: multiplying in frequency equals convolving in time, so FX and
    XF give identical visibilities.  Exact for circular lags within each
    block of L samples: the XF side forms the lag correlation
    r_ij[tau] = sum_b sum_m x_i[bL + (m+tau) mod L] conj(x_j[bL + m]) and
    Fourier-transforms it over tau (explicit sums, no FFT); the FX side
    channelises each block with a DFT and runs the oracle."""
    L, B, N = 16, 5, 4
    x = rng.standard_normal((N, B * L)) + 1j * rng.standard_normal((N, B * L))
    blocks = x.reshape(N, B, L)
    X = np.fft.fft(blocks, axis=2)                     # [N, B, L]  F-engine
    fx = oracle.accumulate_c128(np.transpose(X, (1, 2, 0)))   # [time=B][chan=L][input]
    tau = np.arange(L)
    m = np.arange(L)
    dft = np.exp(-2j * np.pi * np.outer(np.arange(L), tau) / L)   # [k, tau]
    scale = np.abs(fx).max()
    k = 0
    for i in range(N):
        for j in range(i + 1):
            r = np.zeros(L, dtype=np.complex128)
            for t in tau:
                r[t] = np.sum(blocks[i][:, (m + t) % L] * np.conj(blocks[j][:, m]))
            xf = dft @ r
            assert np.max(np.abs(fx[:, k] - xf)) <= 1e-9 * scale, (i, j)
            k += 1


# ------------------------------------------------- delay experiment (Eq. 5)
def test_delay_gives_linear_phase_slope():
    """Sec. 3, Eq. 5: a common signal with a relative delay tau gives a
    visibility phase linear in frequency with slope magnitude 2 pi tau.  The
    paper's cable: L = 7.5 m at v = 0.7c.  Channel f of an F-channel
    spectrum of the 125 MHz band sits at f * 125 MHz / F; input 1 is input 0
    delayed (spectrum times exp(-j 2 pi nu tau)), both with independent
    receiver noise, requantised to 4 bits.  With V_10 = x_1 conj(x_0) the
    slope is -2 pi tau."""
    tau = 7.5 / (0.7 * 299_792_458.0)
    F, T = 256, 512
    nu = np.arange(F) * 125e6 / F
    r = np.random.default_rng(5)
    s = (r.standard_normal((T, F)) + 1j * r.standard_normal((T, F))) * 2.0
    n0 = (r.standard_normal((T, F)) + 1j * r.standard_normal((T, F))) * 0.7
    n1 = (r.standard_normal((T, F)) + 1j * r.standard_normal((T, F))) * 0.7
    x0 = s + n0
    x1 = s * np.exp(-2j * np.pi * nu * tau)[None, :] + n1
    v = np.stack([synth.pack(synth.quantise(x0.real), synth.quantise(x0.imag)),
                  synth.pack(synth.quantise(x1.real), synth.quantise(x1.imag))], axis=-1)
    tri = oracle.accumulate(v)
    k10 = oracle.baseline_index(1, 0)
    phase = np.unwrap(np.arctan2(tri[:, k10, 1], tri[:, k10, 0]).astype(np.float64))
    slope, icpt = np.polyfit(nu, phase, 1)
    assert abs(slope / (-2 * np.pi * tau) - 1) < 0.01
    resid = phase - (slope * nu + icpt)
    assert np.max(np.abs(resid)) < 0.2


# ------------------------------------------------------- statistics (Eq. 3)
def test_uniform_autos_closed_form_mean():
    # re, im iid uniform on {-7..7}: E|x|^2 = 2 * (15^2 - 1) / 12 = 37.33...
    w = synth.WORKLOADS["dish_tiny"]
    v = synth.voltages(w["recipe"], w["seed"], w["n_inputs"], 8, w["n_time"])
    tri = oracle.accumulate(v)
    autos = np.array([tri[:, oracle.baseline_index(i, i), 0] for i in range(w["n_inputs"])])
    mean = autos.mean() / w["n_time"]
    assert abs(mean / (2 * (15**2 - 1) / 12) - 1) < 0.01


@pytest.mark.parametrize("wname,pred", [("dish", (6.25 + 0.5**2 * 6.25 / 2 + 1 / 12) ** 0.5),
                                         ("cylinder", (6.25 * (1 + (0.5**2 + 0.35**2 + 0.25**2) / 2) + 1 / 12) ** 0.5)])
def test_rms_from_autocorrelation_eq3(wname, pred):
    """Eq. 3: RMS = sqrt(P / 2N) from the integrated auto P over N samples;
    the paper's 4-bit data sit at an RMS of 2 to 3 out of +-7.  Predicted
    RMS per component: sqrt(sigma^2 + sum A^2/2 + 1/12) before clipping."""
    w = synth.WORKLOADS[wname]
    T = 2048
    v = synth.voltages(w["recipe"], w["seed"], w["n_inputs"], 4, T)
    tri = oracle.accumulate(v)
    autos = np.array([tri[:, oracle.baseline_index(i, i), 0] for i in range(w["n_inputs"])])
    rms = np.sqrt(autos / (2 * T))
    assert 2.0 <= rms.mean() <= 3.0
    assert abs(rms.mean() / pred - 1) < 0.03
