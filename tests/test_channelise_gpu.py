"""F-stage channeliser (paper Sec. 2.1, Eq. 1-2) on the GPU against the
float64 oracle.  Float32 arithmetic: the tolerance is 2e-5 of the largest
spectral magnitude of each case (about 11 FFT stages and a 4-tap sum of
int8 samples, each rounding at 2^-24 relative)."""
import numpy as np
import pytest

from oracle import channelise as C
from tests.gpu_util import gpu_available

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

TOL = 2e-5


def run(x, F):
    import torch
    from paper_1904_07778_amd.xeng import channelise
    out = channelise(torch.from_numpy(x).cuda(), F)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("N,F,spectra", [(2, 8, 1), (2, 64, 5), (6, 256, 7), (4, 512, 3), (8, 1024, 4),
                                         (192, 1024, 2), (10, 128, 33), (2, 1024, 9), (10, 512, 17),
                                         (14, 256, 12), (4, 1024, 8), (6, 1024, 23)])
def test_random_adc_matches_oracle(N, F, spectra):
    print(f"channelise N={N} F={F} spectra={spectra}", flush=True)
    rng = np.random.default_rng(N * 1000 + F + spectra)
    S_in = 2 * F * (spectra + 3)
    x = rng.integers(-128, 128, size=(N, S_in)).astype(np.int8)
    got = run(x, F)
    want = C.channelise(x, F)
    assert got.shape == want.shape
    err = np.abs(got - want).max()
    assert err <= TOL * np.abs(want).max(), (err, np.abs(want).max())


@pytest.mark.parametrize("N,F,S", [(192, 1024, 8192), (32, 1024, 40037), (16, 512, 20011), (12, 256, 9001)])
def test_full_size_sampled_spectra(N, F, S):
    """Full-size inputs (the cylinder shape first): the longest runs of
    spectra per workgroup, ragged last runs, runs whose length is not a
    multiple of four, every line group of pairs.  Sampled spectra and pairs
    (first and last of runs, first and last pair of line groups) against the
    oracle on exactly the samples each spectrum reads."""
    import torch
    from paper_1904_07778_amd.xeng import channelise
    print(f"channelise full size N={N} F={F} S={S}", flush=True)
    L = 2 * F
    g = torch.Generator(device="cuda")
    g.manual_seed(N * 7919 + S)
    x = torch.randint(-128, 128, (N, (S + 3) * L), dtype=torch.int8, device="cuda", generator=g)
    out = channelise(x, F)
    torch.cuda.synchronize()
    assert tuple(out.shape) == (S, F, N)
    pairs = N // 2
    rng = np.random.default_rng(S)
    spectra = sorted({0, 1, 3, 4, 6, 7, 19, 20, 63, 64, 65, S // 2, S - 2, S - 1} | set(rng.integers(0, S, 6).tolist()))
    qs = sorted({0, 1, 7 % pairs, 8 % pairs, pairs - 1} | set(rng.integers(0, pairs, 3).tolist()))
    worst = 0.0
    for s in spectra:
        if s >= S:
            continue
        for q in qs:
            xs = x[2 * q:2 * q + 2, s * L:(s + 4) * L].cpu().numpy()
            want = C.channelise(xs, F)[0]                      # [F][2]
            got = out[s, :, 2 * q:2 * q + 2].cpu().numpy()
            err = np.abs(got - want).max() / np.abs(want).max()
            worst = max(worst, err)
            assert err <= TOL, (s, q, err)
    print(f"worst relative error {worst:.2e}", flush=True)


def test_tones_and_extremes():
    print("channelise tones", flush=True)
    F = 1024
    L = 2 * F
    n = np.arange(L * 8)
    x = np.stack([np.round(127 * np.cos(2 * np.pi * 100.25 * n / L)),
                  np.full(n.shape, -128), np.full(n.shape, 127),
                  np.round(60 * np.sin(2 * np.pi * 1023 * n / L))]).astype(np.int8)
    got = run(x, F)
    want = C.channelise(x, F)
    assert np.abs(got - want).max() <= TOL * np.abs(want).max()
    assert np.argmax(np.abs(got[0, :, 0])) == 100 and np.argmax(np.abs(got[0, :, 3])) == 1023


def test_samples_short_of_one_spectrum():
    import torch
    from paper_1904_07778_amd.xeng import channelise
    out = channelise(torch.zeros((2, 2 * 64 * 3), dtype=torch.int8, device="cuda"), 64)
    torch.cuda.synchronize()
    assert tuple(out.shape) == (0, 64, 2)
