"""Equaliser / 4-bit requantiser (paper Sec. 2.1) on the GPU: bit-exact
against the CPU oracle on both kernel paths, on the rounding ties and the
saturation edges, at full size on sampled rows, and end to end into the
X-engine."""
import numpy as np
import pytest

import oracle
import synth
from oracle import requant as R
from tests.gpu_util import first_mismatch, gpu_available

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]


def random_words(rng, T, F, N):
    # every bit random: full 18-bit fields and junk in bits 36..63
    return rng.integers(0, 2**63, size=(T, F, N), dtype=np.int64).view(np.uint64) ^ \
        (rng.integers(0, 2, size=(T, F, N), dtype=np.int64).view(np.uint64) << np.uint64(63))


def run(words, gains, out_offset=0):
    import torch
    from paper_1904_07778_amd.xeng import requantize
    w = torch.from_numpy(np.ascontiguousarray(words).view(np.int64)).cuda()
    g = torch.from_numpy(np.ascontiguousarray(gains).view(np.int32)).cuda()
    if out_offset:
        raw = torch.empty(words.size + out_offset, dtype=torch.uint8, device="cuda")
        out = raw[out_offset:].view(words.shape)
        requantize(w, g, out=out)
    else:
        out = requantize(w, g)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("T,F,N,offset", [(1, 1, 8, 0), (37, 3, 16, 0), (100, 5, 24, 0), (17, 2, 7, 0),
                                           (33, 3, 5, 0), (40, 4, 32, 1), (16, 1, 192, 0), (65, 7, 40, 0)])
def test_random_words_and_gains(T, F, N, offset):
    print(f"requant T={T} F={F} N={N} offset={offset}", flush=True)
    rng = np.random.default_rng(T * 1000 + F * 10 + N)
    words = random_words(rng, T, F, N)
    gains = rng.integers(0, 2**32, size=(F, N), dtype=np.uint64).astype(np.uint32)
    gains[:, ::2] &= 0x7FF                      # half the gains small: unsaturated codes
    got = run(words, gains, offset)
    want = R.requantize(words, gains)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_ties_and_saturation_edges():
    print("requant ties", flush=True)
    m = np.arange(-9, 9)
    d = ((2 * m + 1) << 4)                       # d * 2^16 = (2m + 1) 2^20: half-way
    d = np.concatenate([d, [-(1 << 17), (1 << 17) - 1, 0, 1, -1]])
    T = len(d)
    words = (((d & 0x3FFFF) << 18) | (-d & 0x3FFFF)).astype(np.uint64).reshape(T, 1, 1)
    words = np.repeat(words, 8, axis=2)
    gains = np.array([[1 << 16, 1 << 16, 0x3FFFF, 1, 0, 128, 256, 0xFFFFFFFF]], dtype=np.uint32)
    got = run(words, gains)
    want = R.requantize(words, gains)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_full_size_sampled_rows():
    """Cylinder shape (T=8192, F=1024, N=192): realistic words made on the
    device, checked against the oracle on sampled time rows."""
    import torch
    from paper_1904_07778_amd.xeng import requantize
    T, F, N = 8192, 1024, 192
    print("requant full size", flush=True)
    gen = torch.Generator(device="cuda").manual_seed(5)
    z = torch.randn((T, F, N, 2), device="cuda", generator=gen) * 2.0**14
    v = z.round().clamp(-(2**17), 2**17 - 1).to(torch.int64) & 0x3FFFF
    del z
    words = (v[..., 0] << 18) | v[..., 1]
    del v
    gains_h = synth.eq_gains(5, N, F)
    gains = torch.from_numpy(gains_h.view(np.int32)).cuda()
    out = requantize(words, gains)
    torch.cuda.synchronize()
    for t in (0, 1, 4095, T - 1):
        got = out[t].cpu().numpy()
        want = R.requantize(words[t:t + 1].cpu().numpy().view(np.uint64), gains_h)[0]
        assert np.array_equal(got, want), f"row {t}: " + first_mismatch(got, want)


def test_end_to_end_into_the_x_engine():
    import torch
    from paper_1904_07778_amd.xeng import Plan, requantize
    T, F, N = 2048, 8, 64
    print("requant -> X-engine", flush=True)
    words = synth.pfb_words(6, N, F, T)
    gains = synth.eq_gains(6, N, F)
    w = torch.from_numpy(words.view(np.int64)).cuda()
    g = torch.from_numpy(gains.view(np.int32)).cuda()
    with Plan([(N, F, T)]) as p:
        p.correlate([requantize(w, g)])
        vis, _ = p.dump(to_host=True)
    want = oracle.correlate(R.requantize(words, gains))
    assert np.array_equal(vis[0].numpy(), want), first_mismatch(vis[0].numpy(), want)


def test_eq_update_matches_oracle_on_extremes():
    import torch
    from paper_1904_07778_amd.xeng import eq_update
    rng = np.random.default_rng(41)
    F, N = 7, 33
    nbl = N * (N + 1) // 2
    print("eq_update extremes", flush=True)
    for T in (1, 4096, 16777215):
        vis = rng.integers(-2**31, 2**31 - 1, size=(F, nbl, 2), dtype=np.int64).astype(np.int32)
        autos = [i * (i + 1) // 2 + i for i in range(N)]
        P = rng.integers(1, 2**31 - 1, size=(F, N))
        P[:, :3] = [1, 0, 2**31 - 1]                      # smallest, silent, largest auto power
        vis[:, autos, 0] = P
        gains = rng.integers(0, 2**32, size=(F, N), dtype=np.uint64).astype(np.uint32)
        for tx in (1, 40, 255):
            got = eq_update(torch.from_numpy(vis).cuda(), T, torch.from_numpy(gains.view(np.int32)).cuda(),
                            target_rms=tx / 16).cpu().numpy().view(np.uint32)
            want = R.eq_update(vis, T, gains, tx)
            assert np.array_equal(got, want), f"T={T} tx={tx}: " + first_mismatch(got, want)


def test_closed_loop_brings_rms_into_the_paper_band():
    """F -> X -> gains -> F: start with the 4-bit RMS near 1 on half the
    inputs and near 4.3 (clipping) on the others; one update puts every
    input in the 2..3 band of Sec. 2.1, and it stays there."""
    import torch
    from paper_1904_07778_amd.xeng import Plan, eq_update, requantize
    T, F, N = 4096, 16, 48
    print("closed loop", flush=True)
    words = torch.from_numpy(synth.pfb_words(8, N, F, T, sigma=2.0**12).view(np.int64)).cuda()
    g0 = np.where(np.arange(N) % 2 == 0, 512, 2200).astype(np.int32)   # sigma 2^12: RMS ~1 and ~4.3
    gains = torch.from_numpy(np.tile(g0, (F, 1))).cuda()
    for it in range(3):
        with Plan([(N, F, T)]) as p:
            p.correlate([requantize(words, gains)])
            vis, n = p.dump()
        autos = vis[0][:, [i * (i + 1) // 2 + i for i in range(N)], 0].double()
        rms = torch.sqrt(autos / (2 * T))
        if it > 0:
            assert float(rms.min()) > 2.0 and float(rms.max()) < 3.0, (it, float(rms.min()), float(rms.max()))
        gains = eq_update(vis[0], n[0], gains, target_rms=2.5)
