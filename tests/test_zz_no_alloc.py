"""The allocation-free channeliser entry point (xeng_channelise_noalloc)
against the entry point that takes a table workspace (xeng_channelise), on
two calls in a row, the second with a smaller input: the same kernels on the
same tables, so the spectra must be identical; the first call is also
checked against the float64 oracle (paper Sec. 2.1, Eq. 1-2) within the
channeliser's float32 tolerance."""
import numpy as np
import pytest

from oracle import channelise as C
from tests.gpu_util import gpu_available

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]

TOL = 2e-5


def test_noalloc_matches_workspace_entry_point_twice():
    import torch
    from paper_1904_07778_amd import xeng as X
    rng = np.random.default_rng(4242)
    cases = [(16, 1024, 6), (6, 128, 9)]          # (inputs, channels, spectra); the second is smaller
    for k, (N, F, spectra) in enumerate(cases):
        print(f"noalloc channelise call {k}: N={N} F={F} spectra={spectra}", flush=True)
        S_in = 2 * F * (spectra + 3)
        x = rng.integers(-128, 128, size=(N, S_in)).astype(np.int8)
        adc = torch.from_numpy(x).cuda()
        stream = torch.cuda.current_stream()
        want = torch.empty((spectra, F, N), dtype=torch.complex64, device="cuda")
        tables = torch.empty(int(X._lib.xeng_channelise_table_floats(F)), dtype=torch.float32, device="cuda")
        X.xeng_channelise(adc, S_in, N, F, want, tables, stream)
        got = torch.full((spectra, F, N), float("nan"), dtype=torch.complex64, device="cuda")
        X.xeng_channelise_noalloc(adc, S_in, N, F, got, stream)
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"call {k}: noalloc differs from the workspace entry point"
        if k == 0:
            ref = C.channelise(x, F)
            g = got.cpu().numpy()
            assert np.abs(g - ref).max() <= TOL * np.abs(ref).max()


def test_noalloc_rejects_spectra_beyond_its_scratch():
    import torch
    from paper_1904_07778_amd import xeng as X
    adc = torch.zeros((2, 2 * 2048 * 4), dtype=torch.int8, device="cuda")
    out = torch.empty((1, 2048, 2), dtype=torch.complex64, device="cuda")
    with pytest.raises(X.XengError) as ei:
        X.xeng_channelise_noalloc(adc, adc.shape[1], 2, 2048, out, torch.cuda.current_stream())
    assert ei.value.status == X.XENG_EINVAL
