"""Packet ingest and corner turn (paper Sec. 2.3) on the GPU: bit-exact
against the CPU oracle with shuffled, lost, duplicated and foreign packets,
at the paper's packet size and at a large block, and end to end into the
X-engine."""
import numpy as np
import pytest

import oracle
import synth
from oracle import ingest as I
from tests.gpu_util import first_mismatch, gpu_available

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]


def messy_buffer(rng, blk, mcnt0, xid, stride=None):
    pk = synth.packets(blk, mcnt0, xid, stride)
    n = len(pk)
    keep = rng.permutation(n)[: n - max(1, n // 10)]              # ~10% lost, shuffled
    dup = pk[rng.integers(0, n, size=3)].copy()
    dup[:, 8:] = rng.integers(0, 256, size=dup[:, 8:].shape, dtype=np.uint8)
    junk = synth.packets(rng.integers(0, 256, size=(16,) + blk.shape[1:], dtype=np.uint8), mcnt0, xid + 1, stride)
    stale = synth.packets(rng.integers(0, 256, size=(16,) + blk.shape[1:], dtype=np.uint8), mcnt0 - 2, xid, stride)
    # the two time blocks right after the block assembled (ignored)
    past = synth.packets(rng.integers(0, 256, size=(16,) + blk.shape[1:], dtype=np.uint8),
                         mcnt0 + blk.shape[0] // 8, xid, stride)
    return np.concatenate([pk[keep], junk, dup, stale, past, pk[keep[:2]]])


@pytest.mark.parametrize("blocks,boards,chans,stride", [(4, 1, 32, None), (9, 6, 32, None), (5, 8, 16, None),
                                                        (3, 2, 32, 8216), (1, 3, 5, None),
                                                        (2, 4, 7, None), (3, 8, 5, 8216)])
def test_messy_packets_match_oracle(blocks, boards, chans, stride):
    import torch
    from paper_1904_07778_amd.xeng import ingest
    print(f"ingest blocks={blocks} boards={boards} chans={chans} stride={stride}", flush=True)
    rng = np.random.default_rng(blocks * 100 + boards * 10 + chans)
    blk = rng.integers(0, 256, size=(8 * blocks, chans, 32 * boards), dtype=np.uint8)
    buf = messy_buffer(rng, blk, 1 << 40, 5, stride)
    out, idx = ingest(torch.from_numpy(buf).cuda(), 1 << 40, blocks, boards, chans, 5)
    torch.cuda.synchronize()
    want, widx = I.assemble(buf, 1 << 40, blocks, boards, chans, 5)
    assert np.array_equal(idx.cpu().numpy(), widx)
    assert np.array_equal(out.cpu().numpy(), want), first_mismatch(out.cpu().numpy(), want)


def test_no_packets_gives_zeros_and_full_loss():
    import torch
    from paper_1904_07778_amd.xeng import ingest
    print("ingest empty", flush=True)
    out, idx = ingest(torch.empty((0, 8 + 8 * 32 * 32), dtype=torch.uint8, device="cuda"), 0, 2, 2, 32, 0)
    torch.cuda.synchronize()
    assert not out.any() and bool((idx == -1).all())


def test_large_block_and_into_the_x_engine():
    """192 inputs (6 boards), 32 channels (one band of 1024), 8192 samples:
    the block a node integrates; packets shuffled with losses; then the
    X-engine on it against the oracle."""
    import torch
    from paper_1904_07778_amd.xeng import Plan, ingest
    blocks, boards, chans = 1024, 6, 32
    print("ingest large", flush=True)
    rng = np.random.default_rng(77)
    blk = synth.voltages("sources", 9, 32 * boards, chans, 8 * blocks)
    buf = messy_buffer(rng, blk, 123456, 2)
    out, idx = ingest(torch.from_numpy(buf).cuda(), 123456, blocks, boards, chans, 2)
    with Plan([(32 * boards, chans, 8 * blocks)]) as p:
        p.correlate([out])
        vis, n = p.dump(to_host=True)
    torch.cuda.synchronize()
    want, widx = I.assemble(buf, 123456, blocks, boards, chans, 2)
    assert np.array_equal(idx.cpu().numpy(), widx)
    assert np.array_equal(out.cpu().numpy(), want)
    ov = oracle.correlate(np.ascontiguousarray(want[:, [0, 17, 31]]))
    assert np.array_equal(vis[0].numpy()[[0, 17, 31]], ov)
