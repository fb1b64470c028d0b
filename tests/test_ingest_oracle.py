"""Pins of the packet-ingest oracle (paper Sec. 2.3), on the CPU: the header
layout, Eq. 4's packet size, round trip of a block through packets in any
order, and loss, duplicates and foreign packets."""
import numpy as np

import synth
from oracle import ingest as I


def test_header_layout_and_packet_size():
    blk = np.arange(8 * 32 * 32, dtype=np.uint32).astype(np.uint8).reshape(8, 32, 32)
    pk = synth.packets(blk, mcnt0=0x0102030405, xid=7)
    assert pk.shape == (1, 8 + 32 * 32 * 8)
    # Eq. 4: 32 channels x 32 inputs x 8 times + header (8) + CRC (8) = 8208 bytes
    assert pk.shape[1] + 8 == 8208
    assert I.parse_header(pk[0]) == (0x0102030405, 0, 7)
    assert list(pk[0, :8]) == [0x00, 0x01, 0x02, 0x03, 0x04, 0x05, 0, 7]


def test_round_trip_any_order():
    rng = np.random.default_rng(2)
    blk = rng.integers(0, 256, size=(8 * 5, 16, 96), dtype=np.uint8)
    pk = synth.packets(blk, mcnt0=1000, xid=3)
    out, idx = I.assemble(pk[rng.permutation(len(pk))], 1000, 5, 3, 16, 3)
    assert np.array_equal(out, blk) and (idx >= 0).all()


def test_loss_duplicates_and_foreign_packets():
    rng = np.random.default_rng(3)
    blk = rng.integers(0, 256, size=(8 * 4, 32, 64), dtype=np.uint8)
    pk = synth.packets(blk, mcnt0=50, xid=1)
    keep = [p for p in range(len(pk)) if p != 3]              # (mcnt 51, board 1) lost
    foreign = synth.packets(rng.integers(0, 256, size=(8, 32, 64), dtype=np.uint8), 50, xid=2)
    late = synth.packets(rng.integers(0, 256, size=(8, 32, 64), dtype=np.uint8), 60, xid=1)
    # the first time block past the block assembled (MCNT 54) is ignored too
    edge = synth.packets(rng.integers(0, 256, size=(8, 32, 64), dtype=np.uint8), 54, xid=1)
    dup = pk[[0]].copy()
    dup[0, 8:] = 0xAB                                          # a later copy of (50, board 0)
    buf = np.concatenate([pk[keep], foreign, late, edge, dup])
    out, idx = I.assemble(buf, 50, 4, 2, 32, 1)
    want = blk.copy()
    want[8:16, :, 32:64] = 0                                   # the lost packet reads as zeros
    want[0:8, :, 0:32] = 0xAB                                  # the later duplicate wins
    assert np.array_equal(out, want)
    assert (idx == -1).sum() == 1 and idx[1, 1] == -1
