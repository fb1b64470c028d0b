"""CPU oracle of packet ingest and corner turn (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

Paper Sec. 2.3: each UDP payload starts with an 8-byte application header,
6 bytes of packet counter MCNT (the time sequence), 1 byte Fid (the board
that sent it) and 1 byte Xid (the GPU core, i.e. the band, it is for); the
data are 8 consecutive time samples of the packet's channels (32 for the
1024-point spectrum, 16 for 512) for the board's 32 inputs, in [time,
channel, input] order, one byte per complex sample (Eq. 4: 32 x 32 x 8
bytes of data).  Packet loss shows as a jump in MCNT.  Sec. 2.1/2.2: the
X side needs [time, channel, input] over all boards' inputs.

Readings: MCNT is big-endian (network order) and counts packets of 8 time
samples; the block assembled holds time blocks MCNT0 .. MCNT0 + M - 1; a
packet of another Xid, of a board >= B or of an MCNT outside the block is
ignored; of two packets for the same (MCNT, board) the later one in the
buffer wins; a missing packet leaves zeros (zero samples add nothing to a
correlation) and is reported through the index table (-1).
"""
from __future__ import annotations

import numpy as np

TIMES = 8            # time samples per packet
BOARD_INPUTS = 32    # inputs per board
HEADER = 8


def parse_header(h: bytes | np.ndarray) -> tuple[int, int, int]:
    h = bytes(h[:HEADER])
    return int.from_bytes(h[:6], "big"), h[6], h[7]


def index(packets: np.ndarray, mcnt0: int, n_blocks: int, n_boards: int, xid: int) -> np.ndarray:
    """int32 [n_blocks][n_boards]: packet number of each (time block, board), or -1."""
    idx = np.full((n_blocks, n_boards), -1, dtype=np.int32)
    for p in range(packets.shape[0]):
        m, fid, x = parse_header(packets[p])
        if x != xid or fid >= n_boards or not (mcnt0 <= m < mcnt0 + n_blocks):
            continue
        idx[m - mcnt0, fid] = p
    return idx


def assemble(packets: np.ndarray, mcnt0: int, n_blocks: int, n_boards: int, n_chans: int, xid: int):
    """uint8 [n_blocks * 8][n_chans][n_boards * 32] and the index table."""
    idx = index(packets, mcnt0, n_blocks, n_boards, xid)
    out = np.zeros((n_blocks * TIMES, n_chans, n_boards * BOARD_INPUTS), dtype=np.uint8)
    pay = TIMES * n_chans * BOARD_INPUTS
    for m in range(n_blocks):
        for b in range(n_boards):
            p = idx[m, b]
            if p < 0:
                continue
            data = packets[p, HEADER:HEADER + pay].reshape(TIMES, n_chans, BOARD_INPUTS)
            out[m * TIMES:(m + 1) * TIMES, :, b * BOARD_INPUTS:(b + 1) * BOARD_INPUTS] = data
    return out, idx
