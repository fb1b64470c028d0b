"""Streaming X-engine: a continuous-batching serving loop over the C ABI.

The paper's GPU node runs a chain of threads joined by ring buffers
(Sec. 2.2): a network thread fills a ring with packets of all inputs, the GPU
thread correlates and integrates what the ring holds, and the CPU/disk threads
write out each finished integration.  Packet loss is detected from a counter
carried by every packet (Sec. 2.3).

Here the same chain serves several independent sub-arrays at once on one GPU:

* A sub-array is a request: N inputs, F channels, an integration (dump)
  length and a number of dumps.  It is *admitted* when its HBM footprint
  (accumulator plus its share of the block ring) fits the memory budget, and
  leaves when its last dump is out; requests that arrive meanwhile wait in
  order and are admitted as memory frees up (xeng_attach / xeng_detach on
  one batched plan).
* Voltage blocks (uint8 [1024][F][N]) arrive continuously, each with a
  sequence number: either pre-staged in a device ring (Feed), or in a pinned
  host ring from which a copy stream moves each block into a device ring,
  ordered by events against the engine calls that read it (HostFeed, the
  H2D-inclusive form).  A gap in the numbers is counted as lost samples; the
  integration simply has fewer samples, reported with the dump.
* Each iteration makes ONE xeng_correlate call over every resident slot: the
  blocks a slot has ready (consecutive in its ring, up to its next dump
  boundary) go in as one time range, so queued blocks coalesce into fewer,
  longer items and fewer accumulator passes.  The call is one captured graph
  launch of the persistent batch kernel; work of different sub-arrays
  overlaps on the device.
* A slot whose integration is complete is dumped by the dump kernel into a
  device buffer and copied to pinned host memory on a copy stream; its
  latency runs from the arrival of the dump's last block to the moment the
  visibilities are in host memory (p50 / p99 reported), and to the moment
  they are in the device buffer.

Each sub-array's result is independent of what else shares the GPU (integer
sums; tests check a sub-array alone and in a mix give the same bytes).
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import xeng as X

BLOCK_T = 1024  # samples per channel in one voltage block


@dataclass
class Request:
    """One sub-array to serve."""
    name: str
    n_inputs: int
    n_chans: int
    dump_len: int          # samples per integration
    n_dumps: int           # integrations to deliver before leaving
    ring_blocks: int = 4   # device block ring it brings along (counted in its footprint)

    @property
    def block_bytes(self) -> int:
        return BLOCK_T * self.n_chans * self.n_inputs

    def footprint(self) -> int:
        """HBM bytes held while resident: accumulator + block ring + one dump buffer."""
        acc = X.xeng_accumulator_bytes(self.n_inputs, self.n_chans)
        return 2 * acc + self.ring_blocks * self.block_bytes


@dataclass
class Block:
    seq: int               # sequence number (gaps = lost blocks)
    data: object           # uint8 device tensor [BLOCK_T, F, N] (a row range of a ring)
    ring: object = None    # the ring tensor data is a slice of (for coalescing)
    row: int = 0           # first time row of data in ring
    arrival: float = 0.0   # host time the block became available
    ready: object = None   # event after which data is valid (its host-to-device copy), or None
    on_consumed: object = None  # called with an event recorded after the engine call that read it


@dataclass
class Dump:
    name: str
    index: int
    vis: object            # int32 [F, nbl, 2] pinned host tensor
    n_integrated: int
    lost_samples: int
    latency_ms: float      # last block arrival -> visibilities in host memory
    device_latency_ms: float  # last block arrival -> visibilities in the device buffer


class Admission:
    """First-come admission under a memory budget (host logic only).

    Requests are admitted strictly in arrival order while the head fits:
    a large request is not overtaken by smaller ones behind it."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self.used = 0
        self.waiting: collections.deque[Request] = collections.deque()

    def submit(self, req: Request) -> None:
        if req.footprint() > self.budget:
            raise ValueError(f"{req.name}: footprint {req.footprint()} B exceeds the budget {self.budget} B")
        self.waiting.append(req)

    def admit(self) -> list[Request]:
        out = []
        while self.waiting and self.used + self.waiting[0].footprint() <= self.budget:
            r = self.waiting.popleft()
            self.used += r.footprint()
            out.append(r)
        return out

    def release(self, req: Request) -> None:
        self.used -= req.footprint()
        assert self.used >= 0


@dataclass
class _Slot:
    req: Request
    slot: int
    queue: collections.deque = field(default_factory=collections.deque)
    integrated: int = 0        # samples in the current integration (received)
    covered: int = 0           # samples of the current integration's span (received or lost)
    next_seq: int = 0
    lost: int = 0              # samples lost in the current integration
    last_arrival: float = 0.0
    dumps_done: int = 0
    host_bufs: list = field(default_factory=list)


@dataclass
class _Pending:
    name: str
    index: int
    host: object
    n: int
    lost: int
    t_last: float
    dev_ev: object
    ev: object
    t_dev: float | None = None


class Server:
    """Continuous-batching loop around one batched xeng plan.

    Drive it with submit() (requests), push() (blocks as they arrive) and
    step() (one engine iteration); poll() collects finished dumps."""

    def __init__(self, budget_bytes: int, stream=None, on_admit=None, on_leave=None,
                 keep_results: bool = True):
        """keep_results: hand each dump's visibilities to the caller (a copy of
        the pinned buffer); otherwise only its metadata and timing."""
        import torch
        self.torch = torch
        self.keep_results = keep_results
        self.adm = Admission(budget_bytes)
        self.plan = X.Plan([], stream=stream, batch=True)
        self.copy_stream = torch.cuda.Stream()
        self.slots: dict[str, _Slot] = {}
        self.pending: list[_Pending] = []   # dumps whose host copy is in flight
        self.done: list[Dump] = []
        self.on_admit, self.on_leave = on_admit, on_leave
        self.iterations = 0
        self.cmac = 0                        # useful complex MACs issued

    # -- requests and blocks
    def submit(self, req: Request) -> None:
        self.adm.submit(req)

    def resident(self) -> list[str]:
        return list(self.slots)

    def push(self, name: str, block: Block) -> None:
        s = self.slots[name]
        if block.seq < s.next_seq:
            raise ValueError(f"{name}: block {block.seq} arrived after {s.next_seq - 1}")
        s.queue.append(block)

    # -- one iteration
    def _admit(self) -> None:
        for req in self.adm.admit():
            idx = self.plan.attach(req.n_inputs, req.n_chans, req.dump_len)
            s = _Slot(req, idx)
            torch = self.torch
            nbl = req.n_inputs * (req.n_inputs + 1) // 2
            s.host_bufs = [torch.empty((req.n_chans, nbl, 2), dtype=torch.int32, pin_memory=True)
                           for _ in range(2)]
            self.slots[req.name] = s
            if self.on_admit:
                self.on_admit(req)

    def _take(self, s: _Slot):
        """Blocks of s for this call: consecutive sequence numbers, contiguous
        rows of one ring, not past the dump boundary.  Lost blocks in front of
        the head count toward the span."""
        if not s.queue:
            return None
        head = s.queue[0]
        gap = head.seq - s.next_seq
        if gap > 0:
            # lost blocks: they fill the span of the integration without samples
            room = (s.req.dump_len - s.covered) // BLOCK_T
            lost = min(gap, room)
            s.covered += lost * BLOCK_T
            s.lost += lost * BLOCK_T
            s.next_seq += lost
            if s.covered >= s.req.dump_len:
                return None
        n = 0
        room = (s.req.dump_len - s.covered) // BLOCK_T
        while n < len(s.queue) and n < room:
            b = s.queue[n]
            if b.seq != s.next_seq + n:
                break
            if n > 0:
                p = s.queue[n - 1]
                if b.ring is None or b.ring is not p.ring or b.row != p.row + BLOCK_T:
                    break
            n += 1
        if n == 0:
            return None
        blocks = [s.queue.popleft() for _ in range(n)]
        if n == 1 or blocks[0].ring is None:
            data = blocks[0].data
        else:
            data = blocks[0].ring[blocks[0].row: blocks[0].row + n * BLOCK_T]
        s.next_seq += n
        s.covered += n * BLOCK_T
        s.integrated += n * BLOCK_T
        s.last_arrival = max(b.arrival for b in blocks)
        return data, blocks

    def step(self) -> bool:
        """Admit what fits, correlate every slot's ready blocks in one call,
        dump the slots whose integration is complete.  Returns whether any
        work was issued.

        The iteration runs on the engine's stream, after the caller's current
        stream (which wrote the blocks of a device feed); so the engine's calls
        are in stream order and make no waits between streams."""
        torch = self.torch
        caller = torch.cuda.current_stream()
        if caller == self.plan.stream:
            return self._step()
        self.plan.stream.wait_stream(caller)
        with torch.cuda.stream(self.plan.stream):
            return self._step()

    def _step(self) -> bool:
        self._admit()
        if not self.slots:
            return False
        n_slots = len(self.plan.specs)
        volts = [None] * n_slots
        issued = False
        taken = []
        for s in self.slots.values():
            got = self._take(s)
            if got is not None:
                d, blocks = got
                volts[s.slot] = d
                taken.extend(blocks)
                nbl = s.req.n_inputs * (s.req.n_inputs + 1) // 2
                self.cmac += nbl * s.req.n_chans * d.shape[0]
                issued = True
        for b in taken:                 # blocks still being copied in from host memory
            if b.ready is not None:
                self.plan.stream.wait_event(b.ready)
        fused = {}
        if issued:
            # slots whose integration this block completes are integrated and
            # dumped in the same call, straight into their output buffer
            ending = [s for s in self.slots.values()
                      if volts[s.slot] is not None and s.covered >= s.req.dump_len]
            for s in ending:
                if self.keep_results:
                    self._collect_older(s)
            if ending:
                outs = [None] * n_slots
                for s in ending:
                    outs[s.slot] = self.plan.new_output(s.slot)
                outs, n = self.plan.correlate_dump(volts, out=outs)
                fused = {s.slot: (outs[s.slot], n[s.slot]) for s in ending}
            else:
                self.plan.correlate(volts)
            self.iterations += 1
            if any(b.on_consumed is not None for b in taken):
                ev = self.torch.cuda.Event()
                ev.record(self.plan.stream)
                for b in taken:
                    if b.on_consumed is not None:
                        b.on_consumed(ev)
        for name in list(self.slots):
            s = self.slots[name]
            if s.covered >= s.req.dump_len:
                self._dump(s, fused.get(s.slot))
        return issued

    def _collect_older(self, s: _Slot) -> None:
        """The pinned buffer of dump k-2 is reused by dump k: collect that dump."""
        k = s.dumps_done
        for item in [i for i in self.pending if i.name == s.req.name and i.index == k - 2]:
            self._finish(item, wait=True)

    def _dump(self, s: _Slot, done=None) -> None:
        """Hand dump k of slot s to the copy stream; `done` = (device output,
        samples) when the correlate call already dumped it."""
        torch = self.torch
        k = s.dumps_done
        if self.keep_results:
            self._collect_older(s)
        if done is None:
            out, n = self.plan.dump(s.slot)                  # dump kernel, device buffer
        else:
            out, n = [done[0]], [done[1]]
        dev_ev = torch.cuda.Event()
        dev_ev.record(self.plan.stream)
        host = s.host_bufs[k % 2]
        self.copy_stream.wait_stream(self.plan.stream)
        with torch.cuda.stream(self.copy_stream):
            host.copy_(out[0], non_blocking=True)
            out[0].record_stream(self.copy_stream)
        ev = torch.cuda.Event()
        ev.record(self.copy_stream)
        self.pending.append(_Pending(s.req.name, k, host, n[0], s.lost, s.last_arrival, dev_ev, ev))
        s.dumps_done += 1
        s.integrated = s.covered = s.lost = 0
        if s.dumps_done == s.req.n_dumps:
            # leaves: free the slot (detach waits for the engine), admit the next
            self.plan.detach(s.slot)
            del self.slots[s.req.name]
            self.adm.release(s.req)
            if self.on_leave:
                self.on_leave(s.req)

    def _finish(self, item: "_Pending", wait: bool) -> bool:
        """Move a pending dump to done once its copies have completed."""
        if item.t_dev is None and (wait or item.dev_ev.query()):
            if wait:
                item.dev_ev.synchronize()
            item.t_dev = time.perf_counter()
        if item.t_dev is None or not (wait or item.ev.query()):
            return False
        if wait:
            item.ev.synchronize()
        t = time.perf_counter()
        vis = item.host.clone() if self.keep_results else None
        self.done.append(Dump(item.name, item.index, vis, item.n, item.lost,
                              1e3 * (t - item.t_last), 1e3 * (item.t_dev - item.t_last)))
        self.pending.remove(item)
        return True

    def poll(self, wait: bool = False) -> list[Dump]:
        """Collect dumps whose host copy has completed (all of them with wait)."""
        before = len(self.done)
        for item in list(self.pending):
            self._finish(item, wait)
        return self.done[before:]

    def idle(self) -> bool:
        return not self.slots and not self.adm.waiting and not self.pending

    def close(self) -> None:
        self.torch.cuda.synchronize()
        self.plan.close()


def latency_stats(dumps: list[Dump]) -> dict:
    if not dumps:
        return {}
    lat = np.array([d.latency_ms for d in dumps])
    dev = np.array([d.device_latency_ms for d in dumps])
    return {"dumps": len(dumps),
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "device_latency_ms_p50": float(np.percentile(dev, 50)),
            "device_latency_ms_p99": float(np.percentile(dev, 99))}


@dataclass
class Feed:
    """Block source of one request: a device ring of pre-staged blocks.

    Block seq lives in ring rows (seq % R) * BLOCK_T ..; the producer keeps at
    most R blocks queued (a slot is refilled once its block has been taken by
    an engine call).  ``drop`` lists sequence numbers that never arrive (lost
    packets)."""
    ring: object                  # uint8 device tensor [R * BLOCK_T, F, N]
    n_blocks: int                 # blocks to send (lost ones included)
    drop: frozenset = frozenset()
    next_seq: int = 0
    t_start: float | None = None

    @property
    def ring_blocks(self) -> int:
        return self.ring.shape[0] // BLOCK_T

    def block(self, seq: int, arrival: float) -> Block:
        row = (seq % self.ring_blocks) * BLOCK_T
        return Block(seq, self.ring[row: row + BLOCK_T], self.ring, row, arrival)


class HostFeed(Feed):
    """Block source in host memory, the H2D-inclusive form of the network
    thread's ring (Sec. 2.2): blocks arrive in a pinned host ring and are
    copied into a device ring on a copy stream.

    Block seq comes from host rows (seq % R_host) * BLOCK_T .. and lands in
    device ring slot seq % R_dev.  Its copy waits for the engine call that
    read the slot's previous block (event from the server), and the engine
    waits for the copy (the block's ready event) before it reads the block."""

    def __init__(self, host, ring, n_blocks: int, copy_stream, drop: frozenset = frozenset()):
        super().__init__(ring, n_blocks, drop)
        self.host = host            # pinned uint8 host tensor [R_host * BLOCK_T, F, N]
        self.copy_stream = copy_stream
        self.slot_free = [None] * self.ring_blocks   # event: the slot's last block has been read

    def block(self, seq: int, arrival: float) -> Block:
        import torch
        slot = seq % self.ring_blocks
        row = slot * BLOCK_T
        hrow = (seq % (self.host.shape[0] // BLOCK_T)) * BLOCK_T
        if self.slot_free[slot] is not None:
            self.copy_stream.wait_event(self.slot_free[slot])
        with torch.cuda.stream(self.copy_stream):
            self.ring[row: row + BLOCK_T].copy_(self.host[hrow: hrow + BLOCK_T], non_blocking=True)
        ready = torch.cuda.Event()
        ready.record(self.copy_stream)

        def consumed(ev, slot=slot):
            self.slot_free[slot] = ev
        return Block(seq, self.ring[row: row + BLOCK_T], self.ring, row, arrival, ready, consumed)


def realtime_period(n_chans: int, sample_rate: float = 250e6) -> float:
    """Seconds per block of BLOCK_T spectra at real sampling rate sample_rate:
    an F-channel spectrum spans 2F real samples (Sec. 2.1 and Sec. 1)."""
    return BLOCK_T * 2 * n_chans / sample_rate


def drive(server: Server, arrivals: list[tuple[float, Request]], feeds: dict[str, Feed],
          paced: bool, time_limit: float = 120.0) -> float:
    """Run the loop until every request has been served.

    arrivals: (seconds after start, request) in time order.  A request's
    blocks start arriving when it is admitted: in real time (one block per
    realtime_period) when paced, else as fast as the ring allows.  Returns
    the wall time in seconds."""
    t0 = time.perf_counter()
    todo = list(arrivals)
    n_total = len(arrivals)
    while True:
        now = time.perf_counter()
        if now - t0 > time_limit:
            raise TimeoutError(f"serving loop still busy after {time_limit} s")
        while todo and todo[0][0] <= now - t0:
            server.submit(todo.pop(0)[1])
        for name in server.resident():
            f = feeds[name]
            s = server.slots[name]
            if f.t_start is None:
                f.t_start = now
            per = realtime_period(s.req.n_chans)
            while f.next_seq < f.n_blocks and len(s.queue) < f.ring_blocks:
                arrival = f.t_start + (f.next_seq + 1) * per if paced else now
                if arrival > now:
                    break
                if f.next_seq not in f.drop:
                    server.push(name, f.block(f.next_seq, arrival))
                f.next_seq += 1
            if f.next_seq == f.n_blocks and not s.queue and s.covered:
                # stream ended inside an integration: the missing tail counts as lost
                s.lost += s.req.dump_len - s.covered
                s.covered = s.req.dump_len
        issued = server.step()
        server.poll()
        if not todo and server.idle() and len(server.done) >= 0 and \
                all(feeds[r.name].next_seq >= feeds[r.name].n_blocks for _, r in arrivals) and \
                len({d.name for d in server.done}) == n_total:
            break
        if not issued:
            time.sleep(2e-4 if paced else 0)
    server.poll(wait=True)
    return time.perf_counter() - t0
