"""Streaming form: continuous batching of sub-arrays through one batched plan.

Exact integer results: every dump equals the oracle over the blocks it
integrated, a sub-array gives the same bytes alone and in a mix (with
admission forcing requests to wait for memory), and lost blocks are detected
and left out of the integration.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import first_mismatch, gpu_available

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]


def make_feed(name, N, F, n_blocks, ring_blocks, seed, drop=()):
    """Ring of distinct random blocks; block seq uses ring slot seq % R."""
    import torch
    from paper_1904_07778_amd.serve import BLOCK_T, Feed
    rng = np.random.default_rng(seed)
    host = synth.pack(rng.integers(-8, 8, size=(ring_blocks * BLOCK_T, F, N)),
                      rng.integers(-8, 8, size=(ring_blocks * BLOCK_T, F, N)))
    return Feed(torch.from_numpy(host).cuda(), n_blocks, frozenset(drop)), host


def expected_dumps(host, N, F, dump_len, n_dumps, ring_blocks, drop=()):
    from paper_1904_07778_amd.serve import BLOCK_T
    per = dump_len // BLOCK_T
    out = []
    for d in range(n_dumps):
        e = oracle.Engine(N, F)
        n = 0
        for seq in range(d * per, (d + 1) * per):
            if seq in drop:
                continue
            r = (seq % ring_blocks) * BLOCK_T
            e.correlate(host[r: r + BLOCK_T])
            n += BLOCK_T
        out.append((e.dump()[0], n))
    return out


SUBS = [("A", 32, 8, 2048, 3), ("B", 48, 4, 3072, 2), ("C", 20, 3, 1024, 4), ("D", 192, 2, 4096, 2)]


def run(subs, budget, paced=False, drops=None, ring=3, seed_of=lambda name: 100 + ord(name[0])):
    from paper_1904_07778_amd.serve import BLOCK_T, Request, Server, drive
    drops = drops or {}
    srv = Server(budget)
    feeds, hosts, reqs = {}, {}, []
    for k, (name, N, F, dump_len, n_dumps) in enumerate(subs):
        r = Request(name, N, F, dump_len, n_dumps, ring_blocks=ring)
        feeds[name], hosts[name] = make_feed(name, N, F, n_dumps * dump_len // BLOCK_T, ring,
                                             seed=seed_of(name), drop=drops.get(name, ()))
        reqs.append(r)
    admitted = []
    srv.on_admit = lambda r: admitted.append((r.name, list(srv.resident())))
    drive(srv, [(0.0, r) for r in reqs], feeds, paced=paced, time_limit=60)
    srv.close()
    return srv, hosts, admitted


def check(srv, hosts, subs, ring=3, drops=None):
    drops = drops or {}
    for name, N, F, dump_len, n_dumps in subs:
        mine = sorted([d for d in srv.done if d.name == name], key=lambda d: d.index)
        assert [d.index for d in mine] == list(range(n_dumps))
        want = expected_dumps(hosts[name], N, F, dump_len, n_dumps, ring, drops.get(name, ()))
        for d, (w, n) in zip(mine, want):
            assert d.n_integrated == n
            assert d.lost_samples == dump_len - n
            got = d.vis.numpy()
            assert np.array_equal(got, w), f"{name} dump {d.index}: " + first_mismatch(got, w)


def test_mix_under_memory_pressure_matches_oracle_and_alone():
    from paper_1904_07778_amd.serve import Request
    fp = {n: Request(n, N, F, dl, nd, ring_blocks=3).footprint() for n, N, F, dl, nd in SUBS}
    budget = max(fp.values()) + min(fp.values())        # never all four at once
    print("serve mix, budget", budget, fp, flush=True)
    srv, hosts, admitted = run(SUBS, budget)
    check(srv, hosts, SUBS)
    assert max(len(res) for _, res in admitted) < len(SUBS)   # someone had to wait
    # the same sub-array alone gives the same bytes
    alone, hosts1, _ = run([SUBS[3]], budget=fp["D"])
    for d1, d2 in zip(sorted([d for d in srv.done if d.name == "D"], key=lambda d: d.index),
                      sorted(alone.done, key=lambda d: d.index)):
        assert np.array_equal(d1.vis.numpy(), d2.vis.numpy())


def test_paced_arrivals_and_latency_report():
    from paper_1904_07778_amd.serve import latency_stats
    subs = [("P", 32, 16, 2048, 3), ("Q", 64, 4, 1024, 4)]
    print("serve paced", subs, flush=True)
    srv, hosts, _ = run(subs, budget=1 << 30, paced=True)
    check(srv, hosts, subs)
    st = latency_stats(srv.done)
    assert st["dumps"] == 7 and st["latency_ms_p50"] > 0
    assert st["latency_ms_p99"] >= st["latency_ms_p50"]


def test_lost_blocks_are_detected_and_skipped():
    subs = [("L", 48, 5, 4096, 3)]
    drops = {"L": {2, 4, 5, 11}}     # block 11 is the last of the last integration
    print("serve gaps", subs, drops, flush=True)
    srv, hosts, _ = run(subs, budget=1 << 30, drops=drops)
    check(srv, hosts, subs, drops=drops)
    lost = [d.lost_samples for d in sorted(srv.done, key=lambda d: d.index)]
    assert lost == [1024, 2048, 1024]


def test_full_size_subarrays_configured_dumps():
    """The streaming workload's four sub-arrays at full size and at their
    configured dump lengths (8192 to 65536 samples), fed from device rings of
    16 blocks as the bench runs them, so queued blocks coalesce; two
    sub-arrays wait for memory.  The first dump of every sub-array is checked
    on every channel against the oracle, the second on every 16th channel."""
    import torch
    from paper_1904_07778_amd.serve import BLOCK_T, Feed, Request, Server, drive
    subs = synth.stream_subarrays()
    ring = 16
    reqs, feeds, hosts = [], {}, {}
    rng = np.random.default_rng(55)
    for k, s in enumerate(subs):
        n, f = s["n_inputs"], s["n_chans"]
        r = Request(f"{n}x{f}", n, f, s["dump_len"], 2, ring_blocks=ring)
        host = rng.integers(0, 256, size=(ring * BLOCK_T, f, n), dtype=np.uint8)
        hosts[r.name] = host
        feeds[r.name] = Feed(torch.from_numpy(host).cuda(), 2 * r.dump_len // BLOCK_T)
        reqs.append(r)
    budget = reqs[0].footprint() + reqs[1].footprint()       # the two small ones wait
    print("serve full size, configured dumps", [(r.name, r.dump_len) for r in reqs], "budget", budget, flush=True)
    srv = Server(budget)
    drive(srv, [(0.0, r) for r in reqs], feeds, paced=False, time_limit=300)
    srv.close()
    assert srv.iterations < sum(2 * r.dump_len // BLOCK_T for r in reqs)   # blocks coalesced
    for r in reqs:
        mine = sorted([d for d in srv.done if d.name == r.name], key=lambda d: d.index)
        assert [d.index for d in mine] == [0, 1]
        per = r.dump_len // BLOCK_T
        for d in mine:
            chans = list(range(r.n_chans)) if d.index == 0 else list(range(0, r.n_chans, 16))
            print(f"  oracle {r.name} dump {d.index} on {len(chans)} channels", flush=True)
            e = oracle.Engine(r.n_inputs, len(chans))
            for seq in range(d.index * per, (d.index + 1) * per):
                row = (seq % ring) * BLOCK_T
                blk = hosts[r.name][row:row + BLOCK_T]
                e.correlate(blk if d.index == 0 else np.ascontiguousarray(blk[:, chans]))
            want = e.dump()[0]
            got = d.vis.numpy()[chans]
            assert d.n_integrated == r.dump_len
            assert np.array_equal(got, want), f"{r.name} dump {d.index}: " + first_mismatch(got, want)


def test_arrival_while_others_run():
    """Requests that arrive while others are on the GPU (mid-run, not at time
    zero) are admitted as memory frees up and their work overlaps the
    residents' in the same engine calls; every dump equals the oracle and the
    same sub-array alone gives the same bytes."""
    from paper_1904_07778_amd.serve import BLOCK_T, Request, Server, drive
    # real-time block periods 2.1 / 1.05 / 0.52 / 0.26 ms (F = 256 / 128 / 64 / 32):
    # R0 runs for about 50 ms, the others arrive at 10, 15 and 20 ms
    subs = [("R0", 64, 256, 8192, 3), ("R1", 32, 128, 4096, 3), ("R2", 48, 64, 2048, 4), ("R3", 96, 32, 4096, 2)]
    ring = 4
    fp = {n: Request(n, N, F, dl, nd, ring_blocks=ring).footprint() for n, N, F, dl, nd in subs}
    budget = fp["R0"] + fp["R1"] + fp["R2"]             # R3 must wait for someone to leave
    feeds, hosts, reqs = {}, {}, []
    for name, N, F, dump_len, n_dumps in subs:
        feeds[name], hosts[name] = make_feed(name, N, F, n_dumps * dump_len // BLOCK_T, ring,
                                             seed=300 + ord(name[1]))
        reqs.append(Request(name, N, F, dump_len, n_dumps, ring_blocks=ring))
    # R0 from the start; the others arrive while R0 (and then each other) run
    arrivals = [(0.0, reqs[0]), (0.010, reqs[1]), (0.015, reqs[2]), (0.020, reqs[3])]
    srv = Server(budget)
    resident_at_admit = {}
    srv.on_admit = lambda r: resident_at_admit.setdefault(r.name, [x for x in srv.resident() if x != r.name])
    print("serve mid-run arrivals", subs, "budget", budget, flush=True)
    drive(srv, arrivals, feeds, paced=True, time_limit=120)
    srv.close()
    check(srv, hosts, subs, ring=ring)
    # at least one late request joined residents that were already running
    assert any(resident_at_admit[n] for n in ("R1", "R2", "R3")), resident_at_admit
    # a late arrival alone gives the same bytes as in the mix
    for name in ("R1", "R3"):
        spec = [x for x in subs if x[0] == name]
        alone, _, _ = run(spec, budget=fp[name], ring=ring, seed_of=lambda nm: 300 + ord(nm[1]))
        for d1, d2 in zip(sorted([d for d in srv.done if d.name == name], key=lambda d: d.index),
                          sorted(alone.done, key=lambda d: d.index)):
            assert np.array_equal(d1.vis.numpy(), d2.vis.numpy())


def test_host_feed_h2d_matches_oracle():
    """Blocks that arrive in pinned host memory and are copied into a device
    ring of only two slots on a copy stream (so every slot is rewritten while
    the engine works on the other): every dump equals the oracle."""
    import torch
    from paper_1904_07778_amd.serve import BLOCK_T, HostFeed, Request, Server, drive
    name, N, F, dump_len, n_dumps = "H", 48, 6, 3072, 3
    host_blocks = 5                                     # host ring longer than the device ring
    rng = np.random.default_rng(77)
    host = synth.pack(rng.integers(-8, 8, size=(host_blocks * BLOCK_T, F, N)),
                      rng.integers(-8, 8, size=(host_blocks * BLOCK_T, F, N)))
    n_blocks = n_dumps * dump_len // BLOCK_T
    copy_stream = torch.cuda.Stream()
    feed = HostFeed(torch.from_numpy(host).pin_memory(),
                    torch.empty((2 * BLOCK_T, F, N), dtype=torch.uint8, device="cuda"), n_blocks, copy_stream)
    srv = Server(1 << 30)
    print("serve h2d feed", flush=True)
    drive(srv, [(0.0, Request(name, N, F, dump_len, n_dumps, ring_blocks=2))], {name: feed}, paced=False,
          time_limit=60)
    srv.close()
    check(srv, {name: host}, [(name, N, F, dump_len, n_dumps)], ring=host_blocks)
