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


def run(subs, budget, paced=False, drops=None, ring=3):
    from paper_1904_07778_amd.serve import BLOCK_T, Request, Server, drive
    drops = drops or {}
    srv = Server(budget)
    feeds, hosts, reqs = {}, {}, []
    for k, (name, N, F, dump_len, n_dumps) in enumerate(subs):
        r = Request(name, N, F, dump_len, n_dumps, ring_blocks=ring)
        feeds[name], hosts[name] = make_feed(name, N, F, n_dumps * dump_len // BLOCK_T, ring,
                                             seed=100 + ord(name[0]), drop=drops.get(name, ()))
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


def test_full_size_subarrays_sampled_channels():
    """The streaming workload's four sub-arrays at full size (1024-sample
    blocks from device rings, as the bench runs them), two of them waiting
    for memory; each sub-array's dumps checked on sampled channels."""
    import torch
    from paper_1904_07778_amd.serve import BLOCK_T, Feed, Request, Server, drive
    subs = synth.stream_subarrays()
    ring = 2
    reqs, feeds, hosts = [], {}, {}
    for k, s in enumerate(subs):
        n, f = s["n_inputs"], s["n_chans"]
        dump_len = min(s["dump_len"], 4 * BLOCK_T)          # keep the oracle's share short
        r = Request(f"{n}x{f}", n, f, dump_len, 2, ring_blocks=ring)
        host = synth.voltages("sources", 5, n, f, ring * BLOCK_T, array=k, n_src=1)
        hosts[r.name] = host
        feeds[r.name] = Feed(torch.from_numpy(host).cuda(), 2 * dump_len // BLOCK_T)
        reqs.append(r)
    budget = reqs[0].footprint() + reqs[1].footprint()       # the two small ones wait
    print("serve full size, budget", budget, flush=True)
    srv = Server(budget)
    drive(srv, [(0.0, r) for r in reqs], feeds, paced=False, time_limit=120)
    srv.close()
    for r in reqs:
        mine = sorted([d for d in srv.done if d.name == r.name], key=lambda d: d.index)
        assert [d.index for d in mine] == [0, 1]
        chans = [0, r.n_chans // 2, r.n_chans - 1]
        per = r.dump_len // BLOCK_T
        for d in mine:
            e = oracle.Engine(r.n_inputs, len(chans))
            for seq in range(d.index * per, (d.index + 1) * per):
                row = (seq % ring) * BLOCK_T
                e.correlate(np.ascontiguousarray(hosts[r.name][row:row + BLOCK_T][:, chans]))
            want = e.dump()[0]
            got = d.vis.numpy()[chans]
            assert d.n_integrated == r.dump_len
            assert np.array_equal(got, want), f"{r.name} dump {d.index}: " + first_mismatch(got, want)
