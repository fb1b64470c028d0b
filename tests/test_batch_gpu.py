"""Batched form: one persistent, graph-recorded launch over many arrays.

Integer work, so every check is exact: the batched engine against the CPU
oracle (whole arrays, at small sizes and at the full batched workload), and
against the plain per-array engine bit for bit.  Also the graph paths (the same call replayed, calls whose sizes change, more arrays
than one launch takes), the autotuner, slot attach/detach, and the dump
kernel next to the copy fallback.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import first_mismatch, gpu_available

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]


def rand_block(rng, T, F, N):
    return synth.pack(rng.integers(-8, 8, size=(T, F, N)), rng.integers(-8, 8, size=(T, F, N)))


def oracle_vis(blocks, N, F, chans=None):
    e = oracle.Engine(N, F if chans is None else len(chans))
    for b in blocks:
        e.correlate(b if chans is None else np.ascontiguousarray(b[:, chans]))
    return e.dump()[0]


def to_dev(b):
    import torch
    return torch.from_numpy(np.ascontiguousarray(b)).cuda()


# Ragged mix: every batched N from 16 to 192, plus N the batch kernel does not
# take (not a multiple of 16, or above 192), which run as plain launches inside
# the same graph; uneven F and T, ragged time tails.
MIX = [(16, 5, 300), (32, 3, 64), (48, 2, 1000), (64, 4, 129), (80, 1, 33), (96, 3, 257),
       (112, 2, 64), (128, 1, 700), (144, 2, 96), (160, 1, 65), (176, 1, 128), (192, 2, 513),
       (40, 3, 200), (200, 1, 96), (1, 2, 50)]


def test_batched_mix_matches_oracle():
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(7)
    blocks = [rand_block(rng, T, F, N) for N, F, T in MIX]
    print("batched mix", MIX, flush=True)
    with Plan([(N, F, T) for N, F, T in MIX]) as p:
        assert p.batched
        p.correlate([to_dev(b) for b in blocks])
        out, n = p.dump(to_host=True)
    torch.cuda.synchronize()
    for (N, F, T), b, got, k in zip(MIX, blocks, out, n):
        assert k == T
        want = oracle_vis([b], N, F)
        assert np.array_equal(got.numpy(), want), f"N={N} F={F} T={T}: " + first_mismatch(got.numpy(), want)


def test_batched_repeat_and_resize():
    """Several calls through the graph ring: same sizes (graph update with
    identical parameters), then changed T per array and a skipped array, with
    a kept dump in the middle."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    shapes = [(192, 2, 4096), (32, 9, 4096), (64, 3, 4096), (16, 17, 4096)]
    rng = np.random.default_rng(11)
    calls = [[640, 640, 640, 640], [640, 640, 640, 640], [100, 0, 4096, 33],
             [640, 640, 640, 640], [640, 640, 640, 640], [1, 2, 3, 4]]
    blocks = [[rand_block(rng, t, F, N) if t else None for (N, F, _), t in zip(shapes, ts)] for ts in calls]
    print("batched repeat", shapes, calls, flush=True)
    with Plan(shapes) as p:
        for ci, ts in enumerate(calls):
            p.correlate([to_dev(b) if b is not None else None for b in blocks[ci]])
            if ci == 2:
                kept, _ = p.dump(keep=True, to_host=True)
        out, n = p.dump(to_host=True)
    torch.cuda.synchronize()
    for a, (N, F, _) in enumerate(shapes):
        mine = [blocks[ci][a] for ci in range(len(calls)) if blocks[ci][a] is not None]
        mine_kept = [blocks[ci][a] for ci in range(3) if blocks[ci][a] is not None]
        assert n[a] == sum(b.shape[0] for b in mine)
        want = oracle_vis(mine, N, F)
        assert np.array_equal(out[a].numpy(), want), f"array {a}: " + first_mismatch(out[a].numpy(), want)
        want_k = oracle_vis(mine_kept, N, F)
        assert np.array_equal(kept[a].numpy(), want_k), f"kept {a}: " + first_mismatch(kept[a].numpy(), want_k)


def test_more_arrays_than_one_launch():
    """30 arrays: two persistent launches in one graph."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(13)
    shapes = [(int(16 * rng.integers(1, 13)), int(rng.integers(1, 6)), int(rng.integers(1, 400)))
              for _ in range(30)]
    blocks = [rand_block(rng, T, F, N) for N, F, T in shapes]
    print("30 arrays", flush=True)
    with Plan(shapes) as p:
        p.correlate([to_dev(b) for b in blocks])
        out, _ = p.dump(to_host=True)
    torch.cuda.synchronize()
    for (N, F, T), b, got in zip(shapes, blocks, out):
        want = oracle_vis([b], N, F)
        assert np.array_equal(got.numpy(), want), f"N={N} F={F} T={T}: " + first_mismatch(got.numpy(), want)


def test_autotune_keeps_results_exact():
    import torch
    from paper_1904_07778_amd.xeng import Plan
    shapes = [(192, 8, 8192), (48, 64, 4096), (16, 40, 2048)]
    rng = np.random.default_rng(17)
    blocks = [rand_block(rng, T, F, N) for N, F, T in shapes]
    print("autotune", shapes, flush=True)
    dev = [to_dev(b) for b in blocks]
    with Plan(shapes) as p:
        ms = p.autotune(dev, reps=2)
        assert ms > 0
        _, n0 = p.dump(keep=True, to_host=True)
        assert list(n0) == [0, 0, 0]          # the trials leave nothing behind
        p.correlate(dev)
        out, _ = p.dump(to_host=True)
    torch.cuda.synchronize()
    for (N, F, T), b, got in zip(shapes, blocks, out):
        want = oracle_vis([b], N, F)
        assert np.array_equal(got.numpy(), want), f"N={N}: " + first_mismatch(got.numpy(), want)


@pytest.mark.parametrize("N", [16, 48, 192])
def test_plain_autotune_keeps_results_exact(N):
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(N)
    b = rand_block(rng, 3000, 6, N)
    print(f"plain autotune N={N}", flush=True)
    with Plan([(N, 6, 3000)]) as p:
        assert not p.batched
        p.autotune([to_dev(b)], reps=1)
        p.correlate([to_dev(b)])
        out, _ = p.dump(to_host=True)
    torch.cuda.synchronize()
    want = oracle_vis([b], N, 6)
    assert np.array_equal(out[0].numpy(), want), first_mismatch(out[0].numpy(), want)


def test_attach_detach_slots():
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(19)
    print("attach/detach", flush=True)
    with Plan([], batch=True) as p:
        a = p.attach(32, 4, 1024)
        b = p.attach(192, 2, 1024)
        c = p.attach(20, 3, 1024)
        assert (a, b, c) == (0, 1, 2)
        x = {k: rand_block(rng, 512, s.n_chans, s.n_inputs) for k, s in enumerate(p.specs)}
        p.correlate([to_dev(x[0]), to_dev(x[1]), to_dev(x[2])])
        out_b, _ = p.dump(b, to_host=True)
        p.detach(b)
        with pytest.raises(Exception):
            p.correlate([None, to_dev(x[1]), None])   # free slot
        d = p.attach(64, 5, 2048)                   # reuses the free slot
        assert d == 1
        y = rand_block(rng, 2048, 5, 64)
        p.correlate([to_dev(x[0]), to_dev(y), None])
        out, n = p.dump(to_host=True)
    torch.cuda.synchronize()
    assert np.array_equal(out_b[0].numpy(), oracle_vis([x[1]], 192, 2))
    assert np.array_equal(out[0].numpy(), oracle_vis([x[0], x[0]], 32, 4))
    assert np.array_equal(out[1].numpy(), oracle_vis([y], 64, 5))
    assert np.array_equal(out[2].numpy(), oracle_vis([x[2]], 20, 3))
    assert list(n) == [1024, 2048, 512]


def test_dump_kernel_and_copy_paths_agree():
    """Device dumps to 8-byte aligned buffers go through the dump kernel; a
    misaligned destination falls back to a plain copy."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(23)
    shapes = [(32, 3, 256), (48, 2, 256)]
    blocks = [rand_block(rng, T, F, N) for N, F, T in shapes]
    print("dump paths", flush=True)
    with Plan(shapes) as p:
        p.correlate([to_dev(b) for b in blocks])
        aligned = [p.new_output(0), p.new_output(1)]
        raw = torch.empty(aligned[1].numel() + 1, dtype=torch.int32, device="cuda")
        odd = raw[1:].view(aligned[1].shape)             # 4-byte offset: copy path
        p.dump(-1, out=[aligned[0], odd], keep=True)
        p.dump(-1, out=[p.new_output(0), p.new_output(1)])  # clears
        again, n = p.dump(to_host=True)
    torch.cuda.synchronize()
    for (N, F, T), b, got in zip(shapes, blocks, [aligned[0], odd]):
        want = oracle_vis([b], N, F)
        assert np.array_equal(got.cpu().numpy(), want)
    assert list(n) == [0, 0]
    assert all(int(x.abs().max()) == 0 for x in again)


def test_full_batched_workload_all_channels():
    """The 12-array batched workload at full size, in the launch the bench
    times (both forms autotuned, then one correlate-and-dump call): the
    batched outputs are bit-identical to 12 plain calls and equal to the
    oracle on every channel of every array."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    specs = synth.batch_arrays()
    print("full batched workload", specs, flush=True)
    host = [synth.voltages("noise", 4, s["n_inputs"], s["n_chans"], s["n_time"], array=k)
            for k, s in enumerate(specs)]
    dev = [to_dev(h) for h in host]
    shapes = [(s["n_inputs"], s["n_chans"], s["n_time"]) for s in specs]
    with Plan(shapes) as p:
        p.autotune(dev, reps=2)
        batched, _ = p.correlate_dump(dev)
    plain = []
    for sh, v in zip(shapes, dev):
        with Plan([sh]) as q:
            q.autotune([v], reps=2)
            plain.append(q.correlate_dump([v])[0][0])
    torch.cuda.synchronize()
    for k, (s, h) in enumerate(zip(specs, host)):
        assert torch.equal(batched[k], plain[k]), f"array {k}: batched != plain"
        want = oracle_vis([h], s["n_inputs"], s["n_chans"])
        got = batched[k].cpu().numpy()
        assert np.array_equal(got, want), f"array {k}: " + first_mismatch(got, want)


def test_full_batched_workload_shipped_launch_choices():
    """The 12-array workload in the launch the benchmark runs by default: the
    tuning cache shipped with the library, loaded before the plans are made.
    Batched and plain outputs equal the oracle on every channel."""
    import os
    import torch
    from paper_1904_07778_amd import xeng as X
    from paper_1904_07778_amd.xeng import Plan
    path = os.path.join(os.path.dirname(X.__file__), "tune_gfx950.txt")
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    if arch != "gfx950" or not os.path.exists(path):
        pytest.skip("the shipped launch choices are for gfx950")
    specs = synth.batch_arrays()
    print("full batched workload, shipped launch choices", flush=True)
    host = [synth.voltages("noise", 4, s["n_inputs"], s["n_chans"], s["n_time"], array=k)
            for k, s in enumerate(specs)]
    dev = [to_dev(h) for h in host]
    shapes = [(s["n_inputs"], s["n_chans"], s["n_time"]) for s in specs]
    X.xeng_tune_cache_clear()
    X.xeng_tune_cache_load(path)
    try:
        with Plan(shapes) as p:
            batched, _ = p.correlate_dump(dev)
        plain = []
        for sh, v in zip(shapes, dev):
            with Plan([sh]) as q:
                plain.append(q.correlate_dump([v])[0][0])
    finally:
        X.xeng_tune_cache_clear()
    torch.cuda.synchronize()
    for k, (s, h) in enumerate(zip(specs, host)):
        want = oracle_vis([h], s["n_inputs"], s["n_chans"])
        got = batched[k].cpu().numpy()
        assert np.array_equal(got, want), f"array {k}: " + first_mismatch(got, want)
        assert torch.equal(plain[k], batched[k]), f"array {k}: plain != batched"


def test_batched_restart_after_dump_with_time_split():
    """Batched call whose items split time (atomic adds) right after a dump
    that left the old sums in memory."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(37)
    shapes = [(192, 1, 20000), (48, 2, 20000), (40, 1, 20000)]
    b1 = [rand_block(rng, 700, F, N) for N, F, _ in shapes]
    b2 = [rand_block(rng, 20000, F, N) for N, F, _ in shapes]
    print("batched restart after dump", flush=True)
    with Plan(shapes) as p:
        p.correlate([to_dev(b) for b in b1])
        p.dump()
        p.correlate([to_dev(b) for b in b2])
        out, n = p.dump(to_host=True)
    torch.cuda.synchronize()
    for (N, F, _), b, got in zip(shapes, b2, out):
        want = oracle_vis([b], N, F)
        assert np.array_equal(got.numpy(), want), f"N={N}: " + first_mismatch(got.numpy(), want)


def test_batched_call_with_nothing_to_do():
    """A batched call whose arrays all pass zero samples launches nothing and
    changes nothing; the next real call still lands exactly."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(43)
    shapes = [(32, 3, 512), (64, 2, 512)]
    b = [rand_block(rng, 512, F, N) for N, F, _ in shapes]
    print("batched empty call", flush=True)
    with Plan(shapes) as p:
        p.correlate([None, None])
        _, n0 = p.dump(keep=True, to_host=True)
        p.correlate([to_dev(x) for x in b])
        p.correlate([None, None])
        out, n = p.dump(to_host=True)
    torch.cuda.synchronize()
    assert list(n0) == [0, 0] and list(n) == [512, 512]
    for (N, F, _), x, got in zip(shapes, b, out):
        assert np.array_equal(got.numpy(), oracle_vis([x], N, F))


def test_cached_own_launches_in_a_batched_plan(tmp_path):
    """Tuning-cache entries that give arrays of a batched plan plain launches
    of their own (16-row, 32-row and staging tile shapes) inside the graph:
    the results still equal the oracle; a plain plan picks up its cached tile
    shape too."""
    import torch
    from paper_1904_07778_amd import xeng as X
    from paper_1904_07778_amd.xeng import Plan
    dev_arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    rng = np.random.default_rng(61)
    shapes = [(192, 3, 700), (48, 5, 1500), (32, 4, 300), (64, 2, 1000)]
    blocks = [rand_block(rng, T, F, N) for N, F, T in shapes]
    # log2 buckets of F and of max_time_per_call, as the library computes them
    bucket = lambda v: max(0, int(v - 1).bit_length())
    lines = [f"{dev_arch} 1 192 {bucket(3)} {bucket(700)} 0 1 1",     # own launch, 16-row tiles
             f"{dev_arch} 1 48 {bucket(5)} {bucket(1500)} 1 2 1",     # own launch, 32-row tiles
             f"{dev_arch} 1 32 {bucket(4)} {bucket(300)} 2 1 1",      # own launch, staging kernel
             f"{dev_arch} 0 64 {bucket(2)} {bucket(1000)} 1 4 0",     # plain plan: 32-row tiles
             f"{dev_arch} 1 0 0 {bucket(4)} 0 8 0"]                   # batched plan: 8 items per workgroup
    f = tmp_path / "tune.txt"
    f.write_text("\n".join(lines) + "\n")
    X.xeng_tune_cache_clear()
    X.xeng_tune_cache_load(str(f))
    print("cached own launches", shapes, flush=True)
    try:
        with Plan(shapes) as p:
            p.correlate([to_dev(b) for b in blocks])
            out, n = p.dump(to_host=True)
        with Plan([shapes[3]]) as q:
            q.correlate([to_dev(blocks[3])])
            out_plain, _ = q.dump(to_host=True)
    finally:
        X.xeng_tune_cache_clear()
    torch.cuda.synchronize()
    for (N, F, T), b, got, k in zip(shapes, blocks, out, n):
        assert k == T
        want = oracle_vis([b], N, F)
        assert np.array_equal(got.numpy(), want), f"N={N}: " + first_mismatch(got.numpy(), want)
    assert np.array_equal(out_plain[0].numpy(), oracle_vis([blocks[3]], 64, 2))
