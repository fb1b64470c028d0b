"""Bit-exact parity of the HIP X-engine against the CPU oracle.

Integer work: every visibility must equal the oracle's exactly.  Sizes
span several 16-row tiles with ragged edges in N and ragged tails in T; the
full-size workloads are checked on every channel against the oracle, in the
launch the benchmark times; the ring kernel is run at its largest time chunk
and at the library's int32 integration limit.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import KIND_STAGE, KIND_X32, first_mismatch, forced_kernel, gpu_available, run_engine

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]


def check(v_blocks, N, F, chans=None, max_t=None):
    got, n = run_engine(v_blocks, N, F, max_t=max_t)
    assert n == sum(b.shape[0] for b in v_blocks)
    e = oracle.Engine(N, F if chans is None else len(chans))
    for b in v_blocks:
        e.correlate(b if chans is None else np.ascontiguousarray(b[:, chans]))
    want, _ = e.dump()
    g = got if chans is None else got[chans]
    assert np.array_equal(g, want), first_mismatch(g, want)
    return got


def test_dish_tiny_full():
    w = synth.WORKLOADS["dish_tiny"]
    v = synth.voltages(w["recipe"], w["seed"], w["n_inputs"], w["n_chans"], w["n_time"])
    print(f"dish_tiny N={w['n_inputs']} F={w['n_chans']} T={w['n_time']}", flush=True)
    check([v], w["n_inputs"], w["n_chans"])


# every tile count 1..16, ragged N, ragged T tails, time-split and single-WG launches
SWEEP = [(1, 1, 1), (2, 3, 31), (3, 5, 33), (5, 2, 100), (8, 7, 64), (15, 3, 257),
         (16, 4, 1000), (17, 2, 95), (31, 9, 129), (32, 6, 4096), (33, 3, 333),
         (47, 2, 520), (48, 5, 64), (63, 3, 127), (64, 4, 2048), (80, 2, 96),
         (96, 3, 1024), (100, 2, 77), (112, 2, 300), (127, 1, 513), (128, 3, 1000),
         (144, 2, 256), (150, 1, 99), (160, 2, 640), (176, 2, 160), (191, 1, 400),
         (192, 3, 512), (200, 2, 200), (224, 1, 96), (240, 1, 1100), (255, 1, 65),
         (256, 2, 384), (1, 1, 100000), (48, 1, 70000), (192, 1, 20000),
         (208, 3, 777), (160, 5, 321), (128, 7, 4097), (240, 2, 65), (16, 9, 33000)]


@pytest.mark.parametrize("N,F,T", SWEEP, ids=lambda x: str(x))
def test_random_shape_sweep(N, F, T):
    print(f"sweep N={N} F={F} T={T}", flush=True)
    rng = np.random.default_rng(1000 * N + 10 * F + T % 10)
    re = rng.integers(-8, 8, size=(T, F, N))
    im = rng.integers(-8, 8, size=(T, F, N))
    check([synth.pack(re, im)], N, F)


@pytest.mark.parametrize("N", [17, 64, 192, 256])
@pytest.mark.parametrize("pattern", ["all_minus8", "all_plus7", "alternating", "one_hot"])
def test_adversarial_codes(N, pattern):
    F, T = 3, 1000
    print(f"adversarial {pattern} N={N}", flush=True)
    if pattern == "all_minus8":
        v = np.full((T, F, N), 0x88, np.uint8)
    elif pattern == "all_plus7":
        v = np.full((T, F, N), 0x77, np.uint8)
    elif pattern == "alternating":
        t, f, n = np.indices((T, F, N))
        s = (t + n) % 2
        v = np.where(s == 0, 0x77, 0x88).astype(np.uint8)
        v[:, 1, ::3] = 0x8F   # -8 - 1j
    else:
        v = np.zeros((T, F, N), np.uint8)
        v[::7, :, N // 2] = 0x80
        v[::5, :, 0] = 0x08
        v[::3, :, N - 1] = 0x71
    check([v], N, F)


def test_multi_call_integration_and_keep():
    import torch
    from paper_1904_07778_amd.xeng import Plan
    N, F = 70, 5
    blocks = [synth.voltages("noise", 21, N, F, t, block=b) for b, t in enumerate([100, 257, 32, 1000])]
    e = oracle.Engine(N, F)
    with Plan([(N, F, 1000)]) as p:
        for b in blocks[:2]:
            p.correlate([torch.from_numpy(b).cuda()])
            e.correlate(b)
        out, n = p.dump(keep=True, to_host=True)
        want, _ = e.dump(keep=True)
        assert n == [357] and np.array_equal(out[0].numpy(), want)
        for b in blocks[2:]:
            p.correlate([torch.from_numpy(b).cuda()])
            e.correlate(b)
        out, n = p.dump(to_host=True)
        want, _ = e.dump()
        assert n == [1389] and np.array_equal(out[0].numpy(), want), first_mismatch(out[0].numpy(), want)
        out, n = p.dump(to_host=True)
        assert n == [0] and not out[0].numpy().any()
        # after a dump the next call starts a fresh integration (store path)
        p.correlate([torch.from_numpy(blocks[0]).cuda()])
        out, n = p.dump(to_host=True)
        assert np.array_equal(out[0].numpy(), oracle.correlate(blocks[0]))


@pytest.mark.parametrize("N,kind", [(192, None), (256, None), (96, None), (70, None), (256, KIND_X32),
                                    (96, KIND_X32), (64, KIND_STAGE)], ids=lambda x: str(x))
def test_accumulating_calls_every_kernel(N, kind):
    """Read-modify-write epilogues: calls of under 512 samples keep one
    workgroup per channel (no time split), so the second and later calls of
    an integration add to the accumulator in place.  By default N = 192,
    256 and 96 run the 16-row kernel and N = 70 the staging kernel; the
    32-row kernel (N = 256, 96) and the staging kernel at a multiple of 16
    are forced through the tuning cache.  Extreme codes in some blocks push
    the sums to large magnitudes of both signs.  Every channel against the
    oracle after each call."""
    import contextlib
    import torch
    from paper_1904_07778_amd.xeng import Plan
    F = 3
    rng = np.random.default_rng(N + 5)
    lens = [300, 500, 64, 511, 200]
    blocks = []
    for k, t in enumerate(lens):
        re, im = rng.integers(-8, 8, size=(t, F, N)), rng.integers(-8, 8, size=(t, F, N))
        if k in (1, 3):
            re[:, :, ::2], im[:, :, 1::3] = -8, 7
        blocks.append(synth.pack(re, im))
    print(f"accumulating calls N={N} kind={kind}", flush=True)
    e = oracle.Engine(N, F)
    force = forced_kernel(N, F, 512, kind) if kind is not None else contextlib.nullcontext()
    with force, Plan([(N, F, 512)]) as p:
        for k, b in enumerate(blocks):
            p.correlate([torch.from_numpy(b).cuda()])
            e.correlate(b)
            out, n = p.dump(keep=True, to_host=True)
            want, _ = e.dump(keep=True)
            assert n == [sum(lens[:k + 1])]
            assert np.array_equal(out[0].numpy(), want), (k, first_mismatch(out[0].numpy(), want))


def test_dump_to_device_buffer():
    import torch
    from paper_1904_07778_amd.xeng import Plan
    N, F, T = 33, 4, 200
    v = synth.voltages("tone", 3, N, F, T)
    with Plan([(N, F, T)]) as p:
        p.correlate([torch.from_numpy(v).cuda()])
        out, n = p.dump()
        assert out[0].is_cuda
        assert np.array_equal(out[0].cpu().numpy(), oracle.correlate(v))


def test_caller_on_the_engine_stream():
    """A caller that runs on the engine's stream gets stream order and no
    waits across streams: one device input buffer is refilled in place between
    calls, and every integration still equals the oracle."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    N, F, T = 64, 8, 1024
    blocks = [synth.voltages("sources", 11, N, F, T, block=b) for b in range(3)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream), Plan([(N, F, T)], stream=stream) as p:
        buf = torch.empty((T, F, N), dtype=torch.uint8, device="cuda")
        out = p.new_output(0)
        for b in blocks[:2]:
            buf.copy_(torch.from_numpy(b).pin_memory(), non_blocking=True)
            p.correlate([buf])
        buf.copy_(torch.from_numpy(blocks[2]).pin_memory(), non_blocking=True)
        p.correlate_dump([buf], out=[out])
        got = out.cpu().numpy()
        buf.copy_(torch.from_numpy(blocks[0]).pin_memory(), non_blocking=True)
        p.correlate_dump([buf], out=[out])
        got0 = out.cpu().numpy()
    e = oracle.Engine(N, F)
    for b in blocks:
        e.correlate(b)
    want, _ = e.dump()
    assert np.array_equal(got, want), first_mismatch(got, want)
    want0 = oracle.correlate(blocks[0])
    assert np.array_equal(got0, want0), first_mismatch(got0, want0)


@pytest.mark.parametrize("N", [1, 40])
def test_integration_exact_at_int32_bound(N):
    """Staging kernel (N not a multiple of 16; N = 40 spans three 16-row
    tiles), all codes -8: every visibility reaches 128 * 16,777,215 =
    2,147,483,520, the largest integration the library accepts, and must be
    exact; one sample more is refused."""
    import torch
    from paper_1904_07778_amd.xeng import XENG_EOVERFLOW, XENG_MAX_INTEGRATION, Plan, XengError
    T = XENG_MAX_INTEGRATION
    print(f"staging kernel int32 bound N={N}", flush=True)
    v = torch.full((T, 1, N), 0x88, dtype=torch.uint8, device="cuda")
    with Plan([(N, 1, T)]) as p:
        p.correlate([v])
        with pytest.raises(XengError) as ei:
            p.correlate([v[:1]])
        assert ei.value.status == XENG_EOVERFLOW
        out, n = p.dump(to_host=True)
    del v
    assert n == [T]
    got = out[0].numpy()
    want = np.broadcast_to(np.array([128 * T, 0], np.int32), got.shape)
    assert got.shape == (1, N * (N + 1) // 2, 2)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_dish_scale_eight_calls_all_channels():
    """Dish-array workload at full size: 8 calls of 16384 samples, then one
    dump; every channel against the oracle."""
    w = synth.WORKLOADS["dish"]
    N, F, T = w["n_inputs"], w["n_chans"], w["n_time"]
    print(f"dish N={N} F={F} T={T} x {w['calls']} calls", flush=True)
    blocks = [synth.voltages(w["recipe"], w["seed"], N, F, T, block=b) for b in range(w["calls"])]
    got = check(blocks, N, F, max_t=T)
    autos = got[:, [i * (i + 1) // 2 + i for i in range(N)]]
    assert (autos[..., 1] == 0).all() and (autos[..., 0] >= 0).all()


@pytest.mark.parametrize("name", ["dish_tiny", "dish", "cylinder"])
def test_full_workload_in_shipped_launch_choices(name):
    """Each plain workload at full size in the launch the benchmark runs by
    default (the tuning cache shipped with the library), integrated over its
    calls with correlate and finished with correlate_dump as the bench step
    does: every channel against the oracle."""
    import os
    import torch
    from paper_1904_07778_amd import xeng as X
    from paper_1904_07778_amd.xeng import Plan
    path = os.path.join(os.path.dirname(X.__file__), "tune_gfx950.txt")
    if torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] != "gfx950" or not os.path.exists(path):
        pytest.skip("the shipped launch choices are for gfx950")
    w = synth.WORKLOADS[name]
    N, F, T, calls = w["n_inputs"], w["n_chans"], w["n_time"], w["calls"]
    print(f"{name} in shipped launch choices: N={N} F={F} T={T} x {calls}", flush=True)
    blocks = [synth.voltages(w["recipe"], w["seed"], N, F, T, block=b) if calls > 1 else
              synth.voltages(w["recipe"], w["seed"], N, F, T) for b in range(calls)]
    X.xeng_tune_cache_clear()
    X.xeng_tune_cache_load(path)
    try:
        with Plan([(N, F, T)]) as p:
            for b in blocks[:-1]:
                p.correlate([torch.from_numpy(b).cuda()])
            out, n = p.correlate_dump([torch.from_numpy(blocks[-1]).cuda()])
            got = out[0].cpu().numpy()
    finally:
        X.xeng_tune_cache_clear()
    assert n[0] == T * calls
    e = oracle.Engine(N, F)
    for b in blocks:
        e.correlate(b)
    want, _ = e.dump()
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_cylinder_scale_all_channels():
    """Cylinder workload at full size in the launch the benchmark times (one
    fused correlate-and-dump call into a device buffer): every channel
    against the oracle."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    w = synth.WORKLOADS["cylinder"]
    N, F, T = w["n_inputs"], w["n_chans"], w["n_time"]
    print(f"cylinder N={N} F={F} T={T}", flush=True)
    v = synth.voltages(w["recipe"], w["seed"], N, F, T)
    with Plan([(N, F, T)]) as p:
        out, n = p.correlate_dump([torch.from_numpy(v).cuda()])
        got = out[0].cpu().numpy()
    assert n == [T]
    want = oracle.correlate(v)
    assert np.array_equal(got, want), first_mismatch(got, want)
    autos = got[:, [i * (i + 1) // 2 + i for i in range(N)]]
    assert (autos[..., 1] == 0).all() and (autos[..., 0] > 0).all()
    # Eq. 3: RMS = sqrt(P / 2N) of every input on every channel lies in 2..3
    rms = np.sqrt(autos[..., 0] / (2 * T))
    assert 2.0 < rms.mean() < 3.0


def _closed_form(re, im, T):
    """V_ij = T x_i conj(x_j) for inputs x_i = re_i + j im_i held constant over
    T samples: (T (a_i a_j + b_i b_j), T (b_i a_j - a_i b_j)), lower triangle."""
    N = len(re)
    vis = np.zeros((N * (N + 1) // 2, 2), np.int64)
    for i in range(N):
        for j in range(i + 1):
            vis[i * (i + 1) // 2 + j] = (T * (re[i] * re[j] + im[i] * im[j]),
                                         T * (im[i] * re[j] - re[i] * im[j]))
    return vis


@pytest.mark.parametrize("N,batched,kind", [(16, False, None), (16, True, None), (192, False, None),
                                             (192, True, None), (256, False, None), (256, True, None),
                                             (256, False, KIND_X32), (192, False, KIND_X32)],
                         ids=lambda x: str(x))
def test_ring_kernel_at_int32_bound(N, batched, kind):
    """Ring kernels at the library's integration limit: all codes -8,
    T = 16,777,215 in one call, so every workgroup integrates the largest
    time chunk its kernel takes (the x256-scaled sums at their headroom) and
    the chunks meet in the accumulator by atomic adds.  By default every N
    here runs the 16-row-tile kernel (in a batched plan N = 16 and 192 run
    inside the persistent launch, N = 256 as a launch of its own); the
    32-row-tile kernel is forced through the tuning cache for N = 256 and
    192.  Every visibility must be 128 T = 2,147,483,520 (the closed form),
    exact."""
    import contextlib
    import torch
    from paper_1904_07778_amd.xeng import XENG_MAX_INTEGRATION, Plan
    T, F = XENG_MAX_INTEGRATION, 1
    print(f"ring kernel int32 bound N={N} batched={batched} kind={kind}", flush=True)
    v = torch.full((T, F, N), 0x88, dtype=torch.uint8, device="cuda")
    force = forced_kernel(N, F, T, kind) if kind is not None else contextlib.nullcontext()
    with force, Plan([(N, F, T)], batch=batched) as p:
        p.correlate([v])
        out, n = p.dump(to_host=True)
    del v
    got = out[0].numpy()
    assert n == [T]
    want = np.broadcast_to(np.array([128 * T, 0], np.int32), got.shape)
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("batched", [False, True], ids=["plain", "batched"])
def test_ring_kernel_full_chunks_extreme_codes(batched):
    """N = 192 with 512 channels and 65536 samples: every workgroup owns one
    channel over 32768 samples (the ring kernel's largest chunk) and two
    chunks meet by atomic adds.  Each input holds one extreme code for the
    whole integration (the -8 corners included), so the x256-scaled real and
    imaginary sums grow linearly to their largest per-chunk magnitudes.
    Checked on every channel against the closed form V_ij = T x_i conj(x_j)
    and on two channels against the oracle."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    N, F, T = 192, 512, 65536
    rng = np.random.default_rng(97)
    re = rng.choice(np.array([-8, -8, 7, 7, -7, 0, 3]), size=N)
    im = rng.choice(np.array([-8, -8, 7, -7, 0, 5]), size=N)
    re[:4], im[:4] = [-8, 7, -8, 7], [-8, -8, 7, 7]
    codes = synth.pack(re, im)
    print(f"ring kernel full chunks N={N} F={F} T={T} batched={batched}", flush=True)
    v = torch.from_numpy(codes).cuda().view(1, 1, N).expand(T, F, N).contiguous()
    with Plan([(N, F, T)], batch=batched) as p:
        p.correlate([v])
        out, n = p.dump(to_host=True)
    got = out[0].numpy()
    assert n == [T]
    want = _closed_form(re.astype(np.int64), im.astype(np.int64), T)
    assert np.abs(want).max() == 128 * T                 # the -8 - 8j autos
    want = np.broadcast_to(want.astype(np.int32), got.shape)
    assert np.array_equal(got, want), first_mismatch(got, want)
    vh = v[:, :2].cpu().numpy()
    del v
    w2 = oracle.correlate(np.ascontiguousarray(vh))
    assert np.array_equal(got[:2], w2), first_mismatch(got[:2], w2)


@pytest.mark.parametrize("to_host", [False, True])
def test_restart_after_dump_every_epilogue(to_host):
    """After a dump the integration restarts from zero whatever the next launch
    does: plain stores (one workgroup per channel), atomic adds (time split
    over workgroups) or read-modify-write (second call), and an empty
    integration dumps as zeros; device and host destinations."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(31)
    N, F = 192, 2
    blocks = [synth.pack(rng.integers(-8, 8, size=(t, F, N)), rng.integers(-8, 8, size=(t, F, N)))
              for t in (3000, 20000, 512, 700)]
    print("restart after dump, to_host", to_host, flush=True)

    def dump(p):
        out, n = p.dump(to_host=to_host)
        return (out[0] if to_host else out[0].cpu()).numpy(), n[0]

    with Plan([(N, F, 20000)]) as p:
        p.correlate([torch.from_numpy(blocks[0]).cuda()])        # plain stores
        g0, _ = dump(p)
        p.correlate([torch.from_numpy(blocks[1]).cuda()])        # time split: atomics on a dumped accumulator
        g1, _ = dump(p)
        g2, n2 = dump(p)                                         # empty integration
        p.correlate([torch.from_numpy(blocks[2]).cuda()])        # plain stores
        p.correlate([torch.from_numpy(blocks[3]).cuda()])        # read-modify-write
        g3, n3 = dump(p)
    torch.cuda.synchronize()
    for got, bl in ((g0, [blocks[0]]), (g1, [blocks[1]]), (g3, blocks[2:])):
        e = oracle.Engine(N, F)
        for b in bl:
            e.correlate(b)
        want = e.dump()[0]
        assert np.array_equal(got, want), first_mismatch(got, want)
    assert n2 == 0 and not g2.any()
    assert n3 == 1212


def test_checkpoint_resume_and_counters():
    """A KEEP dump is a snapshot; a new plan seeded with it (xeng_load_acc)
    and fed the remaining blocks ends bit-identical to the uninterrupted run.
    The plan counters add up."""
    import subprocess
    import sys
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(51)
    N, F = 96, 5
    blocks = [synth.pack(rng.integers(-8, 8, size=(t, F, N)), rng.integers(-8, 8, size=(t, F, N)))
              for t in (700, 1200, 300)]
    print("checkpoint / resume", flush=True)
    with Plan([(N, F, 2000)]) as p:
        for b in blocks:
            p.correlate([torch.from_numpy(b).cuda()])
        whole, n_whole = p.dump(to_host=True)
        st = p.stats()
    assert st["calls"] == 3 and st["samples"] == 2200 and st["dumps"] == 1
    assert st["cmacs"] == 2200 * F * N * (N + 1) // 2 and st["bytes_in"] == 2200 * F * N
    with Plan([(N, F, 2000)]) as p:
        p.correlate([torch.from_numpy(blocks[0]).cuda()])
        snap, n_snap = p.dump(keep=True, to_host=True)          # checkpoint
    with Plan([(N, F, 2000)]) as q:
        q.load(0, snap[0], n_snap[0])                           # resume from host memory
        for b in blocks[1:]:
            q.correlate([torch.from_numpy(b).cuda()])
        resumed, n_res = q.dump(to_host=True)
    torch.cuda.synchronize()
    assert n_res[0] == n_whole[0] == 2200
    assert np.array_equal(resumed[0].numpy(), whole[0].numpy())
    # the launch trace goes to stderr when XENG_TRACE is set
    code = ("import torch, numpy as np; from paper_1904_07778_amd.xeng import Plan\n"
            "p = Plan([(32, 2, 64)]); p.correlate([torch.zeros((64, 2, 32), dtype=torch.uint8, device='cuda')]);"
            " torch.cuda.synchronize(); p.close()")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       env={**__import__("os").environ, "XENG_TRACE": "1"})
    assert r.returncode == 0 and "plain launch N=32 F=2 T=64" in r.stderr, r.stderr[-500:]
