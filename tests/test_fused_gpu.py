"""xeng_correlate_dump: integrate and dump in one call, bit-exact against the
oracle and against the separate correlate + dump calls, over every epilogue
(plain stores, additions after a carried-over integration, atomic adds when
the time range is split), the staging kernel, batched plans with some slots
left integrating, dump-only slots and argument errors."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import first_mismatch, gpu_available

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]


def block(rng, T, F, N):
    return synth.pack(rng.integers(-8, 8, size=(T, F, N)), rng.integers(-8, 8, size=(T, F, N)))


def want(N, F, *blocks):
    e = oracle.Engine(N, F)
    for b in blocks:
        e.correlate(b)
    return e.dump()[0]


def dev(b):
    import torch
    return torch.from_numpy(np.ascontiguousarray(b)).cuda()


@pytest.mark.parametrize("N,F,T", [(192, 3, 700), (96, 4, 1000), (40, 3, 500), (32, 2, 40000)])
def test_fresh_carried_and_after(N, F, T):
    """Clean start (stores or atomics into the destination), then a carried-over
    integration, then the accumulator's own path still works."""
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(N + T)
    a, b, c, d = (block(rng, T, F, N) for _ in range(4))
    print("fused", N, F, T, flush=True)
    with Plan([(N, F, T)]) as p:
        out, n = p.correlate_dump([dev(a)])
        got = out[0].cpu().numpy()
        assert n[0] == T and np.array_equal(got, want(N, F, a)), first_mismatch(got, want(N, F, a))
        p.correlate([dev(b)])                                   # earlier samples in the accumulator
        out, n = p.correlate_dump([dev(c)])
        got = out[0].cpu().numpy()
        assert n[0] == 2 * T and np.array_equal(got, want(N, F, b, c))
        p.correlate([dev(d)])                                   # accumulator restarted
        out, n = p.dump(to_host=True)
        assert n[0] == T and np.array_equal(out[0].numpy(), want(N, F, d))
        assert p.stats()["dumps"] == 3


def test_batched_mixed_slots():
    """Batched plan: two slots dumped by the fused call, one left integrating,
    one dumped without new samples; then the integrating one is dumped."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    rng = np.random.default_rng(7)
    shapes = [(192, 2, 600), (48, 3, 900), (40, 2, 333), (64, 2, 256)]
    first = [block(rng, t, f, n) for n, f, t in shapes]
    second = [block(rng, t, f, n) for n, f, t in shapes]
    print("fused batched", flush=True)
    with Plan(shapes) as p:
        p.correlate([dev(x) for x in first])
        outs = [p.new_output(0), None, p.new_output(2), p.new_output(3)]
        v = [dev(second[0]), dev(second[1]), dev(second[2]), dev(second[3][:0])]
        outs, n = p.correlate_dump(v, out=outs)
        for k in (0, 2):
            N, F, T = shapes[k]
            assert n[k] == 2 * T
            assert np.array_equal(outs[k].cpu().numpy(), want(N, F, first[k], second[k])), k
        N, F, T = shapes[3]
        assert n[3] == T and np.array_equal(outs[3].cpu().numpy(), want(N, F, first[3]))
        rest, m = p.dump(1, to_host=True)
        N, F, T = shapes[1]
        assert m[0] == 2 * T and np.array_equal(rest[0].numpy(), want(N, F, first[1], second[1]))
        torch.cuda.synchronize()


def test_matches_separate_calls_at_full_size_sampled():
    """Cylinder shape (N=192, F=1024, T=8192): fused and separate calls give
    identical visibilities; sampled channels equal the oracle's."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    N, F, T = 192, 1024, 8192
    g = torch.Generator(device="cuda").manual_seed(3)
    v = torch.randint(0, 256, (T, F, N), dtype=torch.uint8, device="cuda", generator=g)
    print("fused full size", flush=True)
    with Plan([(N, F, T)]) as p:
        fused, _ = p.correlate_dump([v])
        p.correlate([v])
        sep, _ = p.dump()
        torch.cuda.synchronize()
        assert torch.equal(fused[0], sep[0])
    chans = [0, 511, 1023]
    vh = v[:, chans].cpu().numpy()
    got = fused[0][chans].cpu().numpy()
    assert np.array_equal(got, want(N, len(chans), vh))


def test_destination_errors():
    import torch
    from paper_1904_07778_amd import xeng as X
    with X.Plan([(32, 2, 64)]) as p:
        v = torch.full((64, 2, 32), 0x11, dtype=torch.uint8, device="cuda")
        host = torch.zeros((2, 528, 2), dtype=torch.int32)
        with pytest.raises(RuntimeError, match="device memory"):
            X.xeng_correlate_dump(p.handle, [v], [64], [host])
        d = torch.zeros(2 * 528 * 2 + 1, dtype=torch.int32, device="cuda")
        with pytest.raises(RuntimeError, match="aligned"):
            X.xeng_correlate_dump(p.handle, [v], [64], [d.data_ptr() + 4])
        out, n = p.correlate_dump([v])                           # the plan still works
        assert n[0] == 64 and int(out[0].abs().sum()) > 0
