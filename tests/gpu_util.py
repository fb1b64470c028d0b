"""Helpers shared by the GPU tests: run the HIP engine through the C ABI."""
import numpy as np


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def run_engine(blocks, N, F, max_t=None, keep_dumps=()):
    """Integrate numpy uint8 blocks [T, F, N] in order on the GPU, dump to host.

    Returns (vis int32 [F, nbl, 2] numpy, n_integrated)."""
    import torch
    from paper_1904_07778_amd.xeng import Plan
    max_t = max_t or max(1, max(b.shape[0] for b in blocks))
    with Plan([(N, F, max_t)]) as p:
        for b in blocks:
            p.correlate([torch.from_numpy(np.ascontiguousarray(b)).cuda()])
        out, n = p.dump(to_host=True)
    return out[0].numpy(), n[0]


def first_mismatch(got, want):
    bad = np.argwhere(got != want)
    return f"{len(bad)} mismatches, first at {tuple(bad[0])}: got {got[tuple(bad[0])]} want {want[tuple(bad[0])]}" if len(bad) else ""


KIND_X16, KIND_X32, KIND_STAGE = 0, 1, 2


class forced_kernel:
    """Context: plain plans of (N, F, max_time_per_call) made inside it use the
    given tile shape (a one-line tuning cache; the cache is cleared on exit)."""

    def __init__(self, N, F, max_t, kind, split=2):
        self.line = (N, F, max_t, kind, split)

    def __enter__(self):
        import os
        import tempfile
        import torch
        from paper_1904_07778_amd import xeng as X
        N, F, max_t, kind, split = self.line
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        bucket = lambda v: max(0, int(v - 1).bit_length())   # ceil(log2 v), the cache's buckets
        fd, path = tempfile.mkstemp(suffix=".txt")
        with os.fdopen(fd, "w") as fh:
            fh.write(f"{arch} 0 {N} {bucket(F)} {bucket(max_t)} {kind} {split} 0\n")
        X.xeng_tune_cache_clear()
        X.xeng_tune_cache_load(path)
        os.unlink(path)
        return self

    def __exit__(self, *exc):
        from paper_1904_07778_amd import xeng as X
        X.xeng_tune_cache_clear()
