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
