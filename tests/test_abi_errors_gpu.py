"""Argument checking and error codes of the C ABI on a GPU."""
import numpy as np
import pytest

from tests.gpu_util import gpu_available

pytestmark = pytest.mark.gpu
if not gpu_available():
    pytestmark = [pytest.mark.gpu, pytest.mark.skip(reason="no GPU")]


def test_error_codes():
    import torch
    from paper_1904_07778_amd import xeng as X
    p = X.xeng_plan([(8, 2, 100)])
    try:
        v = torch.zeros((101, 2, 8), dtype=torch.uint8, device="cuda")
        with pytest.raises(X.XengError) as e:
            X.xeng_correlate(p, [v], [101])                    # T > max_time_per_call
        assert e.value.status == X.XENG_EINVAL
        with pytest.raises(X.XengError) as e:
            X.xeng_correlate(p, [v.data_ptr() + 1], [10])      # misaligned
        assert e.value.status == X.XENG_EINVAL
        with pytest.raises(X.XengError) as e:
            X.xeng_correlate(p, [None], [10])                  # null
        assert e.value.status == X.XENG_EINVAL
        X.xeng_correlate(p, [None], [0])                       # T = 0 skips
        out = torch.empty((2, 36, 2), dtype=torch.int32, device="cuda")
        with pytest.raises(X.XengError) as e:
            X.xeng_dump(p, 1, [out])                           # array index out of range
        assert e.value.status == X.XENG_EINVAL
        X.xeng_correlate(p, [v], [100])
        assert X.xeng_integrated(p, 0) == 100
        assert X.xeng_dump(p, 0, [out]) == [100]
        assert X.xeng_integrated(p, 0) == 0
    finally:
        X.xeng_destroy(p)
