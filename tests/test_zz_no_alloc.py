"""The allocation-free variant of lbm_column_moments (for callers that cannot
allocate device memory) against the allocating entry point, through the C
ABI: the same kernel and host arithmetic, so the results must agree bit for
bit, on two calls in a row (the second smaller, so that stale sums of the
first call in the shared static array would show), plus the size limit."""
import ctypes

import numpy as np
import pytest

import paper_2605_02185_amd as lbm
from paper_2605_02185_amd import _lib

pytestmark = pytest.mark.gpu


def _call(fn, x, stream):
    M, nc = x.shape
    mean, std = np.full(nc, np.nan), np.full(nc, np.nan)
    st = fn(ctypes.c_void_p(x.data_ptr()), M, nc, mean.ctypes.data, std.ctypes.data, ctypes.c_void_p(stream))
    return st, mean, std


def test_noalloc_moments_match_the_allocating_entry_point_on_two_calls():
    import torch

    stream = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(31)
    shapes = [(20000, 4096), (3001, 37)]
    for M, nc in shapes:
        a = rng.standard_normal((M, nc)) * rng.uniform(0.1, 3.0, nc) + rng.uniform(-2, 2, nc)
        x = torch.from_numpy(a.astype(np.float32)).cuda()
        st0, m0, s0 = _call(_lib.lib.lbm_column_moments_noalloc, x, stream)
        st1, m1, s1 = _call(_lib.lib.lbm_column_moments, x, stream)
        assert st0 == 0 and st1 == 0, _lib.lib.lbm_last_error()
        assert np.array_equal(m0, m1) and np.array_equal(s0, s1), (M, nc)
        # and both are the moments of the data (FP64 sums of FP32 values)
        a32 = a.astype(np.float32).astype(np.float64)
        assert np.allclose(m0, a32.mean(0), rtol=1e-12, atol=1e-12)
        assert np.allclose(s0, a32.std(0), rtol=1e-9, atol=1e-12)


def test_noalloc_moments_reject_more_columns_than_the_scratch_holds():
    import torch

    x = torch.zeros((2, 4097), dtype=torch.float32, device="cuda")
    st, _, _ = _call(_lib.lib.lbm_column_moments_noalloc, x, torch.cuda.current_stream().cuda_stream)
    assert st == lbm._lib.ERR_INVALID_ARG
    assert b"4096" in _lib.lib.lbm_last_error()
