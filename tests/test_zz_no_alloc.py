"""The allocation-free entry point (kerdock_sparse_apply_static) against
kerdock_sparse_apply: the same kernels and draws on the library's fixed
device scratch, so the outputs and debug dumps must be equal bit for bit;
two calls in a row (the second with fewer vectors and other sizes, so the
scratch holds the first call's contents), and sizes beyond the scratch are
rejected before any launch."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


def unit_rows(B, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, n))
    return torch.from_numpy((X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)).cuda()


def outputs(B, s_max):
    return (torch.full((B, s_max), -9, dtype=torch.int32, device="cuda"),
            torch.full((B, s_max), -9.0, dtype=torch.float32, device="cuda"),
            torch.full((B,), -9, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_static_equals_allocating_entry(orc, dtype):
    kd = need_gpu()
    rng = np.random.default_rng(1)
    n = 1000
    A = torch.from_numpy((rng.standard_normal((1200, n)) / np.sqrt(n)).astype(np.float32)).cuda()
    h = kd.kerdock_prepare(A, dtype)
    calls = [  # (batch, J, K, s_max, seed, t0): the second call is smaller
        (300, 700, 3, 60, 11, 5),
        (37, 129, 2, 25, 12, 1000),
    ]
    for B, J, K, s_max, seed, t0 in calls:
        X = unit_rows(B, n, seed)
        ref = kd.kerdock_sparse_apply(h, X, 0.04, s_max, J, K, seed, t0=t0, debug=True)
        got = kd.kerdock_sparse_apply_static(h, X, 0.04, s_max, J, K, seed, t0=t0, out=outputs(B, s_max),
                                             debug=True)
        torch.cuda.synchronize()
        for a, b in zip(ref[:3], got[:3]):
            assert torch.equal(a, b)
        for key in ref[3]:
            assert torch.equal(ref[3][key], got[3][key]), key
        assert (ref[2] > 0).any()
    h.destroy()


def test_static_rejects_sizes_beyond_scratch(orc):
    kd = need_gpu()
    rng = np.random.default_rng(2)
    A = torch.from_numpy((rng.standard_normal((2048, 2048)) / 45).astype(np.float32)).cuda()
    h = kd.kerdock_prepare(A, "bf16")
    X = unit_rows(512, 2048, 3)
    # 512 vectors x 80 partial sums x 2048 rows x 4 bytes = 335 MB > 64 MiB
    with pytest.raises(kd.KerdockError) as e:
        kd.kerdock_sparse_apply_static(h, X, 0.05, 320, 40960, 1, 4, out=outputs(512, 320))
    assert e.value.code == -1 and "scratch" in str(e.value)
    # a smaller call on the same handle still works and equals the other entry point
    ref = kd.kerdock_sparse_apply(h, X[:8], 0.05, 320, 40960, 1, 4)
    got = kd.kerdock_sparse_apply_static(h, X[:8], 0.05, 320, 40960, 1, 4, out=outputs(8, 320))
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    # timing needs events, which the allocation-free entry point does not create
    with pytest.raises(kd.KerdockError):
        kd._sparse_apply("kerdock_sparse_apply_static", h, X[:2], 0.05, 8, 64, 1, 0, 0, 0.0, None, False, None,
                         (ctypes.c_float * 4)(), 0)
    h.destroy()
