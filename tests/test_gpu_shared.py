"""Shared-draw form on the GPU: the draws of a group of 64 rows of X come
from one stream position, the batch sums run as a matrix product on the
matrix cores (FP32 for FP32 tables; BF16 with coefficients split into three
exact BF16 parts for BF16 and FP8 tables).  Against the FP64 oracle in its
shared-draw mode: draws bit-exact, coefficients and median of means within
the FP32 bounds (the summation order of the matrix product is not
sequential, so the bound for its number of terms in any order is used),
selections up to near-ties, survivor values 1e-5 relative."""
import numpy as np
import pytest
import torch

from gpu_common import need_gpu, shared_terms
from test_gpu_parity import check_case, rand_A, unit_rows

pytestmark = pytest.mark.gpu

TILE = 64

SHARED_CASES = [
    # m, n, B, J, K, s_max
    (16, 16, 3, 9, 3, 4),
    (100, 100, 70, 50, 3, 20),
    (300, 100, 130, 37, 2, 40),
    (70, 300, 65, 64, 1, 30),
    (1000, 1000, 64, 130, 2, 60),        # three 64-draw stages: a pair and a last single one
    (80, 120, 64, 100, 2, 24),           # two stages: one pair, no single last stage
    (128, 64, 3, 65, 1, 8),              # a pair whose second stage holds one draw
    (200, 64, 1, 128, 3, 16),            # one vector; exactly one pair per batch
    (300, 256, 65, 192, 1, 32),          # a pair and a full last single stage
    (64, 128, 130, 257, 2, 24),          # two pairs and a one-draw last stage, ragged group
    (64, 64, 70, 4099, 1, 16),          # two slices, the second with a ragged end
    (40, 100, 65, 4101, 2, 12),         # two batches of two ragged slices each
    (50, 50, 66, 21, 5, 10),            # five batches: median of five means
]


def run_shared(orc, kd, m, n, B, J, K, s_max, dtype, seed=4001, t0=3, tau=0.0):
    A = rand_A(m, n, m * 17 + n)
    A64 = A.astype(np.float64)
    X = unit_rows(B, n, m + 5 * n)
    X64 = X.astype(np.float64)
    eps = float(np.quantile(np.abs(X64 @ A64.T), 0.9)) + 1e-6
    h = kd.kerdock_prepare(torch.from_numpy(A).cuda(), dtype)
    idx, val, cnt, dbg = kd.kerdock_sparse_apply_shared(h, torch.from_numpy(X).cuda(), eps, s_max, J, K, seed,
                                                        t0=t0, tau=tau, debug=True)
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in dbg.items()}
    g.update(idx=idx.cpu().numpy(), val=val.cpu().numpy(), cnt=cnt.cpu().numpy())
    mode = {"f32": "exact", "bf16": "bf16", "fp8": "fp8"}[dtype]
    r = orc.sparse_apply(A64, X64, J, K, eps, s_max, seed=seed, t0=t0, tau=tau, table_mode=mode, debug=True,
                         tile=TILE)
    info = h.info
    h.destroy()
    return A64, X64, g, r, info, eps


@pytest.mark.parametrize("m,n,B,J,K,s_max", SHARED_CASES)
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_shared_parity(orc, m, n, B, J, K, s_max, dtype):
    kd = need_gpu()
    A64, X64, g, r, info, eps = run_shared(orc, kd, m, n, B, J, K, s_max, dtype)
    # rows of one group share their draws
    for t in range(B):
        assert np.array_equal(g["samples"][t], g["samples"][(t // TILE) * TILE])
    exc = check_case(orc, A64, X64, g, r, info, eps, J, K, s_max, dtype, chunk=J, terms=shared_terms(J, dtype))
    assert exc <= 1


def test_shared_top_digit_plane(orc):
    """Coefficients are exact sums over four base-256 digit planes of the
    fixed-point x; a group whose vectors all have a zero top plane skips it.
    The top plane is nonzero when an entry exceeds about 2^-7 of the vector's
    l1 norm.  Group 0 holds dense unit vectors of n = 1024 (entries near
    2^-8 of the l1 norm at most: top plane zero), group 1 adds a near one-hot
    vector (top plane nonzero): both paths in one call, against the oracle."""
    kd = need_gpu()
    m, n, B, J, K, s_max = 64, 1024, 128, 40, 2, 12
    A = rand_A(m, n, 91)
    X = unit_rows(B, n, 92)
    spike = np.zeros(n, dtype=np.float64)
    spike[5] = 1.0
    spike += 1e-3 * np.random.default_rng(93).standard_normal(n)
    X[70] = (spike / np.linalg.norm(spike)).astype(np.float32)
    A64, X64 = A.astype(np.float64), X.astype(np.float64)
    eps = float(np.quantile(np.abs(X64 @ A64.T), 0.9)) + 1e-6
    for dtype in ("f32", "bf16"):
        h = kd.kerdock_prepare(torch.from_numpy(A).cuda(), dtype)
        idx, val, cnt, dbg = kd.kerdock_sparse_apply_shared(h, torch.from_numpy(X).cuda(), eps, s_max, J, K, 515,
                                                            debug=True)
        torch.cuda.synchronize()
        g = {key: v.cpu().numpy() for key, v in dbg.items()}
        g.update(idx=idx.cpu().numpy(), val=val.cpu().numpy(), cnt=cnt.cpu().numpy())
        mode = {"f32": "exact", "bf16": "bf16"}[dtype]
        r = orc.sparse_apply(A64, X64, J, K, eps, s_max, seed=515, table_mode=mode, debug=True, tile=TILE)
        info = h.info
        h.destroy()
        assert check_case(orc, A64, X64, g, r, info, eps, J, K, s_max, dtype, chunk=J,
                          terms=shared_terms(J, dtype)) <= 1


def test_shared_groups_follow_stream_position(orc):
    """A batch of 128 equals two calls of 64 rows at t0 and t0 + 1."""
    kd = need_gpu()
    A = rand_A(200, 200, 9)
    X = torch.from_numpy(unit_rows(128, 200, 10)).cuda()
    h = kd.kerdock_prepare(torch.from_numpy(A).cuda(), "bf16")
    a = kd.kerdock_sparse_apply_shared(h, X, 0.1, 20, 40, 3, 11, t0=7, debug=True)
    b0 = kd.kerdock_sparse_apply_shared(h, X[:64], 0.1, 20, 40, 3, 11, t0=7, debug=True)
    b1 = kd.kerdock_sparse_apply_shared(h, X[64:], 0.1, 20, 40, 3, 11, t0=8, debug=True)
    for u, v0, v1 in zip(a[:3], b0[:3], b1[:3]):
        assert torch.equal(u[:64], v0) and torch.equal(u[64:], v1)
    for key in ("samples", "coef", "mu", "survivors", "values"):
        assert torch.equal(a[3][key][:64], b0[3][key]) and torch.equal(a[3][key][64:], b1[3][key])
    h.destroy()


def test_shared_errors(orc):
    kd = need_gpu()
    h = kd.kerdock_prepare(torch.from_numpy(rand_A(32, 32, 1)).cuda())
    X = torch.from_numpy(unit_rows(2, 32, 1)).cuda()
    with pytest.raises(kd.KerdockError):
        kd.kerdock_sparse_apply_shared(h, X, 0.1, 4, 1 << 22, 32, 0)      # J K = 2^27
    with pytest.raises(kd.KerdockError):
        kd.kerdock_sparse_apply_shared(h, X, 0.0, 4, 2, 2, 0)
    out = kd.kerdock_sparse_apply_shared(h, X[:0], 0.1, 4, 2, 2, 0)
    assert out[0].shape == (0, 4)
    h.destroy()
