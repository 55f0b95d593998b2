"""GPU: one vector per call.

A call with one vector takes the small-launch shapes (single 4 KiB gather
tiles, the split survivor step); its outputs must be bit-identical to the
vector's row of a large call at the same stream position, and agree with the
oracle to the same bounds as the other streaming-step tests."""
import pytest
import torch

from gpu_common import need_gpu
from test_gpu_parity import check_case, prepare, rand_A, run_case, unit_rows

pytestmark = pytest.mark.gpu

KEYS = ("samples", "coef", "mu", "survivors", "values")


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_single_vector_equals_its_row_of_a_batch(monkeypatch, dtype):
    """One vector per call against its row of a 300-vector call, at the same
    stream position (every output, the debug outputs included)."""
    kd = need_gpu()
    monkeypatch.setenv("KERDOCK_BUCKET", "0")
    n = 1024
    A = rand_A(n, n, 31)
    X = torch.from_numpy(unit_rows(300, n, 32)).cuda()
    h = prepare(kd, A, dtype)
    eps, s_max, J, K = 0.06, 64, 150, 2
    big = kd.kerdock_sparse_apply(h, X, eps, s_max, J, K, 9, t0=500, debug=True)
    for t in (0, 1, 150, 299):
        one = kd.kerdock_sparse_apply(h, X[t:t + 1], eps, s_max, J, K, 9, t0=500 + t, debug=True)
        for u, v in zip(big[:3], one[:3]):
            assert torch.equal(u[t:t + 1], v)
        for key in KEYS:
            assert torch.equal(big[3][key][t:t + 1], one[3][key]), key
    h.destroy()


@pytest.mark.parametrize("m,n,J,K,s_max", [(100, 100, 50, 2, 20), (300, 100, 64, 4, 40),
                                           (2048, 2048, 96, 2, 320), (600, 3000, 47, 8, 50)])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_single_vector_parity(orc, m, n, J, K, s_max, dtype):
    """One vector per call against the oracle (short grouped columns, single
    tiles, n > 2048 with 47 draws per chunk: a partial last round of loads)."""
    need_gpu()
    from paper_2105_05879_amd import kerdock as kd
    A64, X64, g, r, info, eps = run_case(orc, kd, m, n, J, K, s_max, dtype, B=1)
    check_case(orc, A64, X64, g, r, info, eps, J, K, s_max, dtype)
