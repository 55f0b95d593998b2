"""Batched form on the GPU: several matrices of different n in one persistent
launch, graph capture and replay, autotuning.

The persistent kernel runs the same device code as the single-handle path,
with the same draws per workgroup, so its outputs must equal the per-handle
kerdock_sparse_apply outputs bit for bit; every handle of a multi launch is
also checked against the oracle directly (all three table types, and the
n = 4096 BF16 matrix of the batched workload)."""
import numpy as np
import pytest
import torch

from gpu_common import check_outputs, need_gpu

pytestmark = pytest.mark.gpu


def unit_rows(B, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, n))
    return torch.from_numpy((X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)).cuda()


def setup(kd, dtype, shapes, seed=0, keep_A=False):
    hs, Xs, As = [], [], []
    for q, (m, n, B) in enumerate(shapes):
        rng = np.random.default_rng(seed + q)
        A = torch.from_numpy((rng.standard_normal((m, n)) / np.sqrt(n)).astype(np.float32)).cuda()
        hs.append(kd.kerdock_prepare(A, dtype))
        Xs.append(unit_rows(B, n, seed + 10 + q))
        As.append(A.cpu().numpy().astype(np.float64) if keep_A else None)
        del A
    return (hs, Xs, As) if keep_A else (hs, Xs)


SHAPES = [(64, 64, 3), (300, 100, 5), (1000, 1000, 4), (2048, 2048, 2), (700, 3000, 3)]
PARAMS = [dict(J=41, K=3, seed=11, t0=7), dict(J=130, K=2, seed=12, t0=0),
          dict(J=700, K=1, seed=13, t0=100), dict(J=257, K=4, seed=14, t0=5),
          dict(J=90, K=5, seed=15, t0=1 << 33)]
S_MAX = [10, 40, 64, 320, 100]
EPS = 0.04


def single_outputs(kd, hs, Xs):
    res = []
    for h, X, p, sm in zip(hs, Xs, PARAMS, S_MAX):
        res.append(kd.kerdock_sparse_apply(h, X, EPS, sm, p["J"], p["K"], p["seed"], t0=p["t0"]))
    torch.cuda.synchronize()
    return res


def assert_same(a, b):
    for (i1, v1, c1), (i2, v2, c2) in zip(a, b):
        assert torch.equal(c1, c2)
        assert torch.equal(i1, i2)
        assert torch.equal(v1, v2)


@pytest.mark.parametrize("bucket", ["0", "1"])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_multi_equals_single(orc, monkeypatch, dtype, bucket):
    kd = need_gpu()
    monkeypatch.setenv("KERDOCK_BUCKET", bucket)
    hs, Xs = setup(kd, dtype, SHAPES)
    ref = single_outputs(kd, hs, Xs)
    got = kd.kerdock_sparse_apply_multi(hs, Xs, PARAMS, EPS, S_MAX)
    assert_same(ref, got)
    for h in hs:
        h.destroy()


MODES = {"f32": "exact", "bf16": "bf16", "fp8": "fp8"}


def multi_vs_oracle(orc, kd, dtype, shapes, params, s_max, seed):
    hs, Xs, As = setup(kd, dtype, shapes, seed=seed, keep_A=True)
    got = kd.kerdock_sparse_apply_multi(hs, Xs, params, EPS, s_max)
    torch.cuda.synchronize()
    infos = [h.info for h in hs]
    outs = [tuple(o.cpu().numpy() for o in out) for out in got]
    Xn = [X.cpu().numpy().astype(np.float64) for X in Xs]
    for h in hs:
        h.destroy()
    del got, Xs
    torch.cuda.empty_cache()
    exc = 0
    for q, (A64, X64, p, sm, info) in enumerate(zip(As, Xn, params, s_max, infos)):
        r = orc.sparse_apply(A64, X64, p["J"], p["K"], EPS, sm, seed=p["seed"], t0=p["t0"],
                             table_mode=MODES[dtype], debug=True)
        idx, val, cnt = outs[q]
        exc += check_outputs(orc, A64, X64, idx, val, cnt, r, info, EPS, p["J"], p["K"], sm, dtype)
    return exc


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_multi_against_oracle(orc, dtype):
    """Every handle of one persistent launch against the oracle's run of
    Algorithm 1 on the same draws (outputs: exact values, rows equal up to
    FP32 near-ties of the selection)."""
    kd = need_gpu()
    assert multi_vs_oracle(orc, kd, dtype, SHAPES, PARAMS, S_MAX, seed=50) <= 2


def test_multi_n4096_bf16_against_oracle(orc):
    """The batched workload's largest matrix (n = 4096, BF16 table of
    68.8 GB) inside a multi-handle launch with a small one, against the
    oracle."""
    kd = need_gpu()
    shapes = [(4096, 4096, 3), (256, 256, 5)]
    params = [dict(J=64, K=2, seed=31, t0=3), dict(J=300, K=1, seed=32, t0=0)]
    assert multi_vs_oracle(orc, kd, "bf16", shapes, params, [64, 40], seed=60) <= 1


def test_multi_graph_replays(orc):
    kd = need_gpu()
    hs, Xs = setup(kd, "bf16", SHAPES, seed=40)
    plan = kd.kerdock_multi_create(hs, Xs, PARAMS, EPS, S_MAX)
    t0s = [p["t0"] for p in PARAMS]
    # eager references at consecutive stream positions
    eager = []
    kd.kerdock_multi_set_position(plan, t0s)
    for r in range(3):
        kd.kerdock_multi_run(plan)
        torch.cuda.synchronize()
        eager.append([tuple(o.clone() for o in out) for out in plan.outs])
    # the eager runs equal single-handle calls at the advanced positions
    for r in range(3):
        for q, (h, X, p, sm) in enumerate(zip(hs, Xs, PARAMS, S_MAX)):
            one = kd.kerdock_sparse_apply(h, X, EPS, sm, p["J"], p["K"], p["seed"], t0=p["t0"] + r * X.shape[0])
            assert_same([one], [eager[r][q]])
    # graph replays, with eager work and synchronisations between them
    kd.kerdock_multi_set_position(plan, t0s)
    for r in range(3):
        for out in plan.outs:
            for o in out:
                o.fill_(-7)
        junk = torch.randn(1 << 20, device="cuda").sum()     # unrelated eager work
        kd.kerdock_multi_graph_launch(plan)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert_same(eager[r], plan.outs)
    plan.destroy()
    for h in hs:
        h.destroy()


def test_multi_autotune_keeps_results(orc):
    kd = need_gpu()
    hs, Xs = setup(kd, "bf16", SHAPES[:3], seed=70)
    params, s_max = PARAMS[:3], S_MAX[:3]
    plan = kd.kerdock_multi_create(hs, Xs, params, EPS, s_max)
    kd.kerdock_multi_run(plan)
    torch.cuda.synchronize()
    before = [tuple(o.clone() for o in out) for out in plan.outs]
    u = kd.kerdock_multi_autotune(plan)
    assert u in (2, 4, 8, 16)
    kd.kerdock_multi_set_position(plan, [p["t0"] for p in params])
    kd.kerdock_multi_run(plan)
    torch.cuda.synchronize()
    assert_same(before, plan.outs)
    plan.destroy()
    for h in hs:
        h.destroy()


def test_single_autotune_then_parity(orc):
    """After autotuning (which may change the draws per workgroup, hence the
    FP32 summation order) the outputs still match the oracle."""
    from test_gpu_parity import check_case
    kd = need_gpu()
    rng = np.random.default_rng(3)
    A = (rng.standard_normal((1000, 1000)) / 32).astype(np.float32)
    X = unit_rows(3, 1000, 4)
    h = kd.kerdock_prepare(torch.from_numpy(A).cuda(), "bf16")
    c, u, ms = kd.kerdock_autotune(h, unit_rows(8, 1000, 5), 3000, 2)
    assert c in (256, 512, 1024) and u in (4, 8, 16) and ms > 0
    J, K, s_max, seed = 1500, 2, 50, 77
    A64, X64 = A.astype(np.float64), X.cpu().numpy().astype(np.float64)
    eps = float(np.quantile(np.abs(X64 @ A64.T), 0.9))
    idx, val, cnt, dbg = kd.kerdock_sparse_apply(h, X, eps, s_max, J, K, seed, debug=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in dbg.items()}
    g.update(idx=idx.cpu().numpy(), val=val.cpu().numpy(), cnt=cnt.cpu().numpy())
    r = orc.sparse_apply(A64, X64, J, K, eps, s_max, seed=seed, table_mode="bf16", debug=True)
    assert check_case(orc, A64, X64, g, r, h.info, eps, J, K, s_max, "bf16", chunk=1024) <= 1
    h.destroy()


def test_multi_errors(orc):
    kd = need_gpu()
    hs, Xs = setup(kd, "bf16", SHAPES[:2], seed=90)
    with pytest.raises(kd.KerdockError):
        kd.kerdock_sparse_apply_multi(hs, Xs, [dict(J=0, K=1), dict(J=5, K=1)], EPS, [4, 4])
    with pytest.raises(kd.KerdockError):
        kd.kerdock_sparse_apply_multi(hs, Xs, PARAMS[:2], EPS, [4, 10_000])
    other = kd.kerdock_prepare(torch.zeros((8, 8), device="cuda"), "f32")
    with pytest.raises(kd.KerdockError):
        kd.kerdock_sparse_apply_multi([hs[0], other], [Xs[0], unit_rows(2, 8, 1)], PARAMS[:2], EPS, [4, 4])
    other.destroy()
    for h in hs:
        h.destroy()
