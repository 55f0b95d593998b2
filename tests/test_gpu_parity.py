"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bit-exact: sign patterns, drawn design indices.  Within derived FP32 bounds:
table entries (FWHT rounding), coefficients, median-of-means estimates.
Selections: identical up to FP32 near-ties at the s_max-th value.  Survivor
values: 1e-5 relative (compensated dot product from FP32 A and x)."""
import numpy as np
import pytest
import torch

from gpu_common import (U32, check_selection, coef_tol, entry_tolerance, mu_tolerance, need_gpu,
                        orc_scales, quant_interval_check, table_tol)
from paper_2105_05879_amd import workloads

pytestmark = pytest.mark.gpu

DTYPES = ["f32", "bf16", "fp8"]


def rand_A(m, n, seed):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((m, n)) / np.sqrt(n)).astype(np.float32)


def unit_rows(B, n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((B, n))
    return (X / np.linalg.norm(X, axis=1, keepdims=True)).astype(np.float32)


def prepare(kd, A, dtype):
    return kd.kerdock_prepare(torch.from_numpy(A).cuda(), dtype)


# --------------------------------------------------------------- signs ---

@pytest.mark.parametrize("n", [1, 4, 16, 64, 256, 1024, 4096])
def test_signs_and_field_bit_exact(orc, n):
    kd = need_gpu()
    h = prepare(kd, rand_A(4, n, n), "f32")
    k = orc.choose_k(n)
    assert h.info.k == k and h.info.d == 1 << k and h.info.L == orc.design_size(k)
    assert h.info.field_poly == orc.field_poly(k - 1)
    nb = (1 << k) // 2
    bases = range(nb) if nb <= 128 else sorted(set([0, 1, nb - 1] + list(
        np.random.default_rng(n).integers(0, nb, 61))))
    for b in bases:
        assert np.array_equal(np.array(kd.kerdock_debug_signs(h, b), dtype=np.uint32),
                              orc.sign_words(k, b)), "basis %d" % b
    h.destroy()


# --------------------------------------------------------------- tables ---

# (130, 257) and (33, 4095): d = 1024 and 4096 with n not a multiple of 4 (rows read element by
# element) and a partial last segment of a lane
TABLE_CASES = [(1, 1), (3, 4), (16, 16), (50, 50), (64, 64), (100, 100), (300, 100), (70, 300),
               (256, 256), (130, 257), (1000, 1000), (2048, 2048), (33, 4095)]


def pick_columns(L, d, n, count, seed):
    rng = np.random.default_rng(seed)
    nb = d // 2
    fixed = [0, d - 1, d, 2 * d - 1, (nb - 1) * d, nb * d - 1, nb * d, nb * d + n - 1, L - 1]
    if n < d:
        fixed.append(nb * d + n)
    cols = sorted(set([c for c in fixed if 0 <= c < L] + list(rng.integers(0, L, count))))
    return np.array(cols, dtype=np.int64)


@pytest.mark.parametrize("m,n", TABLE_CASES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_table_columns(orc, m, n, dtype):
    kd = need_gpu()
    A = rand_A(m, n, 7 * m + n)
    A64 = A.astype(np.float64)
    h = prepare(kd, A, dtype)
    k, d, L = h.info.k, h.info.d, h.info.L
    ells = pick_columns(L, d, n, 96, m + n)
    gpu = kd.kerdock_read_columns(h, torch.from_numpy(ells.astype(np.int32)).cuda()).cpu().numpy().astype(np.float64)
    ref = np.stack([orc.table_column(A64, l) for l in ells])
    tolT = np.broadcast_to(table_tol(A64, k)[None, :], ref.shape)
    if dtype == "f32":
        bad = np.abs(gpu - ref) > tolT
        assert not bad.any(), "max excess %g" % (np.abs(gpu - ref) - tolT).max()
    elif dtype == "bf16":
        assert quant_interval_check(orc, gpu, ref - tolT, ref + tolT, "bf16").all()
    else:
        s_orc = orc_scales(A64, d)
        s_gpu = kd.kerdock_row_scales(h).cpu().numpy().astype(np.float64)
        rel = 4 * n * U32
        assert np.all(np.abs(s_gpu / s_orc - 1) <= rel)
        q_gpu = orc.quant_e4m3(gpu / s_gpu[None, :])
        cands = [orc.quant_e4m3(v / (s_orc[None, :] * f))
                 for v in (ref - tolT, ref + tolT) for f in (1 - rel, 1 + rel)]
        lo, hi = np.minimum.reduce(cands), np.maximum.reduce(cands)
        assert np.all((q_gpu >= lo) & (q_gpu <= hi))
        assert np.all(np.abs(q_gpu) <= 448)
    h.destroy()


# ------------------------------------------------------ streaming step ---

APPLY_CASES = [
    # m, n, J, K, s_max
    (1, 1, 5, 1, 1),
    (16, 16, 9, 3, 4),
    (64, 64, 37, 3, 10),
    (100, 100, 50, 2, 20),
    (300, 100, 64, 4, 40),
    (70, 300, 33, 5, 70),
    (256, 256, 200, 1, 30),
    (1000, 1000, 130, 2, 60),
    (2048, 2048, 96, 2, 320),
]


def run_case(orc, kd, m, n, J, K, s_max, dtype, B=3, seed=3001, t0=5, tau=0.0, eps=None, chunk=0, A=None, X=None):
    if A is None:
        if m == n and n >= 64:
            A = workloads.structured_dictionary(n, np.random.default_rng(n)).astype(np.float32)
        else:
            A = rand_A(m, n, m * 31 + n)
    A64 = A.astype(np.float64)
    if X is None:
        X = unit_rows(B, n, m + 3 * n)
    X64 = X.astype(np.float64)
    if eps is None:
        eps = float(np.quantile(np.abs(X64 @ A64.T), 0.9)) + 1e-6
    h = prepare(kd, A, dtype)
    idx, val, cnt, dbg = kd.kerdock_sparse_apply(h, torch.from_numpy(X).cuda(), eps, s_max, J, K,
                                                  seed, t0=t0, tau=tau, debug=True, chunk=chunk)
    torch.cuda.synchronize()
    g = {key: v.cpu().numpy() for key, v in dbg.items()}
    g.update(idx=idx.cpu().numpy(), val=val.cpu().numpy(), cnt=cnt.cpu().numpy())
    mode = {"f32": "exact", "bf16": "bf16", "fp8": "fp8"}[dtype]
    r = orc.sparse_apply(A64, X64, J, K, eps, s_max, seed=seed, t0=t0, tau=tau, table_mode=mode, debug=True)
    info = h.info
    h.destroy()
    return A64, X64, g, r, info, eps


def check_case(orc, A64, X64, g, r, info, eps, J, K, s_max, dtype, tau=0.0, chunk=512, terms=None):
    k, d, n = info.k, info.d, A64.shape[1]
    exceptions = 0
    for t in range(X64.shape[0]):
        # draws: bit-exact
        assert np.array_equal(g["samples"][t].view(np.uint32).astype(np.int64), r["samples"][t])
        # coefficients
        ct = coef_tol(X64[t], n)
        assert np.all(np.abs(g["coef"][t] - r["coef"][t]) <= ct), np.abs(g["coef"][t] - r["coef"][t]).max()
        # median of means
        ref = np.stack([orc.table_column(A64, l) for l in r["samples"][t]])
        tolE, used = entry_tolerance(orc, ref, A64, k, d, dtype)
        mt = mu_tolerance(used, r["coef"][t], J, K, tolE, np.full(J * K, ct), chunk, terms)
        dmu = np.abs(g["mu"][t] - r["mu"][t])
        assert np.all(dmu <= mt), "mu excess %g" % (dmu - mt).max()
        # selection
        gs = g["survivors"][t]
        gset = gs[gs >= 0]
        assert np.all(np.diff(gset) > 0), "survivors not ascending"
        exceptions += check_selection(r["mu"][t], mt, gset.tolist(), s_max, tau)
        # survivor values: Dot2 vs FP64
        ns = len(gset)
        v64 = A64[gset] @ X64[t]
        gv = g["values"][t][:ns].astype(np.float64)
        scale = np.abs(A64[gset] * X64[t][None, :]).sum(1)
        assert np.all(np.abs(gv - v64) <= 1e-5 * np.abs(v64) + 4 * U32 * U32 * n * scale + 1e-30)
        assert np.all(g["values"][t][ns:] == 0)
        # threshold
        c = g["cnt"][t]
        keep = gset[np.abs(gv) >= eps]
        assert np.array_equal(g["idx"][t][:c], keep)
        assert np.all(g["idx"][t][c:] == -1) and np.all(g["val"][t][c:] == 0)
        assert np.array_equal(g["val"][t][:c], gv[np.abs(gv) >= eps].astype(np.float32))
        # against the oracle's output, rows outside near-ties agree exactly
        oc = r["out_cnt"][t]
        o_idx, o_val = r["out_idx"][t][:oc], r["out_val"][t][:oc]
        common = np.intersect1d(o_idx, keep)
        surv_diff = set(np.setxor1d(gset, r["surv"][t][r["surv"][t] >= 0]).tolist())
        for i in np.setxor1d(o_idx, keep):
            near_eps = abs(abs(A64[i] @ X64[t]) - eps) <= 1e-5 * eps
            assert near_eps or int(i) in surv_diff, "row %d kept by one side only" % i
        gv_map = dict(zip(g["idx"][t][:c].tolist(), g["val"][t][:c].tolist()))
        for i, v in zip(o_idx.tolist(), o_val.tolist()):
            if i in gv_map:
                assert abs(gv_map[i] - v) <= 1e-5 * abs(v)
    return exceptions


@pytest.mark.parametrize("bucket", ["0", "1"])
@pytest.mark.parametrize("m,n,J,K,s_max", APPLY_CASES)
@pytest.mark.parametrize("dtype", DTYPES)
def test_apply_parity(orc, monkeypatch, m, n, J, K, s_max, dtype, bucket):
    """Both orders of the draws: as drawn (bucket 0) and grouped by basis
    with the per-basis transform of the coefficients (bucket 1)."""
    kd = need_gpu()
    monkeypatch.setenv("KERDOCK_BUCKET", bucket)
    A64, X64, g, r, info, eps = run_case(orc, kd, m, n, J, K, s_max, dtype)
    exc = check_case(orc, A64, X64, g, r, info, eps, J, K, s_max, dtype)
    assert exc <= 1


# long runs of draws per basis (J several times d/2 + 1), where grouping the
# draws by basis and transforming each basis once pays; the last case has
# n > 2048 (two sign words per lane)
BUCKET_CASES = [
    (64, 64, 300, 2, 10),
    (256, 256, 2000, 2, 30),
    (300, 100, 1500, 3, 40),
    (70, 300, 2100, 2, 70),
    (40, 3000, 9000, 1, 20),
]


@pytest.mark.parametrize("bucket", ["0", "1"])
@pytest.mark.parametrize("m,n,J,K,s_max", BUCKET_CASES)
@pytest.mark.parametrize("dtype", ["f32", "fp8"])
def test_apply_parity_long_runs(orc, monkeypatch, m, n, J, K, s_max, dtype, bucket):
    kd = need_gpu()
    monkeypatch.setenv("KERDOCK_BUCKET", bucket)
    A64, X64, g, r, info, eps = run_case(orc, kd, m, n, J, K, s_max, dtype, B=2)
    assert check_case(orc, A64, X64, g, r, info, eps, J, K, s_max, dtype) <= 1


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_plain_workload_parity(orc, dtype):
    """The plain-method workload: n = 1024, A with i.i.d. N(0, 1/n) entries
    (general, not orthogonal), x = A^-1 y normalised with y 16-sparse, eps
    = 0.05, s_max = 10 s = 160; four of its vectors against the oracle."""
    kd = need_gpu()
    w = workloads.plain(batch=4)
    A64, X64, g, r, info, eps = run_case(orc, kd, 1024, 1024, 300, 3, 160, dtype, eps=w.eps, A=w.A, X=w.X)
    assert check_case(orc, A64, X64, g, r, info, eps, 300, 3, 160, dtype) <= 1


@pytest.mark.parametrize("dtype", ["f32", "fp8"])
def test_tall_matrix_at_the_row_cap(orc, dtype):
    """m = 16384 rows, the largest m that kerdock_prepare accepts: the
    selection stages one key per row (64 KiB) in LDS."""
    kd = need_gpu()
    A64, X64, g, r, info, eps = run_case(orc, kd, 16384, 64, 40, 2, 100, dtype, B=2)
    assert check_case(orc, A64, X64, g, r, info, eps, 40, 2, 100, dtype) <= 1


def test_apply_tau_and_take_all(orc):
    kd = need_gpu()
    for tau, s_max in [(0.05, 24), (0.0, 64)]:
        A64, X64, g, r, info, eps = run_case(orc, kd, 64, 64, 40, 2, s_max, "f32", tau=tau)
        check_case(orc, A64, X64, g, r, info, eps, 40, 2, s_max, "f32", tau=tau)


@pytest.mark.parametrize("K", [1, 2, 3, 6, 9, 16, 32])
def test_median_all_batch_counts(orc, K):
    kd = need_gpu()
    A64, X64, g, r, info, eps = run_case(orc, kd, 64, 64, 7, K, 12, "f32", B=2)
    check_case(orc, A64, X64, g, r, info, eps, 7, K, 12, "f32")


@pytest.mark.parametrize("chunk", [1, 3, 47, 1024])
def test_chunk_parameter(orc, chunk):
    """An explicit number of draws per FP32 partial sum, from one draw per
    partial to more than J."""
    kd = need_gpu()
    A64, X64, g, r, info, eps = run_case(orc, kd, 100, 100, 300, 3, 20, "f32", chunk=chunk)
    check_case(orc, A64, X64, g, r, info, eps, 300, 3, 20, "f32", chunk=chunk)


@pytest.mark.parametrize("bucket", ["0", "1"])
@pytest.mark.parametrize("dtype", DTYPES)
def test_results_do_not_depend_on_batch_size(orc, monkeypatch, dtype, bucket):
    """Launch shapes change with the batch (single-tile gather workgroups and
    the split survivor step below 2048 vectors); the outputs of a vector
    depend only on its stream position."""
    kd = need_gpu()
    monkeypatch.setenv("KERDOCK_BUCKET", bucket)
    n = 1200                                   # 4800-byte FP32 columns: two tiles
    A = rand_A(n, n, 21)
    X = torch.from_numpy(unit_rows(2100, n, 22)).cuda()
    h = prepare(kd, A, dtype)
    eps, s_max, J, K = 0.08, 40, 24, 3
    big = kd.kerdock_sparse_apply(h, X, eps, s_max, J, K, 5, t0=1000, debug=True)
    for lo, hi in [(0, 1), (7, 12), (2000, 2100)]:
        part = kd.kerdock_sparse_apply(h, X[lo:hi], eps, s_max, J, K, 5, t0=1000 + lo, debug=True)
        for u, v in zip(big[:3], part[:3]):
            assert torch.equal(u[lo:hi], v)
        for key in ("mu", "survivors", "values"):
            assert torch.equal(big[3][key][lo:hi], part[3][key])
    h.destroy()


def test_deterministic(orc):
    kd = need_gpu()
    A = rand_A(256, 256, 5)
    X = torch.from_numpy(unit_rows(4, 256, 6)).cuda()
    h = prepare(kd, A, "bf16")
    a = kd.kerdock_sparse_apply(h, X, 0.05, 16, 300, 2, 9, debug=True)
    b = kd.kerdock_sparse_apply(h, X, 0.05, 16, 300, 2, 9, debug=True)
    for u, v in zip(a[:3], b[:3]):
        assert torch.equal(u, v)
    for key in a[3]:
        assert torch.equal(a[3][key], b[3][key])
    h.destroy()


def test_stream_position(orc):
    """Draws depend only on (seed, t0 + t, j): rows 1.. of a call with t0
    equal rows 0.. of a call with t0 + 1."""
    kd = need_gpu()
    h = prepare(kd, rand_A(64, 64, 1), "f32")
    X = torch.from_numpy(unit_rows(3, 64, 2)).cuda()
    a = kd.kerdock_sparse_apply(h, X, 0.1, 8, 20, 2, 77, t0=100, debug=True)
    b = kd.kerdock_sparse_apply(h, X[1:].contiguous(), 0.1, 8, 20, 2, 77, t0=101, debug=True)
    assert torch.equal(a[3]["samples"][1:], b[3]["samples"])
    h.destroy()


def test_errors(orc):
    kd = need_gpu()
    A = torch.from_numpy(rand_A(32, 32, 1)).cuda()
    with pytest.raises(kd.KerdockError) as e:
        kd.kerdock_prepare(torch.zeros((4, 5000), device="cuda"))
    assert e.value.code == -2
    with pytest.raises(kd.KerdockError) as e:
        kd.kerdock_prepare(torch.zeros((16385, 8), device="cuda"))
    assert e.value.code == -1
    # a table that cannot fit in HBM (16384 x 8,392,704 FP32 entries, 550 GB)
    with pytest.raises(kd.KerdockError) as e:
        kd.kerdock_prepare(torch.zeros((16384, 4096), device="cuda"), "f32")
    assert e.value.code == -3
    torch.cuda.empty_cache()
    h = kd.kerdock_prepare(A)
    X = torch.from_numpy(unit_rows(2, 32, 1)).cuda()
    for kw, code in [(dict(eps=0.0, s_max=4, J=2, K=2), -1), (dict(eps=0.1, s_max=33, J=2, K=2), -1),
                     (dict(eps=0.1, s_max=4, J=2, K=2, chunk=-1), -1),
                     (dict(eps=0.1, s_max=4, J=2, K=2, chunk=1025), -1),
                     (dict(eps=0.1, s_max=4, J=0, K=2), -1), (dict(eps=0.1, s_max=4, J=2, K=33), -1),
                     (dict(eps=float("nan"), s_max=4, J=2, K=2), -1)]:
        with pytest.raises(kd.KerdockError) as e:
            kd.kerdock_sparse_apply(h, X, seed=0, **kw)
        assert e.value.code == code
    # J K beyond the 32-bit draw counter, in every entry point that takes it
    for call in (lambda: kd.kerdock_sparse_apply(h, X, 0.1, 4, 1 << 30, 2, 0),
                 lambda: kd.kerdock_reserve(h, 2, 1 << 30, 2, 4),
                 lambda: kd.kerdock_autotune(h, X, 1 << 30, 2)):
        with pytest.raises(kd.KerdockError) as e:
            call()
        assert e.value.code == -1
    # empty batch is a no-op
    out = kd.kerdock_sparse_apply(h, X[:0], 0.1, 4, 2, 2, 0)
    assert out[0].shape == (0, 4)
    h.destroy()


def test_binding_rejects_bad_shapes(orc):
    """The Python binding checks shapes before any launch: an X of the wrong
    width or rank, or an output of the wrong shape or dtype, raises instead
    of letting a kernel read or write past an allocation."""
    kd = need_gpu()
    h = prepare(kd, rand_A(40, 32, 1), "f32")
    X = torch.from_numpy(unit_rows(3, 32, 1)).cuda()
    bad_outs = [(torch.empty((3, 3), dtype=torch.int32, device="cuda"),
                 torch.empty((3, 4), dtype=torch.float32, device="cuda"),
                 torch.empty((3,), dtype=torch.int32, device="cuda")),
                (torch.empty((3, 4), dtype=torch.int32, device="cuda"),
                 torch.empty((3, 4), dtype=torch.float64, device="cuda"),
                 torch.empty((3,), dtype=torch.int32, device="cuda")),
                (torch.empty((3, 4), dtype=torch.int32, device="cuda"),
                 torch.empty((3, 4), dtype=torch.float32, device="cuda"),
                 torch.empty((2,), dtype=torch.int32, device="cuda"))]
    for fn in (kd.kerdock_sparse_apply, kd.kerdock_sparse_apply_shared):
        for Xb in (X[:, :31].contiguous(), torch.zeros((3, 33), device="cuda"), X.view(-1)):
            with pytest.raises(ValueError):
                fn(h, Xb, 0.1, 4, 8, 2, 0)
        for out in bad_outs:
            with pytest.raises((ValueError, TypeError)):
                fn(h, X, 0.1, 4, 8, 2, 0, out=out)
    with pytest.raises(ValueError):
        kd.kerdock_features(h, torch.zeros((2, 16), device="cuda"))
    with pytest.raises(ValueError):
        kd.kerdock_sparse_apply_multi([h], [torch.zeros((2, 16), device="cuda")], [dict(J=4, K=1)], 0.1, [4])
    h.destroy()


@pytest.mark.parametrize("shared", [False, True])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_non_finite_input_is_flagged(orc, shared, dtype):
    """An inf or NaN in x makes the survivor values non-finite: count -1 and
    all-padding rows for that vector, the other vectors unaffected (in the
    shared-draw form too, where all four vectors are one group and a vector
    alone at t0 = 0 uses the same draws)."""
    kd = need_gpu()
    A = rand_A(64, 64, 7)
    Xn = unit_rows(4, 64, 8)
    Xn[1, 5] = np.nan
    Xn[2, 9] = np.inf
    h = prepare(kd, A, dtype)
    fn = kd.kerdock_sparse_apply_shared if shared else kd.kerdock_sparse_apply
    idx, val, cnt = fn(h, torch.from_numpy(Xn).cuda(), 0.05, 8, 40, 2, 11, t0=0)
    torch.cuda.synchronize()
    assert cnt[1].item() == -1 and cnt[2].item() == -1
    assert torch.all(idx[1:3] == -1) and torch.all(val[1:3] == 0)
    for t in (0, 3):
        ref = fn(h, torch.from_numpy(Xn[t:t + 1]).cuda(), 0.05, 8, 40, 2, 11, t0=0 if shared else t)
        assert torch.equal(ref[0][0], idx[t]) and torch.equal(ref[1][0], val[t]) and ref[2][0].item() == cnt[t].item()
        assert cnt[t].item() >= 0
    h.destroy()


def test_graph_capture_replays(orc):
    """A call whose workspace is already sized allocates nothing and records
    only kernels, so it can be captured in a HIP graph: every replay (with
    unrelated eager work in between) reproduces the eager outputs."""
    kd = need_gpu()
    A = rand_A(300, 256, 3)
    X = torch.from_numpy(unit_rows(40, 256, 4)).cuda()
    h = prepare(kd, A, "bf16")
    for fn in (kd.kerdock_sparse_apply, kd.kerdock_sparse_apply_shared):
        out = (torch.empty((40, 24), dtype=torch.int32, device="cuda"),
               torch.empty((40, 24), dtype=torch.float32, device="cuda"),
               torch.empty((40,), dtype=torch.int32, device="cuda"))
        fn(h, X, 0.05, 24, 64, 3, 5, t0=9, out=out)           # sizes the workspace
        torch.cuda.synchronize()
        ref = tuple(o.clone() for o in out)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn(h, X, 0.05, 24, 64, 3, 5, t0=9, out=out)
        for r in range(3):
            for o in out:
                o.fill_(-3)
            junk = torch.randn(1 << 20, device="cuda").sum()
            g.replay()
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            for a, b in zip(ref, out):
                assert torch.equal(a, b)
        del g
    h.destroy()


def test_zero_matrix(orc):
    kd = need_gpu()
    h = prepare(kd, np.zeros((40, 40), dtype=np.float32), "fp8")
    X = torch.from_numpy(unit_rows(2, 40, 3)).cuda()
    idx, val, cnt = kd.kerdock_sparse_apply(h, X, 0.01, 5, 10, 3, 1)
    assert cnt.sum().item() == 0 and (idx == -1).all()
    h.destroy()
