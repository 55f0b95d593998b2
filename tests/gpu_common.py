"""Shared helpers of the GPU parity tests: tolerances derived from the FP32
arithmetic of each kernel, and the near-tie rule for row selections."""
import numpy as np
import pytest

U32 = 2.0 ** -24


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_05879_amd import kerdock
    kerdock.lib()          # raises when the HIP library is missing
    return kerdock


def table_tol(A64, k):
    """|T32 - T| for a Kerdock entry: k butterfly levels, each adding one
    rounding of a partial sum bounded by sum_x |a_ix|."""
    return (k + 1) * U32 * np.abs(A64).sum(1) * 1.01 + 1e-30


def coef_tol(x64, n):
    """c = s^T x on the GPU: an exact integer signed sum of x rounded to a
    fixed-point grid of spacing <= |x|_1 2^-29 (n roundings of half a step),
    then one FP32 rounding; also covers a plain FP32 summation (32 or 64
    sequential adds per lane and a 6-level cross-lane tree)."""
    P = 1 if n <= 2048 else 2
    a = np.abs(x64).sum()
    return max((32 * P + 8) * U32, n * 2.0 ** -30 + 2 * U32) * a


def quant_interval_check(orc, gpu, lo, hi, mode, scale=None):
    """The GPU code is valid iff it is the rounding of some value in [lo, hi]
    (rounding is monotone, so it must lie between the roundings of the ends)."""
    if mode == "bf16":
        qlo, qhi = orc.quant_bf16(lo), orc.quant_bf16(hi)
    else:
        qlo, qhi = orc.quant_e4m3(lo / scale) * scale, orc.quant_e4m3(hi / scale) * scale
    return (gpu >= np.minimum(qlo, qhi) - 1e-30 * np.abs(qlo)) & (gpu <= np.maximum(qlo, qhi) + 1e-30 * np.abs(qhi))


def shared_terms(J, dtype):
    """Rounded FP32 additions behind one batch sum of the shared-draw form,
    each term bounded by |T c|: the FP32 product sums J products in some
    order; the BF16 product (BF16 and FP8 tables) sums three exact products
    per draw (c split into three BF16 parts whose magnitudes add up to at most
    (1 + 2^-7) |c|) within slices of at most ceil(J / splits) + 3 draws, then
    the slices."""
    if dtype == "f32":
        return J + 1
    splits = min(16, max(1, J // 2048))
    return int(np.ceil((3 * (-(-J // splits) + 3) + splits) * (1 + 2.0 ** -7)))


def mu_tolerance(cols, coef, J, K, tolT, tolc, chunk, terms=None):
    """Bound on |mu_gpu - mu_oracle| per row from the per-draw errors of the
    table entries (tolT, per draw and row) and coefficients (tolc, per draw), plus the
    FP32 accumulation over at most `chunk` FMAs and J/chunk partial sums, or,
    when `terms` is given, over `terms` additions in any order.
    The median is 1-Lipschitz in the max norm, so the batch bound carries over."""
    N = J * K
    ac = np.abs(coef)[:, None]
    aT = np.abs(cols)
    adds = (min(chunk, J) + J // max(1, chunk)) if terms is None else terms
    per = ac * tolT + aT * tolc[:, None] + (adds + 4) * U32 * ac * aT
    per = per.reshape(K, J, -1).sum(1) / J
    return per.max(0) + 4 * U32 * np.abs((cols * coef[:, None]).reshape(K, J, -1).sum(1) / J).max(0)


def check_selection(mu_orc, mu_tol, gpu_set, s_max, tau=0.0):
    """S_gpu must equal the oracle's top-s_max by |mu| (ties: smaller index),
    except for rows whose oracle |mu| lies within the tolerance of the s_max-th
    largest value (an FP32 near-tie).  Returns the number of admitted
    exceptions; fails on any other difference."""
    m = mu_orc.size
    a = np.abs(mu_orc)
    order = np.lexsort((np.arange(m), -a))
    orc_set = set(order[:s_max][a[order[:s_max]] >= tau].tolist())
    theta = a[order[min(s_max, m) - 1]]
    diff = orc_set.symmetric_difference(set(gpu_set))
    for i in diff:
        assert abs(a[i] - theta) <= mu_tol[i] + mu_tol.max() + 1e-12, \
            "row %d: |mu| %.9g vs cut %.9g (tol %.3g)" % (i, a[i], theta, mu_tol[i])
    return len(diff)


def orc_scales(A64, d):
    b = np.maximum(np.abs(A64).sum(1), np.sqrt(d) * np.abs(A64).max(1)) / 448.0
    s = b.astype(np.float32).astype(np.float64)
    s[s == 0] = 1.0
    return s


def entry_tolerance(orc, ref, A64, k, d, dtype):
    """Per-entry bound on |T_gpu - T_oracle| for the values each side uses.
    FP32: the FWHT rounding bound.  BF16/FP8: both sides round a value in
    [ref - e, ref + e]; they agree unless that interval straddles a rounding
    boundary, in which case they differ by at most one quantum."""
    tolT = np.broadcast_to(table_tol(A64, k)[None, :], ref.shape)
    if dtype == "f32":
        return tolT, ref
    if dtype == "bf16":
        lo, hi = orc.quant_bf16(ref - tolT), orc.quant_bf16(ref + tolT)
        used = orc.quant_bf16(ref)
    else:
        s = orc_scales(A64, d)[None, :]
        rel = 4 * A64.shape[1] * U32
        lo = orc.quant_e4m3((ref - tolT) / (s * (1 + rel))) * s
        hi = orc.quant_e4m3((ref + tolT) / (s * (1 - rel))) * s
        lo2 = orc.quant_e4m3((ref - tolT) / (s * (1 - rel))) * s
        hi2 = orc.quant_e4m3((ref + tolT) / (s * (1 + rel))) * s
        lo, hi = np.minimum(lo, lo2), np.maximum(hi, hi2)
        used = orc.quant_e4m3(ref / s) * s
    return np.abs(hi - lo) * 1.0001 + 1e-30, used


def check_outputs(orc, A64, X64, idx, val, cnt, r, info, eps, J, K, s_max, dtype, chunk=512):
    """Outputs alone (entry points without debug dumps) against the oracle's
    run on the same draws: every returned value is the exact a_i.x within
    1e-5 relative, rows are ascending and keep |v| >= eps, padding is (-1, 0),
    and the returned rows equal the oracle's output rows except rows at an
    FP32 near-tie of the selection (oracle |mu| within the mu tolerance of
    the s_max-th largest value) or with |a_i.x| within 1e-5 of eps.
    Returns the number of such exceptions."""
    k, d, n = info.k, info.d, A64.shape[1]
    m = A64.shape[0]
    exceptions = 0
    for t in range(X64.shape[0]):
        c = int(cnt[t])
        assert 0 <= c <= s_max
        gi, gv = idx[t][:c], val[t][:c].astype(np.float64)
        assert np.all(np.diff(gi) > 0), "rows not ascending"
        assert np.all(idx[t][c:] == -1) and np.all(val[t][c:] == 0)
        v64 = A64[gi] @ X64[t]
        scale = np.abs(A64[gi] * X64[t][None, :]).sum(1)
        assert np.all(np.abs(gv - v64) <= 1e-5 * np.abs(v64) + 4 * U32 * U32 * n * scale + 1e-30)
        assert np.all(np.abs(gv) >= eps)
        oc = r["out_cnt"][t]
        diff = np.setxor1d(r["out_idx"][t][:oc], gi)
        if len(diff) == 0:
            continue
        ct = coef_tol(X64[t], n)
        ent = orc.table_entries(A64, r["samples"][t], np.arange(m))
        tolE, used = entry_tolerance(orc, ent, A64, k, d, dtype)
        mt = mu_tolerance(used, r["coef"][t], J, K, tolE, np.full(J * K, ct), chunk)
        a = np.abs(r["mu"][t])
        order = np.lexsort((np.arange(m), -a))
        theta = a[order[min(s_max, m) - 1]]
        for i in diff:
            near_eps = abs(abs(A64[i] @ X64[t]) - eps) <= 1e-5 * eps
            near_cut = abs(a[i] - theta) <= mt[i] + mt.max() + 1e-12
            assert near_eps or near_cut, "vector %d row %d returned by one side only" % (t, i)
            exceptions += 1
    return exceptions
