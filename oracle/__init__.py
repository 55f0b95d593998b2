"""FP64 CPU oracle for the Kerdock fast sparsifying transform (arXiv 2105.05879).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product library.  It shares
no code with the GPU path.

The arithmetic lives in ``kerdock_oracle.c`` (plain C, FP64); this module only
compiles it with gcc and marshals numpy arrays through ctypes.  The MLP oracle
for the learned-proposal form is in ``mlp.py`` (numpy, FP64).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kerdock_oracle.c")
_LIB = os.path.join(_HERE, "libkerdock_oracle.so")
_lib = None


def build(force=False):
    """Compile the C oracle with gcc (OpenMP over the batch of x)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    c_i, c_i64, c_u64, c_d, c_p = (ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_double, ctypes.c_void_p)
    sigs = {
        "ko_choose_k": (c_i, [c_i]),
        "ko_design_size": (c_i64, [c_i]),
        "ko_field_poly": (c_u64, [c_i]),
        "ko_gf_mul": (c_u64, [c_u64, c_u64, c_u64]),
        "ko_gf_trace": (c_i, [c_u64, c_u64]),
        "ko_kerdock_matrix": (None, [c_i, c_u64, c_p]),
        "ko_quadratic_form": (c_i, [c_i, c_p, c_u64]),
        "ko_design_vector": (None, [c_i, c_i, c_i64, c_p]),
        "ko_table_column": (None, [c_p, c_i, c_i, c_i, c_i64, c_p]),
        "ko_table": (None, [c_p, c_i, c_i, c_p]),
        "ko_philox4x64_10": (None, [c_p, c_p, c_p]),
        "ko_draw_samples": (None, [c_u64, c_i64, c_i64, c_i64, c_p]),
        "ko_draw_samples_stream": (None, [c_u64, c_i64, c_u64, c_i64, c_i64, c_p]),
        "ko_quant_bf16": (c_d, [c_d]),
        "ko_quant_e4m3": (c_d, [c_d]),
        "ko_quant_array": (None, [c_p, c_i64, c_i]),
        "ko_sign_words": (None, [c_i, c_u64, c_p]),
        "ko_table_entries": (None, [c_p, c_i, c_i, c_p, c_i64, c_p, c_i, c_p]),
        "ko_mu_rows": (None, [c_p, c_i, c_i, c_p, c_p, c_i, c_i, c_p, c_i, c_i, c_p]),
        "ko_sparse_apply": (c_i, [c_p, c_i, c_i, c_p, c_i, c_i64, c_u64, c_i, c_i, c_d, c_i,
                                  c_d, c_i, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_i]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def choose_k(n):
    """Smallest even k with 2^k >= n (Lemma 8)."""
    return _load().ko_choose_k(int(n))


def design_size(k):
    """L = d (d/2 + 1) with d = 2^k (Algorithm 1)."""
    return _load().ko_design_size(int(k))


def field_poly(D):
    """Smallest irreducible polynomial of degree D over F_2 (integer encoding)."""
    return int(_load().ko_field_poly(int(D)))


def gf_mul(a, b, p):
    return int(_load().ko_gf_mul(int(a), int(b), int(p)))


def gf_trace(z, p):
    return int(_load().ko_gf_trace(int(z), int(p)))


def kerdock_matrix(k, s):
    """The k x k matrix M_s of Proposition 7 over F_2 (uint8 0/1)."""
    M = np.zeros((k, k), dtype=np.uint8)
    _load().ko_kerdock_matrix(int(k), int(s), _ptr(M))
    return M


def quadratic_form(M, x):
    M = np.ascontiguousarray(M, dtype=np.uint8)
    return int(_load().ko_quadratic_form(M.shape[0], _ptr(M), int(x)))


def design_vector(n, k, ell):
    """s_ell = sqrt(d) Pi u_ell in R^n (Algorithm 1)."""
    s = np.zeros(n, dtype=np.float64)
    _load().ko_design_vector(int(n), int(k), int(ell), _ptr(s))
    return s


def table_column(A, ell):
    """A s_ell for a row-major A (m x n)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    col = np.zeros(m, dtype=np.float64)
    _load().ko_table_column(_ptr(A), m, n, choose_k(n), int(ell), _ptr(col))
    return col


def table(A):
    """The whole sketch {A s_ell}, shape (L, m).  Small n only."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    L = design_size(choose_k(n))
    T = np.zeros((L, m), dtype=np.float64)
    _load().ko_table(_ptr(A), m, n, _ptr(T))
    return T


def philox4x64_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64).copy()
    kk = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    _load().ko_philox4x64_10(_ptr(c), _ptr(kk), _ptr(out))
    return out


def draw_samples(seed, t, N, L, stream=None):
    """Draws of stream position t; stream=None is the per-vector stream
    (counter word 1 = 0), an integer w selects counter word 1 = w."""
    out = np.zeros(int(N), dtype=np.int64)
    if stream is None:
        _load().ko_draw_samples(int(seed), int(t), int(N), int(L), _ptr(out))
    else:
        _load().ko_draw_samples_stream(int(seed), int(t), int(stream), int(N), int(L), _ptr(out))
    return out


def _quant(x, mode):
    a = np.array(x, dtype=np.float64, copy=True, order="C")
    _load().ko_quant_array(_ptr(a), a.size, mode)
    return a if a.ndim else float(a)


def quant_bf16(x):
    """Round to bfloat16 (nearest, ties to even), elementwise."""
    return _quant(x, 1)


def quant_e4m3(x):
    """Round to OCP FP8 E4M3 (nearest, ties to even, saturating at 448), elementwise."""
    return _quant(x, 2)


def sign_words(k, s):
    """(-1)^{Q_{M_s}(x)} for x < d as bit x mod 32 of word x // 32."""
    out = np.zeros(max(1, (1 << k) // 32), dtype=np.uint32)
    _load().ko_sign_words(int(k), int(s), _ptr(out))
    return out


def table_entries(A, samples, rows):
    """T[l_j]_r for the given draws (N) and rows (R): array (N, R)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    ls = np.ascontiguousarray(samples, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((ls.size, rows.size), dtype=np.float64)
    _load().ko_table_entries(_ptr(A), m, n, _ptr(ls), ls.size, _ptr(rows), rows.size, _ptr(out))
    return out


def mu_rows(A, x, samples, J, K, rows, table_mode="exact"):
    """Median-of-means estimate on the given rows from given draws."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m, n = A.shape
    x = np.ascontiguousarray(x, dtype=np.float64)
    ls = np.ascontiguousarray(samples, dtype=np.int64)
    assert ls.size == J * K and K <= 64
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros(rows.size, dtype=np.float64)
    _load().ko_mu_rows(_ptr(A), m, n, _ptr(x), _ptr(ls), int(J), int(K), _ptr(rows), rows.size,
                       TABLE_MODES[table_mode], _ptr(out))
    return out


TABLE_MODES = {"f32": 0, "exact": 0, "bf16": 1, "fp8": 2, "fp8e4m3": 2}


def sparse_apply(A, X, J, K, eps, s_max, seed, t0=0, tau=0.0, table_mode="exact", debug=False, tile=0):
    """Algorithm 1's streaming step for every row of X, in FP64.

    Returns a dict with out_idx (B, s_max), out_val, out_cnt and, with
    debug=True, samples (B, N), coef (B, N), ybar (B, K, m), mu (B, m) and
    surv (B, s_max)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    X = np.ascontiguousarray(np.atleast_2d(X), dtype=np.float64)
    m, n = A.shape
    B = X.shape[0]
    assert X.shape[1] == n
    N = int(J) * int(K)
    r = {
        "out_idx": np.full((B, s_max), -1, dtype=np.int32),
        "out_val": np.zeros((B, s_max), dtype=np.float64),
        "out_cnt": np.zeros(B, dtype=np.int32),
    }
    if debug:
        r.update(samples=np.zeros((B, N), dtype=np.int64), coef=np.zeros((B, N)),
                 ybar=np.zeros((B, K, m)), mu=np.zeros((B, m)),
                 surv=np.zeros((B, s_max), dtype=np.int32))
    rc = _load().ko_sparse_apply(
        _ptr(A), m, n, _ptr(X), B, int(t0), int(seed), int(J), int(K), float(eps), int(s_max),
        float(tau), TABLE_MODES[table_mode], _ptr(r["out_idx"]), _ptr(r["out_val"]),
        _ptr(r["out_cnt"]), _ptr(r.get("samples")), _ptr(r.get("coef")), _ptr(r.get("ybar")),
        _ptr(r.get("mu")), _ptr(r.get("surv")), int(tile))
    if rc != 0:
        raise ValueError("oracle sparse_apply rejected its arguments")
    return r
