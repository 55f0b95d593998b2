"""Seeded synthetic inputs for the Kerdock sparsifying transform.

This module holds no arithmetic of the method: it only draws matrices A and
unit vectors x with the shapes and value distributions of the workloads, so
that the GPU library and the FP64 oracle receive exactly the same inputs.
Everything is drawn in FP64 with ``numpy.random.default_rng(seed)`` and
rounded to FP32 at the end (the library's input type); the oracle then works
on the FP64 values of those FP32 numbers.

Workload recipes (A is n x n, x is unit, Ax is nearly s-sparse):
  tiny      n=64,   A Haar-orthogonal, x = A^T y/|A^T y|, y 4-sparse N(0,1)
            on a uniform support plus dense N(0,1e-6); eps = 0.1.
  plain     n=1024, A i.i.d. N(0,1/n), x = A^-1 y normalised, y 16-sparse
            N(0,1) plus N(0,1e-4); batch 256; eps = 0.05.
  precision n=2048, A = Haar-orthogonal * diag(exp U[ln 0.1, ln 10]),
            x = A^-1 y normalised, y 32-sparse + N(0,1e-4); batch 1024;
            eps = 0.05.
  batched   three A i.i.d. N(0,1/n), n in {256, 1024, 4096}, 512/1024/2560
            x (the 1:2:5 split of 4096), per-x sparsity s ~ U{4..64};
            eps = 0.05.
  learned   n=1024 structured dictionary A = Haar * diag(log-uniform),
            supports of y drawn from a fixed pool of 512 size-16 patterns.
  paper     n=4096 Haar-orthogonal A, Ax has s=20 equal-magnitude entries
            +-1/sqrt(20) at random positions (the paper's numerical section).
In N(0, v), v is the variance.
"""
import numpy as np

SEED_A = 1000
SEED_X = 2000
SEED_SAMPLES = 3000


def haar_orthogonal(n, rng):
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    columns' signs fixed by diag(R)."""
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    Q *= np.sign(np.diag(R))[None, :]
    return Q


def log_uniform_diag(n, rng, lo=0.1, hi=10.0):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


def sparse_plus_noise(n, s, rng, noise_var, support=None):
    """y with s N(0,1) entries on a uniform random support plus dense
    N(0, noise_var) noise."""
    y = rng.standard_normal(n) * np.sqrt(noise_var)
    if support is None:
        support = rng.choice(n, size=s, replace=False)
    y[support] += rng.standard_normal(len(support))
    return y, np.sort(np.asarray(support))


def _unit_rows(V):
    return V / np.linalg.norm(V, axis=1, keepdims=True)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


class Workload:
    """A (n x n, FP32), X (B x n, FP32 unit rows), eps, planted supports."""

    def __init__(self, name, A, X, eps, supports, s):
        self.name = name
        self.A = _f32(A)
        self.X = _f32(X)
        self.eps = float(eps)
        self.supports = supports
        self.s = s

    @property
    def n(self):
        return self.A.shape[1]

    @property
    def batch(self):
        return self.X.shape[0]


def _x_from_inverse(A64, Y):
    """x = A^{-1} y / |A^{-1} y| for each row y of Y."""
    Xt = np.linalg.solve(A64, Y.T)
    return _unit_rows(Xt.T)


def tiny(batch=1, seed_A=SEED_A + 1, seed_X=SEED_X + 1):
    n, s = 64, 4
    A = haar_orthogonal(n, np.random.default_rng(seed_A))
    rx = np.random.default_rng(seed_X)
    Y, sup = [], []
    for _ in range(batch):
        y, su = sparse_plus_noise(n, s, rx, 1e-6)
        Y.append(y)
        sup.append(su)
    X = _unit_rows(np.stack(Y) @ A)          # rows: (A^T y)^T
    return Workload("tiny", A, X, 0.1, sup, s)


def gaussian_matrix(n, rng):
    return rng.standard_normal((n, n)) / np.sqrt(n)


def plain(batch=256, n=1024, s=16, seed_A=SEED_A + 2, seed_X=SEED_X + 2):
    A = gaussian_matrix(n, np.random.default_rng(seed_A))
    rx = np.random.default_rng(seed_X)
    Y, sup = [], []
    for _ in range(batch):
        y, su = sparse_plus_noise(n, s, rx, 1e-4)
        Y.append(y)
        sup.append(su)
    X = _x_from_inverse(A, np.stack(Y))
    return Workload("plain", A, X, 0.05, sup, s)


def structured_dictionary(n, rng):
    return haar_orthogonal(n, rng) * log_uniform_diag(n, rng)[None, :]


def precision(batch=1024, n=2048, s=32, seed_A=SEED_A + 3, seed_X=SEED_X + 3):
    A = structured_dictionary(n, np.random.default_rng(seed_A))
    rx = np.random.default_rng(seed_X)
    Y, sup = [], []
    for _ in range(batch):
        y, su = sparse_plus_noise(n, s, rx, 1e-4)
        Y.append(y)
        sup.append(su)
    X = _x_from_inverse(A, np.stack(Y))
    return Workload("precision", A, X, 0.05, sup, s)


def batched(ns=(256, 1024, 4096), counts=(512, 1024, 2560), seed_A=SEED_A + 4,
            seed_X=SEED_X + 4):
    """Three independent Gaussian A with per-x sparsity s ~ U{4..64}."""
    out = []
    for q, (n, cnt) in enumerate(zip(ns, counts)):
        A = gaussian_matrix(n, np.random.default_rng(seed_A + 100 * q))
        rx = np.random.default_rng(seed_X + 100 * q)
        Y, sup, ss = [], [], []
        for _ in range(cnt):
            s = int(rx.integers(4, 65))
            y, su = sparse_plus_noise(n, s, rx, 1e-4)
            Y.append(y)
            sup.append(su)
            ss.append(s)
        X = _x_from_inverse(A, np.stack(Y))
        out.append(Workload("batched_n%d" % n, A, X, 0.05, sup, np.array(ss)))
    return out


def support_pool(n, pool=512, size=16, seed=SEED_X + 50):
    rng = np.random.default_rng(seed)
    return np.stack([np.sort(rng.choice(n, size=size, replace=False)) for _ in range(pool)])


def learned(count, n=1024, offset=0, seed_A=SEED_A + 5, seed_X=SEED_X + 5, pool=None):
    """x whose Ax is supported on one of a fixed pool of 512 size-16
    patterns.  ``offset`` selects disjoint streams (training vs held-out)."""
    A = structured_dictionary(n, np.random.default_rng(seed_A))
    if pool is None:
        pool = support_pool(n)
    rx = np.random.default_rng([seed_X, offset])
    pick = rx.integers(0, len(pool), size=count)
    Y = rx.standard_normal((count, n)) * np.sqrt(1e-4)
    vals = rx.standard_normal((count, pool.shape[1]))
    for r in range(count):
        Y[r, pool[pick[r]]] += vals[r]
    X = _x_from_inverse(A, Y)
    return Workload("learned", A, X, 0.05, [pool[p] for p in pick], 16)


def paper_regime(batch=16, n=4096, s=20, seed_A=SEED_A + 6, seed_X=SEED_X + 6):
    """Numerical section: A random orthogonal, Ax has exactly s nonzero
    entries of equal magnitude at random positions (x = A^T y)."""
    A = haar_orthogonal(n, np.random.default_rng(seed_A))
    rx = np.random.default_rng(seed_X)
    Y = np.zeros((batch, n))
    sup = []
    for r in range(batch):
        su = np.sort(rx.choice(n, size=s, replace=False))
        Y[r, su] = rx.choice([-1.0, 1.0], size=s) / np.sqrt(s)
        sup.append(su)
    X = Y @ A                                 # rows: (A^T y)^T, already unit
    return Workload("paper", A, X, 0.5 / np.sqrt(s), sup, s)


def near_sparse(batch=400, m=768, n=1000, s=8, delta=0.02, seed_A=SEED_A + 7, seed_X=SEED_X + 7):
    """x in Sigma(A, s, delta) for a wide A (m < n) with orthonormal rows (the
    first m rows of a Haar orthogonal n x n matrix, so |A|_{2->inf} = 1):
    y = Ax has every entry uniform in [-delta, delta] except s entries of
    equal magnitude and random sign on a random support, that magnitude
    chosen so that |y| = 1, and x = A^T y is then a unit vector.  eps is set
    at 0.85 of the smallest magnitude that planting can give."""
    A = haar_orthogonal(n, np.random.default_rng(seed_A))[:m]
    rx = np.random.default_rng(seed_X)
    Y = rx.uniform(-delta, delta, size=(batch, m))
    sup = []
    for r in range(batch):
        su = np.sort(rx.choice(m, size=s, replace=False))
        Y[r, su] = 0.0
        mag = np.sqrt((1.0 - np.dot(Y[r], Y[r])) / s)
        Y[r, su] = rx.choice([-1.0, 1.0], size=s) * mag
        sup.append(su)
    X = Y @ A
    mag_min = np.sqrt((1.0 - m * delta * delta) / s)
    w = Workload("near_sparse", A, X, 0.85 * mag_min, sup, s)
    w.delta = float(delta)
    return w


def toy_model(batch, p, n=4096, seed_A=SEED_A + 6, seed_X=SEED_X + 8):
    """Section 2.1's model: A orthogonal (Haar, the paper-regime matrix for
    n = 4096), every entry of y = Ax independently N(0, 1) with probability p
    and 0 otherwise; x = A^T y / |y| so that A x is the unit vector y / |y|.
    eps is not set (the sweep scales it as alpha / sqrt(p n)); supports are
    the nonzero rows of y."""
    A = haar_orthogonal(n, np.random.default_rng(seed_A))
    rx = np.random.default_rng(seed_X + int(round(p * 1e6)))
    Y = np.where(rx.random((batch, n)) < p, rx.standard_normal((batch, n)), 0.0)
    empty = np.linalg.norm(Y, axis=1) == 0
    Y[empty, 0] = 1.0                        # keep every row a unit vector
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    X = Y @ A
    sup = [np.flatnonzero(y) for y in Y]
    return Workload("toy p=%g" % p, A, X, 0.0, sup, int(round(p * n)))
