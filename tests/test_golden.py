"""Values the paper prints for its numerical experiment (Section 'Numerical
results', Figure 1 and the text after it), kept in tests/golden/
numerical_section.json, against the oracle, Theorem 5's parameter formula
and the seeded generator of that workload."""
import json
import math
import os

import numpy as np

from paper_2105_05879_amd import workloads
from test_oracle_theorem import theorem5

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "numerical_section.json")))


def test_design_size_at_n_4096(orc):
    """The paper prints d = n and L = n(n/2+1) = 8392704 for n = 4096."""
    k = orc.choose_k(GOLDEN["n"])
    assert 1 << k == GOLDEN["d"]
    assert orc.design_size(k) == GOLDEN["L"]


def test_theorem5_K_at_eta_one():
    """With eta = 1, Theorem 5's lower bound on K exceeds 16 at m = 4096
    (the paper's remark that its guarantee is off the scale of Figure 1)."""
    _, K = theorem5(np.ones((GOLDEN["n"], 1)), 1.0, 0.0, 1.0)     # K depends on m = n and eta only
    assert K == 17 and K > GOLDEN["theorem5_K_lower_bound_at_eta_1_exceeds"]


def test_workload_is_the_numerical_experiment():
    """A orthogonal, x unit, Ax exactly s nonzero entries of one magnitude."""
    w = workloads.paper_regime(batch=8, n=GOLDEN["n"], s=GOLDEN["s"])
    A = w.A.astype(np.float64)
    assert A.shape == (GOLDEN["n"], GOLDEN["n"])
    cols = A[:, :64]
    assert np.abs(cols.T @ cols - np.eye(64)).max() < 1e-5
    X = w.X.astype(np.float64)
    assert np.allclose(np.linalg.norm(X, axis=1), 1.0, atol=1e-5)
    Y = X @ A.T
    for t in range(w.batch):
        big = np.nonzero(np.abs(Y[t]) > 1e-3)[0]
        assert np.array_equal(big, w.supports[t]) and big.size == GOLDEN["s"]
        assert np.allclose(np.abs(Y[t][big]), 1 / math.sqrt(GOLDEN["s"]), atol=1e-5)
