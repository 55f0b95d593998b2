"""Theorem 5 on the oracle: with J >= 4 e^2 |A|_{2->inf}^2 / gamma^2 and
K >= 2 log(m / eta), gamma = (eps - delta) / 2, the streaming step keeps
every row of |Ax| >= eps and drops every row of |Ax| <= delta (threshold
tau = (eps + delta) / 2, S = the s largest estimates) for at least a
1 - eta fraction of x in Sigma(A, s, delta)."""
import math

import numpy as np

from paper_2105_05879_amd import workloads


def theorem5(A, eps, delta, eta):
    gamma = 0.5 * (eps - delta)
    norm2 = float(np.max(np.sum(np.asarray(A, dtype=np.float64) ** 2, axis=1)))
    return (math.ceil(4 * math.e ** 2 * norm2 / gamma ** 2),
            math.ceil(2 * math.log(A.shape[0] / eta)))


def test_theorem5_failure_rate_on_wide_near_sparse(orc):
    w = workloads.near_sparse(batch=300, m=12, n=16, s=2, delta=0.05)
    eta = 0.1
    J, K = theorem5(w.A, w.eps, w.delta, eta)
    tau = 0.5 * (w.eps + w.delta)
    r = orc.sparse_apply(w.A, w.X, J, K, w.eps, w.s, seed=77, tau=tau, debug=True)
    Y = w.X.astype(np.float64) @ w.A.astype(np.float64).T
    fails = 0
    gamma = 0.5 * (w.eps - w.delta)
    dev = np.abs(r["mu"] - Y).max(axis=1)
    for t in range(w.batch):
        got = r["out_idx"][t][:r["out_cnt"][t]]
        ok = np.array_equal(got, w.supports[t]) and np.allclose(
            r["out_val"][t][:r["out_cnt"][t]], Y[t][w.supports[t]], rtol=1e-12, atol=1e-12)
        fails += not ok
        # a failure is only possible where the estimate strays by gamma
        assert ok or dev[t] >= gamma
    assert fails <= eta * w.batch
    # the event the theorem bounds is itself rarer than eta
    assert np.mean(dev >= gamma) <= eta
