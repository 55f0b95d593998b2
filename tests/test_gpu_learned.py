"""Learned-proposal form on the GPU against the FP64 oracle.

Network kernels (features, forward, backward, Adam) against oracle/mlp.py
with the same bfloat16 rounding points; the learned apply against the exact
definition (verified values, the fallback guarantee) and against the plain
path (fallback rows equal kerdock_sparse_apply bit for bit); and a small
training run that shows what the network gains over the plain method."""
import ctypes
import math

import numpy as np
import pytest
import torch

from gpu_common import need_gpu
from oracle import mlp as omlp
from paper_2105_05879_amd import workloads

pytestmark = pytest.mark.gpu


def rand_params(dims, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for shp in omlp.shapes(*dims):
        fan = shp[1] if len(shp) == 2 else 1
        a = scale * math.sqrt(6.0 / max(fan, 1)) if len(shp) == 2 else 0.1
        out.append(rng.uniform(-a, a, size=int(np.prod(shp))))
    return np.concatenate(out).astype(np.float32)


def test_features_match_oracle(orc):
    kd = need_gpu()
    for n in (16, 100, 1024, 3000):
        rng = np.random.default_rng(n)
        X = rng.standard_normal((5, n)).astype(np.float32)
        h = kd.kerdock_prepare(torch.from_numpy(rng.standard_normal((8, n)).astype(np.float32)).cuda())
        d = h.info.d
        F = kd.kerdock_features(h, torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
        # f[w] = s_w . x / sqrt(d) with s_w the w-th vector of the first (Hadamard) basis
        ref = orc.table_entries(X.astype(np.float64), np.arange(d), np.arange(5)).T / math.sqrt(d)
        tol = (math.log2(d) + 2) * 2.0 ** -24 * np.abs(X).sum(1, keepdims=True) / math.sqrt(d)
        assert np.all(np.abs(F - ref) <= tol)
        h.destroy()


DIMS = (256, 192, 128, 320)


def test_forward_matches_oracle():
    kd = need_gpu()
    net = kd.kerdock_mlp_create(*DIMS, seed=1)
    P = rand_params(DIMS, 2)
    kd.kerdock_mlp_set_params(net, P)
    assert np.array_equal(kd.kerdock_mlp_get_params(net), P)
    rng = np.random.default_rng(3)
    F = rng.standard_normal((100, DIMS[0])).astype(np.float32)       # ragged batch (not a tile multiple)
    Z = kd.kerdock_mlp_forward(net, torch.from_numpy(F).cuda()).cpu().numpy().astype(np.float64)
    Zo, _ = omlp.forward(P.astype(np.float64), F.astype(np.float64), DIMS, emulate=True)
    rel = np.linalg.norm(Z - Zo) / np.linalg.norm(Zo)
    assert rel < 2e-3, rel
    assert np.abs(Z - Zo).max() < 2e-2 * np.abs(Zo).max()
    net.destroy()


def gpu_grads(kd, net, F, Y, pos_w):
    loss, g = kd.kerdock_mlp_train_step(net, torch.from_numpy(F).cuda(), torch.from_numpy(Y).cuda(), 0.0, pos_w,
                                        want_grads=True)
    torch.cuda.synchronize()
    return loss.item(), g.cpu().numpy().astype(np.float64)


def test_gradients_match_oracle():
    kd = need_gpu()
    net = kd.kerdock_mlp_create(*DIMS, seed=4)
    P = rand_params(DIMS, 5)
    kd.kerdock_mlp_set_params(net, P)
    rng = np.random.default_rng(6)
    F = rng.standard_normal((130, DIMS[0])).astype(np.float32)
    Y = (rng.random((130, DIMS[3])) < 0.05).astype(np.uint8)
    loss, G = gpu_grads(kd, net, F, Y, 8.0)
    lo, Go = omlp.loss_and_grad(P.astype(np.float64), F.astype(np.float64), Y, DIMS, 8.0, emulate=True)
    assert abs(loss - lo) <= 1e-4 * abs(lo)
    off = 0
    for shp in omlp.shapes(*DIMS):
        size = int(np.prod(shp))
        g, go = G[off:off + size], Go[off:off + size]
        rel = np.linalg.norm(g - go) / np.linalg.norm(go)
        assert rel < 1e-2, (shp, rel)
        off += size
    net.destroy()


def test_adam_step_matches_oracle():
    kd = need_gpu()
    net = kd.kerdock_mlp_create(*DIMS, seed=7)
    P = rand_params(DIMS, 8)
    kd.kerdock_mlp_set_params(net, P)
    rng = np.random.default_rng(9)
    F = rng.standard_normal((64, DIMS[0])).astype(np.float32)
    Y = (rng.random((64, DIMS[3])) < 0.05).astype(np.uint8)
    lr = 1e-3
    kd.kerdock_mlp_train_step(net, torch.from_numpy(F).cuda(), torch.from_numpy(Y).cuda(), lr, 8.0)
    P1 = kd.kerdock_mlp_get_params(net).astype(np.float64)
    _, Go = omlp.loss_and_grad(P.astype(np.float64), F.astype(np.float64), Y, DIMS, 8.0, emulate=True)
    Po, _, _ = omlp.adam_step(P.astype(np.float64), Go, np.zeros_like(Go), np.zeros_like(Go), 1, lr)
    # step 1 of Adam moves every parameter by about lr sign(g): the two sides
    # agree except where the gradient is so small that its sign may differ
    diff = np.abs(P1 - Po)
    small = np.abs(Go) < 2e-2 * np.abs(Go).max()
    assert np.all(diff[~small] <= 1e-3 * lr + 1e-7)
    assert np.all(diff <= 2.0001 * lr)
    net.destroy()


def test_training_lowers_the_loss():
    kd = need_gpu()
    dims = (128, 128, 128, 64)
    net = kd.kerdock_mlp_create(*dims, seed=10)
    rng = np.random.default_rng(11)
    # a learnable rule: label j is on when feature j is large
    F = rng.standard_normal((2048, dims[0])).astype(np.float32)
    Y = (F[:, :dims[3]] > 1.0).astype(np.uint8)
    Ft, Yt = torch.from_numpy(F).cuda(), torch.from_numpy(Y).cuda()
    losses = []
    for step in range(300):
        idx = torch.from_numpy(rng.integers(0, 2048, 256)).cuda()
        loss, _ = kd.kerdock_mlp_train_step(net, Ft[idx].contiguous(), Yt[idx].contiguous(), 3e-3, 3.0)
        losses.append(loss.item())
    assert np.mean(losses[-20:]) < 0.3 * np.mean(losses[:20])
    net.destroy()


def make_handle(kd, w, dtype="bf16"):
    return kd.kerdock_prepare(torch.from_numpy(w.A).cuda(), dtype)


def test_candidates_are_top_logits(orc):
    """The candidate set C of the learned apply is the s_max rows of largest
    logit, ties to the smaller index: compared with a numpy lexsort of the
    network's logits (kerdock_mlp_forward on kerdock_features, the same
    BF16 inputs), with negative logits and exact ties (output rows sharing
    their weights and bias)."""
    kd = need_gpu()
    w = workloads.learned(48, n=256)
    h = make_handle(kd, w)
    m, d = h.m, h.info.d
    dims = (d, 64, 64, m)
    net = kd.kerdock_mlp_create(*dims, seed=5)
    P = rand_params(dims, 6)
    o3 = dims[1] * dims[0] + dims[1] + dims[2] * dims[1] + dims[2]     # W3 [m][d2], then b3 [m]
    W3 = P[o3:o3 + m * dims[2]].reshape(m, dims[2])
    b3 = P[o3 + m * dims[2]:]
    for twin in (3, 40, 41, 200):
        W3[twin] = W3[2]
        b3[twin] = b3[2]
    kd.kerdock_mlp_set_params(net, P)
    kd.kerdock_learned_attach(h, net)
    X = torch.from_numpy(w.X).cuda()
    Z = kd.kerdock_mlp_forward(net, kd.kerdock_features(h, X)).cpu().numpy()
    assert (Z < 0).any() and (Z > 0).any()
    assert np.all(Z[:, 3] == Z[:, 2]) and np.all(Z[:, 200] == Z[:, 2])
    for s_max in (1, 37, 128, m):
        out = kd.kerdock_learned_apply(h, X, 0.05, s_max, 64, 1, 7, candidates=True)
        cand = out[4].cpu().numpy()
        for t in range(X.shape[0]):
            order = np.lexsort((np.arange(m), -Z[t].astype(np.float64)))
            assert np.array_equal(cand[t], np.sort(order[:s_max])), (s_max, t)
    h.destroy()
    net.destroy()


def test_energy_check_without_proposal_gap(orc):
    """With C = every row the verified energy is the exact energy: no row may
    fall back (the energy path itself is consistent)."""
    kd = need_gpu()
    w = workloads.learned(128, n=1024)
    h = make_handle(kd, w)
    net = kd.kerdock_mlp_create(h.info.d, 64, 64, h.m, seed=3)
    kd.kerdock_learned_attach(h, net)
    idx, val, cnt, fb = kd.kerdock_learned_apply(h, torch.from_numpy(w.X).cuda(), 0.05, h.m, 512, 1, 5)
    torch.cuda.synchronize()
    assert fb.sum().item() == 0
    Y = w.X.astype(np.float64) @ w.A.astype(np.float64).T
    idx, val, cnt = idx.cpu().numpy(), val.cpu().numpy(), cnt.cpu().numpy()
    for t in range(len(cnt)):
        want = np.nonzero(np.abs(Y[t]) >= 0.05)[0]
        assert np.array_equal(idx[t][:cnt[t]], want) or abs(np.abs(Y[t]) - 0.05).min() < 1e-6
    h.destroy()
    net.destroy()


def test_learned_apply_exact_and_fallback(orc):
    """Untrained network: whatever it proposes, every returned value is the
    exact a_i.x, no row of h_eps(Ax) is missing from a row that did not fall
    back, and fallback rows equal the plain path bit for bit."""
    kd = need_gpu()
    w = workloads.learned(96, n=256)
    X = torch.from_numpy(w.X).cuda()
    h = make_handle(kd, w)
    net = kd.kerdock_mlp_create(h.info.d, 64, 64, h.m, seed=12)
    kd.kerdock_learned_attach(h, net)
    eps, s_max, J, K, seed = 0.05, 60, 2000, 2, 13
    idx, val, cnt, fb = kd.kerdock_learned_apply(h, X, eps, s_max, J, K, seed)
    plain = kd.kerdock_sparse_apply(h, X, eps, s_max, J, K, seed)
    torch.cuda.synchronize()
    idx, val, cnt, fb = idx.cpu().numpy(), val.cpu().numpy(), cnt.cpu().numpy(), fb.cpu().numpy()
    pi, pv, pc = (t.cpu().numpy() for t in plain)
    A64, X64 = w.A.astype(np.float64), w.X.astype(np.float64)
    Y = X64 @ A64.T
    assert 0 < fb.sum() <= len(fb)
    for t in range(len(fb)):
        c = cnt[t]
        if fb[t]:
            assert c == pc[t] and np.array_equal(idx[t], pi[t]) and np.array_equal(val[t], pv[t])
        else:
            assert np.all(np.abs(val[t][:c] - Y[t][idx[t][:c]]) <= 1e-5 * np.abs(Y[t][idx[t][:c]]) + 1e-9)
            assert set(np.nonzero(np.abs(Y[t]) >= eps * (1 + 1e-6))[0]) <= set(idx[t][:c])
            assert np.all(np.abs(val[t][:c]) >= eps)
    h.destroy()
    net.destroy()


def test_energy_check_is_sound_with_dense_gram(orc):
    """The fallback guarantee in floating point, on a dense, ill-conditioned
    Gram matrix: A = diag(d) Q with Q Haar-orthogonal and d log-uniform in
    [0.1, 10] (|A|_2 = 10), and a proposer whose candidate set C is fixed and
    never holds row R (logits = biases, R's far below).  Groups of x:
      1. unit x with |(Ax)_R| = 1.5 eps, support of the rest in C -> must
         fall back;
      2. as 1, the rest on the rows of largest d (|Ax|^2 up to ~100);
      3. unit x with Ax supported in C                       -> certified,
         accepted;
      4. 300 times a group-3 vector (not unit: the rounding bound on
         |Ax|^2 exceeds eps^2 / 2)                            -> falls back.
    Accepted rows are exact, and the computed |Ax|^2 and verified energy
    lie within the reported bound of their FP64 values."""
    kd = need_gpu()
    n, s_max, eps, R = 512, 40, 0.05, 5
    rng = np.random.default_rng(77)
    d = np.exp(rng.uniform(np.log(0.1), np.log(10.0), n))
    d[0] = 10.0
    A = (d[:, None] * workloads.haar_orthogonal(n, rng)).astype(np.float32)
    A64 = A.astype(np.float64)
    G64 = A64.T @ A64
    assert np.count_nonzero(np.abs(G64 - np.diag(np.diag(G64))) > 1e-3) > n * n // 2     # dense Gram
    bias = -np.arange(n, dtype=np.float64)
    bias[R] = -1e4
    C = set(np.argsort(-bias, kind="stable")[:s_max].tolist())
    assert R not in C
    inside = np.array(sorted(C))
    big = inside[np.argsort(-d[inside], kind="stable")[:6]]
    xr = np.linalg.solve(A64, np.eye(n)[R])

    def unit_x(y_rest, r_val):
        # x = A^-1 (y_rest + c e_R) / norm with (Ax)_R = r_val: c = r_val |x0 + c xr| (a contraction)
        x0 = np.linalg.solve(A64, y_rest)
        c = 0.0
        for _ in range(60):
            c = r_val * np.linalg.norm(x0 + c * xr)
        x = x0 + c * xr
        return x / np.linalg.norm(x)

    X = []
    for g in range(4):
        for _ in range(12):
            y = np.zeros(n)
            sup = big if g == 1 else rng.choice(inside, size=6, replace=False)
            y[sup] = rng.standard_normal(6)
            x = unit_x(y, 1.5 * eps * rng.choice([-1.0, 1.0]) if g < 2 else 0.0)
            X.append(300.0 * x if g == 3 else x)
    X = np.stack(X).astype(np.float32)
    X64 = X.astype(np.float64)
    Ax = X64 @ A64.T
    assert np.all(np.abs(Ax[:24, R]) >= eps)
    h = kd.kerdock_prepare(torch.from_numpy(A).cuda(), "bf16")
    dims = (h.info.d, 32, 32, n)
    net = kd.kerdock_mlp_create(*dims, seed=1)
    P = rand_params(dims, 2)
    o3 = dims[1] * dims[0] + dims[1] + dims[2] * dims[1] + dims[2]
    P[o3:o3 + n * dims[2]] = 0.0                  # W3 = 0: logits = b3
    P[o3 + n * dims[2]:] = bias.astype(np.float32)
    kd.kerdock_mlp_set_params(net, P)
    kd.kerdock_learned_attach(h, net)
    Xt = torch.from_numpy(X).cuda()
    B = X.shape[0]
    out = tuple(torch.empty(sh, dtype=dt, device="cuda") for sh, dt in
                (((B, s_max), torch.int32), ((B, s_max), torch.float32), ((B,), torch.int32)))
    fb = torch.empty((B,), dtype=torch.int32, device="cuda")
    cand = torch.empty((B, s_max), dtype=torch.int32, device="cuda")
    energy = torch.zeros((B, n), dtype=torch.float32, device="cuda")
    p = kd.ApplyParams(J=2000, K=1, seed=3, t0=0, tau=0.0, chunk=0)
    p.dbg_survivors = cand.data_ptr()
    p.dbg_mu = energy.data_ptr()
    kd._check(kd.lib().kerdock_learned_apply(h.ptr, kd._dev(Xt, torch.float32, "X"), B, eps, s_max,
                                             ctypes.byref(p), kd._ptr(out[0]), kd._ptr(out[1]), kd._ptr(out[2]),
                                             kd._ptr(fb), kd._stream(None)))
    torch.cuda.synchronize()
    cand, fb = cand.cpu().numpy(), fb.cpu().numpy()
    idx, val, cnt = (o.cpu().numpy() for o in out)
    en = energy.cpu().numpy()[:, :3].astype(np.float64)
    for t in range(B):
        assert set(cand[t].tolist()) == C
        E64 = float(Ax[t] @ Ax[t])
        S64 = float(sum(Ax[t][i] ** 2 for i in C))
        E, S, bound = en[t]
        assert abs(E - E64) <= bound and abs(S - S64) <= bound, (t, E, E64, S, S64, bound)
        missing = any(abs(Ax[t][i]) >= eps for i in range(n) if i not in C)
        g = t // 12
        if missing:
            assert fb[t] == 1, t
        if g in (0, 1):
            assert missing and fb[t] == 1
        elif g == 2:
            assert fb[t] == 0 and bound < eps * eps / 2, (t, bound)
        else:
            assert fb[t] == 1 and bound >= eps * eps / 2, (t, bound)
        if fb[t] == 0:
            c = cnt[t]
            want = [i for i in sorted(C) if abs(Ax[t][i]) >= eps]
            assert idx[t][:c].tolist() == want
            assert np.all(np.abs(val[t][:c] - Ax[t][idx[t][:c]]) <= 1e-5 * np.abs(Ax[t][idx[t][:c]]))
    h.destroy()
    net.destroy()


def test_learned_gain_over_plain(orc):
    """Train the proposer on pairs the plain method produces; on held-out
    vectors the learned apply keeps the recall of the plain method, falls
    back rarely, and is faster."""
    kd = need_gpu()
    n, eps = 1024, 0.05
    pool = workloads.support_pool(n)
    ntrain = 65536
    wtr = workloads.learned(ntrain, n=n, offset=0, pool=pool)
    wte = workloads.learned(1024, n=n, offset=1, pool=pool)
    h = make_handle(kd, wtr, "bf16")
    s_max, J, K, seed = 160, 40960, 1, 21
    Xtr = torch.from_numpy(wtr.X).cuda()
    # labels: the support of the plain method's output
    Y = torch.zeros((ntrain, n), dtype=torch.uint8, device="cuda")
    for b in range(0, ntrain, 4096):
        idx, val, cnt = kd.kerdock_sparse_apply(h, Xtr[b:b + 4096].contiguous(), eps, s_max, J, K, seed, t0=b)
        rows = torch.arange(s_max, device="cuda")[None, :] < cnt[:, None]
        nz = torch.nonzero(rows)
        Y[b + nz[:, 0], idx[rows].long()] = 1
    F = kd.kerdock_features(h, Xtr)
    net = kd.kerdock_mlp_create(h.info.d, 512, 512, n, seed=22)
    pos_w = float(n / max(1.0, Y.float().sum(1).mean().item()))
    g = torch.Generator(device="cpu").manual_seed(23)
    for epoch in range(10):
        perm = torch.randperm(ntrain, generator=g).cuda()
        for b in range(0, ntrain, 256):
            sel = perm[b:b + 256]
            kd.kerdock_mlp_train_step(net, F[sel].contiguous(), Y[sel].contiguous(), 1e-3, pos_w)
    kd.kerdock_learned_attach(h, net)
    Xte = torch.from_numpy(wte.X).cuda()
    Yte = wte.X.astype(np.float64) @ wte.A.astype(np.float64).T
    sup = [np.nonzero(np.abs(Yte[t]) >= eps)[0] for t in range(len(Yte))]

    def recall(i, c):
        r = [len(set(i[t][:c[t]]) & set(s)) / len(s) for t, s in enumerate(sup) if len(s)]
        return float(np.mean(r))

    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    li, lv, lc, fb = kd.kerdock_learned_apply(h, Xte, eps, s_max, J, K, seed, t0=1 << 30)
    t1.record()
    torch.cuda.synchronize()
    t_learned = t0.elapsed_time(t1)
    t0.record()
    pi, pv, pc = kd.kerdock_sparse_apply(h, Xte, eps, s_max, J, K, seed, t0=1 << 30)
    t1.record()
    torch.cuda.synchronize()
    t_plain = t0.elapsed_time(t1)
    r_l = recall(li.cpu().numpy(), lc.cpu().numpy())
    r_p = recall(pi.cpu().numpy(), pc.cpu().numpy())
    fb_rate = fb.float().mean().item()
    print("learned: recall %.4f fallback %.3f %.2f ms | plain: recall %.4f %.2f ms" % (r_l, fb_rate, t_learned, r_p, t_plain))
    assert r_l >= r_p - 1e-3
    assert fb_rate < 0.5
    assert t_learned < t_plain
    h.destroy()
    net.destroy()
