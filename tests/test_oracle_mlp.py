"""Pins of the FP64 MLP oracle: finite differences, and library routines
(torch's bfloat16 cast, BCE-with-logits with pos_weight, Adam) in float64."""
import numpy as np
import torch

from oracle import mlp

DIMS = (12, 9, 7, 10)


def params(seed, dims=DIMS):
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.standard_normal(int(np.prod(s))) * 0.5 for s in mlp.shapes(*dims)])


def data(seed, B=6, dims=DIMS):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((B, dims[0]))
    Y = (rng.random((B, dims[3])) < 0.3).astype(np.float64)
    return F, Y


def test_quant_bf16_matches_torch():
    rng = np.random.default_rng(0)
    v = (rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    v = np.concatenate([v, np.float32([0, 1, -1, 1.00390625, 1.01171875, 3.4e38, 1e-39, 2.0 ** -126])])
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.quant_bf16(v.astype(np.float64)), want)


def test_quant_bf16_matches_scalar_oracle(orc):
    rng = np.random.default_rng(1)
    v = rng.standard_normal(500) * np.exp(rng.uniform(-5, 5, 500))
    assert np.array_equal(mlp.quant_bf16(v), orc.quant_bf16(v))


def test_gradient_by_finite_differences():
    """Central differences of the plain FP64 network (no rounding) against the
    chain-rule gradient, on every parameter."""
    P = params(2)
    F, Y = data(3)
    loss, G = mlp.loss_and_grad(P, F, Y, DIMS, pos_weight=3.0, emulate=False)
    h = 1e-6
    fd = np.empty_like(P)
    for i in range(P.size):
        e = np.zeros_like(P)
        e[i] = h
        lp = mlp.loss_and_grad(P + e, F, Y, DIMS, 3.0, emulate=False)[0]
        lm = mlp.loss_and_grad(P - e, F, Y, DIMS, 3.0, emulate=False)[0]
        fd[i] = (lp - lm) / (2 * h)
    assert np.allclose(G, fd, rtol=1e-5, atol=1e-9)


def test_loss_matches_torch():
    P = params(4)
    F, Y = data(5)
    Z, _ = mlp.forward(P, F, DIMS, emulate=False)
    for w in (1.0, 7.5):
        want = torch.nn.functional.binary_cross_entropy_with_logits(
            torch.from_numpy(Z), torch.from_numpy(Y), pos_weight=torch.full((DIMS[3],), w, dtype=torch.float64))
        assert abs(mlp.bce_with_logits(Z, Y, w) - want.item()) < 1e-12


def test_forward_and_gradient_match_torch_autograd():
    P = params(6)
    F, Y = data(7)
    W = [torch.tensor(p, requires_grad=True) for p in mlp.unpack(P.copy(), DIMS)]
    f = torch.from_numpy(F)
    h1 = torch.relu(f @ W[0].T + W[1])
    h2 = torch.relu(h1 @ W[2].T + W[3])
    z = h2 @ W[4].T + W[5]
    loss = torch.nn.functional.binary_cross_entropy_with_logits(
        z, torch.from_numpy(Y), pos_weight=torch.full((DIMS[3],), 2.0, dtype=torch.float64))
    loss.backward()
    want = np.concatenate([w.grad.numpy().reshape(-1) for w in W])
    l, G = mlp.loss_and_grad(P, F, Y, DIMS, 2.0, emulate=False)
    assert abs(l - loss.item()) < 1e-12
    assert np.allclose(G, want, rtol=1e-10, atol=1e-14)


def test_adam_matches_torch():
    P = params(8)
    rng = np.random.default_rng(9)
    p_t = torch.tensor(P.copy(), requires_grad=True)
    opt = torch.optim.Adam([p_t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    M = np.zeros_like(P)
    V = np.zeros_like(P)
    Pn = P.copy()
    for step in range(1, 6):
        G = rng.standard_normal(P.size)
        opt.zero_grad()
        p_t.grad = torch.from_numpy(G.copy())
        opt.step()
        Pn, M, V = mlp.adam_step(Pn, G, M, V, step, 1e-2)
    assert np.allclose(Pn, p_t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_emulated_network_rounds_at_the_stated_points():
    """With emulation the logits equal those of the plain network evaluated on
    the rounded inputs and weights, with rounded activations."""
    P = params(10)
    F, _ = data(11)
    Z, (F0, H1, H2, W1r, W2r, W3r) = mlp.forward(P, F, DIMS, emulate=True)
    b = mlp.unpack(P, DIMS)
    assert np.array_equal(F0, mlp.quant_bf16(F))
    assert np.array_equal(H1, mlp.quant_bf16(np.maximum(F0 @ W1r.T + b[1], 0)))
    assert np.array_equal(Z, H2 @ W3r.T + b[5])
