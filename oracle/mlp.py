"""FP64 oracle of the learned-proposal network (TEST INFRASTRUCTURE ONLY).

z = W3 relu(W2 relu(W1 f + b1) + b2) + b3, binary cross-entropy with logits
and positive weight w+ (mean over all entries of
-[w+ y log s(z) + (1-y) log(1-s(z))]), its gradient by the chain rule, and
Adam (Kingma and Ba, 2015: beta1 0.9, beta2 0.999, eps 1e-8).

With ``emulate=True`` the values that the GPU rounds to bfloat16 are rounded
here too, at the same points (inputs, weights, activations and back-propagated
gradients where they enter a matrix product); all arithmetic stays FP64.  With
``emulate=False`` it is the plain FP64 network (used for the finite-difference
pins).  Parameters are one flat array: W1 [h1][d_in], b1 [h1], W2 [h2][h1],
b2 [h2], W3 [d_out][h2], b3 [d_out].
"""
import numpy as np


def quant_bf16(x):
    """Round every entry to the nearest bfloat16 (ties to even), from the
    format's definition: 8 significant bits, FP32 exponent range."""
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    # log2 may be off by one next to powers of two: correct with an exact test
    e = np.where(np.exp2(e) > ax, e - 1, e)
    e = np.where(np.exp2(e + 1) <= ax, e + 1, e)
    e = np.maximum(e, -126.0)
    q = np.exp2(e - 7)
    y = x / q
    f = np.floor(y)
    r = y - f
    n = np.where(r > 0.5, f + 1, np.where(r < 0.5, f, np.where(np.mod(f, 2) == 0, f, f + 1)))
    out = np.where(ax > 0, n * q, x)
    return np.where(np.abs(out) >= 2.0 ** 128, np.copysign(np.inf, x), out)


def shapes(d_in, h1, h2, d_out):
    return [(h1, d_in), (h1,), (h2, h1), (h2,), (d_out, h2), (d_out,)]


def unpack(P, dims):
    out, off = [], 0
    for shp in shapes(*dims):
        size = int(np.prod(shp))
        out.append(P[off:off + size].reshape(shp))
        off += size
    return out


def _r(x, emulate):
    return quant_bf16(x) if emulate else x


def forward(P, F, dims, emulate=True):
    """Logits and the intermediate values the backward pass needs."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(P, dtype=np.float64), dims)
    W1r, W2r, W3r = _r(W1, emulate), _r(W2, emulate), _r(W3, emulate)
    F0 = _r(np.asarray(F, dtype=np.float64), emulate)
    H1 = _r(np.maximum(F0 @ W1r.T + b1, 0.0), emulate)
    H2 = _r(np.maximum(H1 @ W2r.T + b2, 0.0), emulate)
    Z = H2 @ W3r.T + b3
    return Z, (F0, H1, H2, W1r, W2r, W3r)


def bce_with_logits(Z, Y, pos_weight):
    """Mean over all entries of -[w+ y log s(z) + (1 - y) log(1 - s(z))]."""
    Z = np.asarray(Z, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    softplus_pos = np.logaddexp(0.0, Z)      # -log(1 - s(z))
    softplus_neg = np.logaddexp(0.0, -Z)     # -log s(z)
    return float(np.mean(pos_weight * Y * softplus_neg + (1 - Y) * softplus_pos))


def loss_and_grad(P, F, Y, dims, pos_weight, emulate=True):
    """Loss and its gradient with respect to the flat parameters (through the
    rounded copies when emulating, as the GPU does)."""
    Z, (F0, H1, H2, W1r, W2r, W3r) = forward(P, F, dims, emulate)
    Y = np.asarray(Y, dtype=np.float64)
    loss = bce_with_logits(Z, Y, pos_weight)
    s = 1.0 / (1.0 + np.exp(-Z))
    dZ = (s * (pos_weight * Y + 1 - Y) - pos_weight * Y) / Z.size
    dZr = _r(dZ, emulate)
    dW3 = dZr.T @ H2
    db3 = dZ.sum(0)
    dH2 = (dZr @ W3r) * (H2 > 0)
    dH2r = _r(dH2, emulate)
    dW2 = dH2r.T @ H1
    db2 = dH2.sum(0)
    dH1 = (dH2r @ W2r) * (H1 > 0)
    dH1r = _r(dH1, emulate)
    dW1 = dH1r.T @ F0
    db1 = dH1.sum(0)
    G = np.concatenate([g.reshape(-1) for g in (dW1, db1, dW2, db2, dW3, db3)])
    return loss, G


def adam_step(P, G, M, V, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (P, M, V)."""
    M = b1 * M + (1 - b1) * G
    V = b2 * V + (1 - b2) * G * G
    mh = M / (1 - b1 ** step)
    vh = V / (1 - b2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), M, V
