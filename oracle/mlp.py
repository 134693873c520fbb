"""Reference for the learned pulse proposal (oracle).

A plain multilayer perceptron: Linear layers y = x W^T + b with GELU
(exact, 0.5 x (1 + erf(x / sqrt 2))) after every hidden layer and a head
amax * sigmoid(z). Loss: mean squared error between sigmoid(z) and the target
amplitudes divided by amax. Arithmetic is float64; operands that the GPU keeps
in bfloat16 (weights, activations fed to a product) are rounded with
bf16_round before use when round_bf16 is set, so that both sides multiply
identical values.
"""
import math

import numpy as np

_SQRT2 = math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)
_erf = np.vectorize(math.erf, otypes=[float])


def bf16_round(x):
    """Round to bfloat16 (round to nearest, ties to even) via float32 bits;
    returns float64 values."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / _SQRT2))


def gelu_grad(x):
    return 0.5 * (1.0 + _erf(x / _SQRT2)) + x * _INV_SQRT_2PI * np.exp(-0.5 * x * x)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, X, round_bf16=True):
    """params: list of (W [n_out, n_in], b [n_out]). Returns (pre, acts):
    pre[l] = acts[l] W_l^T + b_l; acts[0] = X; acts[l+1] = gelu(pre[l]) for
    hidden layers; the last pre is the head's logit z."""
    rnd = bf16_round if round_bf16 else (lambda a: np.asarray(a, dtype=float))
    acts = [rnd(X)]
    pre = []
    for li, (W, b) in enumerate(params):
        z = acts[-1] @ rnd(W).T + np.asarray(b, dtype=float)
        pre.append(z)
        if li + 1 < len(params):
            acts.append(rnd(gelu(z)))
    return pre, acts


def mse_loss(z, Yn):
    """mean((sigmoid(z) - Yn)^2) and its gradient with respect to z."""
    p = sigmoid(z)
    diff = p - Yn
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff * p * (1.0 - p) / diff.size
    return loss, dz


def backward(params, pre, acts, dz, round_bf16=True):
    """Gradients [(dW, db)] of the loss whose gradient wrt the head logit is dz.
    With round_bf16 the incoming gradient of every product is rounded to
    bfloat16 before it is multiplied, as on the GPU."""
    rnd = bf16_round if round_bf16 else (lambda a: np.asarray(a, dtype=float))
    grads = [None] * len(params)
    g = dz
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        gq = rnd(g)
        grads[li] = (gq.T @ acts[li], g.sum(axis=0))
        if li > 0:
            da = gq @ rnd(W)
            g = da * gelu_grad(pre[li - 1])
    return grads
