"""Learned-proposal kernels against the FP64 oracle fed the same bfloat16
operands: layer forward (GELU / head), backward (dW, db, dX * gelu'), MSE,
a whole forward/backward pass, a finite-difference weight-gradient check, and a
training run that reduces the loss."""
import numpy as np
import pytest

from oracle import mlp as om

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def net():
    from paper_2511_13330_amd import spin_chain_system
    from paper_2511_13330_amd.mlp import ProposalMLP
    s = spin_chain_system(3, precision="f32", magnus_order=1, hold="zoh")
    return ProposalMLP(s, n_in=133, width=96, n_out=40, depth=4, amax=7.0, seed=3)


def oracle_params(net):
    return [(W.float().cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64))
            for W, b in zip(net.W16, net.b32)]


def test_bf16_cast_matches_oracle_rounding(net):
    x = np.random.default_rng(0).standard_normal(5000).astype(np.float32) * 3
    t = net.to_bf16(torch.tensor(x, device="cuda"))
    assert np.array_equal(t.float().cpu().numpy().astype(np.float64), om.bf16_round(x))


def test_forward_layers_and_head(net):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((70, 133)).astype(np.float32)    # ragged rows and k
    X16 = net.to_bf16(torch.tensor(X, device="cuda"))
    Y, (acts, pres) = net.forward(X16, keep=True)
    P = oracle_params(net)
    # feed each layer the GPU's own bf16 input so rounding decisions agree
    for li, (W, b) in enumerate(P):
        xin = acts[li].float().cpu().numpy().astype(np.float64)
        z = xin @ W.T + b
        assert np.allclose(pres[li].cpu().numpy(), z, rtol=1e-5, atol=1e-5)
        if li + 1 < len(P):
            g = om.bf16_round(om.gelu(pres[li].cpu().numpy().astype(np.float64)))
            a = acts[li + 1].float().cpu().numpy()
            assert np.mean(a != g) < 1e-3       # ties decided by fp32 vs fp64 erf
            assert np.allclose(a, g, rtol=2 ** -7, atol=1e-6)
    zo = pres[-1].cpu().numpy().astype(np.float64)
    assert np.allclose(Y.cpu().numpy(), 7.0 * om.sigmoid(zo), rtol=1e-5, atol=1e-6)


def test_backward_and_mse_match_oracle(net):
    rng = np.random.default_rng(2)
    X = rng.standard_normal((53, 133)).astype(np.float32)
    Yt = rng.uniform(0, 7, (53, 40)).astype(np.float32)
    X16 = net.to_bf16(torch.tensor(X, device="cuda"))
    loss, grads = net.loss_and_grads(X16, torch.tensor(Yt / 7.0, device="cuda"))
    P = oracle_params(net)
    pre, acts = om.forward(P, X16.float().cpu().numpy().astype(np.float64), round_bf16=True)
    lo, dz = om.mse_loss(pre[-1], (Yt / 7.0).astype(np.float64))
    g_or = om.backward(P, pre, acts, dz, round_bf16=True)
    assert abs(loss.item() - lo) < 1e-3 * lo
    for (dW, db), (oW, ob) in zip(grads, g_or):
        assert np.linalg.norm(dW.cpu().numpy() - oW) < 2e-2 * np.linalg.norm(oW)
        assert np.linalg.norm(db.cpu().numpy() - ob) < 2e-2 * np.linalg.norm(ob)


def test_weight_gradient_finite_differences(net):
    # FP64 loss of the network with the bf16 weights, no activation rounding;
    # central differences on 10 weights against the kernel gradient
    rng = np.random.default_rng(5)
    X = rng.standard_normal((32, 133)).astype(np.float32)
    Yt = rng.uniform(0, 1, (32, 40))
    X16 = net.to_bf16(torch.tensor(X, device="cuda"))
    _, grads = net.loss_and_grads(X16, torch.tensor(Yt.astype(np.float32), device="cuda"))
    P = oracle_params(net)
    Xo = X16.float().cpu().numpy().astype(np.float64)

    def L(ps):
        pre, _ = om.forward(ps, Xo, round_bf16=False)
        return om.mse_loss(pre[-1], Yt)[0]

    h = 1e-4
    for k in range(10):
        li = k % 4
        W, b = P[li]
        i, j = rng.integers(W.shape[0]), rng.integers(W.shape[1])
        Wp, Wm = W.copy(), W.copy()
        Wp[i, j] += h; Wm[i, j] -= h
        pp, pm = list(P), list(P)
        pp[li] = (Wp, b); pm[li] = (Wm, b)
        fd = (L(pp) - L(pm)) / (2 * h)
        gk = float(grads[li][0][i, j].item())
        scale = float(np.abs(grads[li][0].cpu().numpy()).max())
        assert abs(gk - fd) < 3e-2 * scale, (li, i, j, gk, fd)


def test_training_reduces_loss():
    from paper_2511_13330_amd import spin_chain_system
    from paper_2511_13330_amd.mlp import ProposalMLP
    s = spin_chain_system(3, precision="f32", magnus_order=1, hold="zoh")
    net = ProposalMLP(s, n_in=16, width=64, n_out=8, depth=4, amax=5.0, seed=1)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((1024, 16)).astype(np.float32)
    M = rng.standard_normal((16, 8)) / 4
    Y = 5.0 / (1.0 + np.exp(-(X @ M)))
    hist = net.train(torch.tensor(X, device="cuda"), torch.tensor(Y, dtype=torch.float32, device="cuda"),
                     epochs=15, batch=128, lr=3e-3)
    assert hist[-1] < 0.3 * hist[0]


def test_full_size_network_forward_backward():
    """The proposal network at its real shapes, 133 -> 512 -> 512 -> 512 -> 512,
    on 300 rows (several row tiles and a ragged tail): every layer's
    pre-activation, the head and all weight and bias gradients against the
    oracle fed the same bfloat16 operands."""
    from paper_2511_13330_amd import spin_chain_system
    from paper_2511_13330_amd.mlp import ProposalMLP
    s = spin_chain_system(3, precision="f32", magnus_order=1, hold="zoh")
    amax = 2 * np.pi * 20
    big = ProposalMLP(s, n_in=133, width=512, n_out=512, depth=4, amax=amax, seed=7)
    rng = np.random.default_rng(12)
    X = rng.standard_normal((300, 133)).astype(np.float32)
    Yt = rng.uniform(0, 1, (300, 512)).astype(np.float32)
    X16 = big.to_bf16(torch.tensor(X, device="cuda"))
    Y, (acts, pres) = big.forward(X16, keep=True)
    P = oracle_params(big)
    for li, (W, b) in enumerate(P):
        xin = acts[li].float().cpu().numpy().astype(np.float64)
        z = xin @ om.bf16_round(W).T + b
        assert np.allclose(pres[li].cpu().numpy(), z, rtol=1e-4, atol=1e-4), li
    zo = pres[-1].cpu().numpy().astype(np.float64)
    assert np.allclose(Y.cpu().numpy(), amax * om.sigmoid(zo), rtol=1e-5, atol=1e-5)
    loss, grads = big.loss_and_grads(X16, torch.tensor(Yt, device="cuda"))
    pre, acts_o = om.forward(P, X16.float().cpu().numpy().astype(np.float64), round_bf16=True)
    lo, dz = om.mse_loss(pre[-1], Yt.astype(np.float64))
    g_or = om.backward(P, pre, acts_o, dz, round_bf16=True)
    assert abs(loss.item() - lo) < 1e-3 * lo
    for (dW, db), (oW, ob) in zip(grads, g_or):
        assert np.linalg.norm(dW.cpu().numpy() - oW) < 2e-2 * np.linalg.norm(oW)
        assert np.linalg.norm(db.cpu().numpy() - ob) < 2e-2 * np.linalg.norm(ob)
