"""Learned pulse proposal: a multilayer perceptron that maps a target unitary
and device parameters to initial pulse amplitudes, trained and run by the
library's own kernels (bfloat16 MFMA products with FP32 accumulation, fused
bias+GELU, scaled-sigmoid head, MSE, Adam on FP32 master weights).

Input features (133 for a 3-spin, 2-control system): the target with its
global phase fixed (largest-magnitude entry of the first column made real and
positive), real parts row-major (64), imaginary parts (64), the Zeeman fields
B_i / (2 pi 10), the field-noise scale / (2 pi 1) and the exchange-noise scale
/ 0.01. Output: n_ctrl x n_slices amplitudes, amax * sigmoid(z), slice-major.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import lib, check


def features(U_target, B, sigB, sigJ):
    """Feature matrix [n, 133] (float32, host) for targets [n, d, d]."""
    U = np.asarray(U_target, dtype=np.complex128).reshape(-1, *np.shape(U_target)[-2:])
    n, d, _ = U.shape
    col = U[:, :, 0]
    k = np.argmax(np.abs(col), axis=1)
    ph = col[np.arange(n), k]
    U = U * (np.abs(ph) / ph)[:, None, None]
    B = np.asarray(B, dtype=float).reshape(n, -1)
    two_pi = 2.0 * np.pi
    X = np.concatenate([U.real.reshape(n, -1), U.imag.reshape(n, -1), B / (two_pi * 10.0),
                        (np.asarray(sigB, float) / (two_pi * 1.0)).reshape(n, 1),
                        (np.asarray(sigJ, float) / 0.01).reshape(n, 1)], axis=1)
    return X.astype(np.float32)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class ProposalMLP:
    """Linear(n_in, 512) GELU Linear(512, 512) GELU Linear(512, 512) GELU
    Linear(512, n_out), head amax * sigmoid."""

    def __init__(self, system, n_in=133, width=512, n_out=512, depth=4, amax=1.0, seed=0):
        self.sys = system
        self.dev = system.device
        self.amax = float(amax)
        self.sizes = [n_in] + [width] * (depth - 1) + [n_out]
        rng = np.random.default_rng(seed)
        self.W32, self.b32, self.W16 = [], [], []
        for i, o in zip(self.sizes[:-1], self.sizes[1:]):
            bound = 1.0 / np.sqrt(i)
            W = torch.tensor(rng.uniform(-bound, bound, (o, i)), dtype=torch.float32, device=self.dev)
            b = torch.tensor(rng.uniform(-bound, bound, o), dtype=torch.float32, device=self.dev)
            self.W32.append(W.contiguous())
            self.b32.append(b.contiguous())
            self.W16.append(torch.empty((o, i), dtype=torch.bfloat16, device=self.dev))
        self._m = [torch.zeros_like(t) for t in self.W32 + self.b32]
        self._v = [torch.zeros_like(t) for t in self.W32 + self.b32]
        self.step_count = 0
        self.sync_weights()

    @property
    def _ctx(self):
        return self.sys._ctx

    def _cast(self, src, dst):
        check(lib().lmag_cast_bf16(self._ctx, _p(src), _p(dst), src.numel(),
                                   _lib.c_void_p(torch.cuda.current_stream().cuda_stream)),
              self._ctx)

    def sync_weights(self):
        for W, W16 in zip(self.W32, self.W16):
            self._cast(W, W16)

    def to_bf16(self, X32):
        X32 = X32.contiguous()
        out = torch.empty(X32.shape, dtype=torch.bfloat16, device=self.dev)
        self._cast(X32, out)
        return out

    # ----------------------------------------------------------------- passes
    def forward(self, X16, keep=False):
        """X16: bf16 [rows, n_in]. Returns amplitudes [rows, n_out] (fp32) and,
        with keep, the cache for backward."""
        rows = X16.shape[0]
        st = _lib.c_void_p(torch.cuda.current_stream().cuda_stream)
        acts, pres = [X16], []
        L = len(self.W16)
        Y = None
        for li in range(L):
            n_in, n_out = self.sizes[li], self.sizes[li + 1]
            pre = torch.empty((rows, n_out), dtype=torch.float32, device=self.dev)
            if li + 1 < L:
                Y = torch.empty((rows, n_out), dtype=torch.bfloat16, device=self.dev)
                act = _lib_act_gelu()
            else:
                Y = torch.empty((rows, n_out), dtype=torch.float32, device=self.dev)
                act = _lib_act_sigmoid()
            check(lib().lmag_mlp_forward(self._ctx, rows, n_in, n_out, _p(acts[-1]), _p(self.W16[li]),
                                         _p(self.b32[li]), act, self.amax, _p(pre), _p(Y), st),
                  self._ctx)
            pres.append(pre)
            if li + 1 < L:
                acts.append(Y)
        return (Y, (acts, pres)) if keep else Y

    def loss_and_grads(self, X16, Yn):
        """MSE of sigmoid(z) against Yn = targets / amax; returns (loss tensor
        [1] float64 on device, [(dW, db)] per layer)."""
        rows = X16.shape[0]
        st = _lib.c_void_p(torch.cuda.current_stream().cuda_stream)
        _, (acts, pres) = self.forward(X16, keep=True)
        z = pres[-1]
        loss = torch.empty(1, dtype=torch.float64, device=self.dev)
        g32 = torch.empty_like(z)
        g16 = torch.empty(z.shape, dtype=torch.bfloat16, device=self.dev)
        check(lib().lmag_mlp_mse(self._ctx, z.numel(), _p(z), _p(Yn.contiguous()), _p(g32), _p(g16),
                                 _p(loss), st), self._ctx)
        grads = [None] * len(self.W16)
        for li in range(len(self.W16) - 1, -1, -1):
            n_in, n_out = self.sizes[li], self.sizes[li + 1]
            dW = torch.empty((n_out, n_in), dtype=torch.float32, device=self.dev)
            db = torch.empty(n_out, dtype=torch.float32, device=self.dev)
            p16 = p32 = pre_prev = None
            if li > 0:
                p16 = torch.empty((rows, n_in), dtype=torch.bfloat16, device=self.dev)
                p32 = torch.empty((rows, n_in), dtype=torch.float32, device=self.dev)
                pre_prev = pres[li - 1]
            check(lib().lmag_mlp_backward(self._ctx, rows, n_in, n_out, _p(acts[li]), _p(self.W16[li]),
                                          _p(g16), _p(g32), _p(dW), _p(db), _p(pre_prev), _p(p16),
                                          _p(p32), st), self._ctx)
            grads[li] = (dW, db)
            g16, g32 = p16, p32
        return loss, grads

    def adam_step(self, grads, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.step_count += 1
        params = self.W32 + self.b32
        gl = [g[0] for g in grads] + [g[1] for g in grads]
        for p, g, m, v in zip(params, gl, self._m, self._v):
            p2 = p.view(-1, 1) if p.dim() == 1 else p
            self.sys_f32_adam(p2, g.view(p2.shape), m.view(p2.shape), v.view(p2.shape),
                              lr, betas, eps)
        self.sync_weights()

    def sys_f32_adam(self, p, g, m, v, lr, betas, eps):
        check(lib().lmag_adam_project(
            self._ctx, _lib.LMAG_F32, p.shape[0], p.shape[1], _p(p), _p(g), _p(m), _p(v),
            self.step_count, float(lr), float(betas[0]), float(betas[1]), float(eps), 1.0,
            float("-inf"), float("inf"), None,
            _lib.c_void_p(torch.cuda.current_stream().cuda_stream)), self._ctx)

    def train(self, X32, Y, epochs=20, batch=256, lr=1e-3, seed=0, log=None):
        """Minibatch Adam on (X32 [n, n_in] fp32, Y [n, n_out] amplitudes)."""
        n = X32.shape[0]
        Yn = (Y / self.amax).to(torch.float32).contiguous()
        rng = np.random.default_rng(seed)
        hist = []
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(n), device=self.dev)
            tot = 0.0
            for s in range(0, n - batch + 1, batch):
                idx = perm[s:s + batch]
                Xb = self.to_bf16(X32[idx])
                loss, grads = self.loss_and_grads(Xb, Yn[idx])
                self.adam_step(grads, lr=lr)
                tot += float(loss.item()) * batch
            hist.append(tot / max(1, (n // batch) * batch))
            if log:
                log(f"epoch {ep}: loss {hist[-1]:.5f}")
        return hist

    def propose(self, X32):
        return self.forward(self.to_bf16(X32))

    def state_dict(self):
        out = {}
        for i, (W, b) in enumerate(zip(self.W32, self.b32)):
            out[f"W{i}"] = W.cpu().numpy()
            out[f"b{i}"] = b.cpu().numpy()
        return out

    def load_state_dict(self, d):
        for i in range(len(self.W32)):
            self.W32[i].copy_(torch.as_tensor(d[f"W{i}"], device=self.dev))
            self.b32[i].copy_(torch.as_tensor(d[f"b{i}"], device=self.dev))
        self.sync_weights()


def _lib_act_gelu():
    return 1


def _lib_act_sigmoid():
    return 2
