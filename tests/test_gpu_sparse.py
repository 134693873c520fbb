"""Sparse-basis kernels (Omega_n built from the nonzero basis entries, compact
K_n^T, sparse traces) against the dense ones. The same physics written in a
randomly rotated Hilbert-space basis, H -> V H V^dag and L -> V L V^dag, has
dense superoperator terms and takes the dense kernels, while the propagator is
conjugated by conj(V) (x) V, so F against the rotated target and the whole
gradient are unchanged: an exact invariance, checked here to rounding."""
import numpy as np
import pytest

import synth
from helpers import rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def pair(prec, order, hold, seed=31, chunk=7):
    from paper_2511_13330_amd import System
    from paper_2511_13330_amd.spin import chain_operators
    cfg = synth.small_case(seed, n_slices=40, dt=2.5e-4 if order == 2 else 1e-3)
    hs, hc, lj = chain_operators(3, cfg["T1"], cfg["T2"])
    V = synth.haar_unitary(np.random.default_rng(seed + 1), 8)
    rot = lambda X: V @ X @ V.conj().T
    kw = dict(precision=prec, magnus_order=order, hold=hold, chunk_slices=chunk)
    s_sp = System(hs, hc, lj, **kw)
    s_dn = System([rot(h) for h in hs], [rot(h) for h in hc], [rot(L) for L in lj], **kw)
    return cfg, V, rot, s_sp, s_dn


@pytest.mark.parametrize("prec,order,hold", [("f32", 2, "foh"), ("f64", 2, "foh"), ("f64", 1, "zoh")])
def test_sparse_and_dense_kernels_agree(prec, order, hold):
    cfg, V, rot, s_sp, s_dn = pair(prec, order, hold)
    dt_ = torch.float32 if prec == "f32" else torch.float64
    a = torch.tensor(cfg["amps"], dtype=dt_, device="cuda").contiguous()
    b = np.asarray(cfg["B"])[None, :]
    F1, g1 = s_sp.fidelity_and_grad(a, [40], cfg["dt"], cfg["U_target"], static_coef=b)
    assert s_sp.last_plan()["sparse_support"] > 0
    F2, g2 = s_dn.fidelity_and_grad(a, [40], cfg["dt"], rot(cfg["U_target"]), static_coef=b)
    assert s_dn.last_plan()["sparse_support"] == 0
    tolF, tolg = (2e-6, 2e-4) if prec == "f32" else (1e-12, 1e-9)
    assert abs(F1.item() - F2.item()) < tolF
    assert rel(g2.cpu().numpy(), g1.cpu().numpy()) < tolg
    # propagators: S_dense = W S_sparse W^dag with W = conj(V) (x) V
    S1 = s_sp.propagate(a, [40], cfg["dt"], static_coef=b).cpu().numpy()[0].astype(complex)
    S2 = s_dn.propagate(a, [40], cfg["dt"], static_coef=b).cpu().numpy()[0].astype(complex)
    W = np.kron(V.conj(), V)
    assert rel(S2, W @ S1 @ W.conj().T) < (1e-5 if prec == "f32" else 1e-12)

