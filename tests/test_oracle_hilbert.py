"""Pins of the oracle's closed-system Hilbert-space reduction and of its
slice-exponential action on a few columns (the references for the
superoperators too large for the dense FP64 path).

* The reduction is checked against the superoperator route it replaces (lifted
  Eq. 8 Liouvillian, Magnus on n x n matrices, Taylor expm): two independent
  evaluations of the same discretised method, so a wrong sign of -i H, a
  missing conjugate or a transposed Kronecker factor fails.
* Its fidelity and adjoint are checked against the superoperator fidelity and
  adjoint, against its own central differences, and on the two-spin SWAP
  closed form.
* The action is checked against scipy's expm (an external routine), against
  the dense Omega_n, and against the dense chain product.
"""
import numpy as np
import scipy.linalg

import oracle
from oracle import hilbert as hb
import synth

SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], complex)


def closed_case(seed, n_slices=6, dt=2.5e-3):
    cfg = synth.small_case(seed, n_slices=n_slices, dt=dt)
    return cfg, np.asarray(cfg["amps"], float)


def test_reduction_matches_superoperator_route():
    for order, hold in ((2, "foh"), (1, "zoh")):
        cfg, amps = closed_case(401)
        sup = oracle.System.from_cfg(cfg, dissipative=False)
        hs = hb.HilbertSystem.from_cfg(cfg)
        S = oracle.propagate(sup.omegas(amps, cfg["dt"], order, hold))
        V = hb.unitary(hs, amps, cfg["dt"], order, hold)
        assert np.allclose(V.conj().T @ V, np.eye(8), atol=1e-12)
        assert np.linalg.norm(hb.superop(V) - S) < 1e-11 * np.linalg.norm(S)


def test_reduction_with_noise_scales():
    cfg, amps = closed_case(402)
    eps, dB = np.array([1.013, 0.991]), np.array([0.3, -1.1, 2.0])
    sup = oracle.System.from_cfg(cfg, dissipative=False, eps=eps, dB=dB)
    hs = hb.HilbertSystem.from_cfg(cfg, eps=eps, dB=dB)
    S = oracle.propagate(sup.omegas(amps, cfg["dt"], 2, "foh"))
    V = hb.unitary(hs, amps, cfg["dt"], 2, "foh")
    assert np.linalg.norm(hb.superop(V) - S) < 1e-11 * np.linalg.norm(S)


def test_fidelity_and_adjoint_match_superoperator():
    cfg, amps = closed_case(403, n_slices=5)
    sup = oracle.System.from_cfg(cfg, dissipative=False)
    hs = hb.HilbertSystem.from_cfg(cfg)
    F_s, g_s = oracle.grad_adjoint(sup, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    F_h, g_h = hb.grad(hs, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    V = hb.unitary(hs, amps, cfg["dt"], 2, "foh")
    assert abs(hb.fidelity(V, cfg["U_target"]) - F_s) < 1e-13
    assert abs(F_h - F_s) < 1e-13
    assert np.linalg.norm(g_h - g_s) < 1e-9 * np.linalg.norm(g_s)


def test_adjoint_against_central_differences():
    cfg, amps = closed_case(404, n_slices=7)
    hs = hb.HilbertSystem.from_cfg(cfg, eps=np.array([0.98, 1.02]))
    _, g = hb.grad(hs, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    coords = np.arange(amps.size)
    fd = hb.grad_fd(hs, amps, cfg["dt"], 2, "foh", cfg["U_target"], coords, h=1e-3)
    assert np.linalg.norm(g.reshape(-1) - fd) < 1e-6 * np.linalg.norm(fd)
    rows = [0, 3, 6]
    _, g_at = hb.grad_at(hs, amps, cfg["dt"], 2, "foh", cfg["U_target"], rows)
    for r in rows:
        assert np.allclose(g_at[r], g[r], rtol=1e-12, atol=1e-15)


def test_two_spin_swap_closed_form():
    hs = hb.HilbertSystem(2, [0.0, 0.0])
    J, N = 2 * np.pi * 5.0, 10
    h = np.pi / J / N
    V = hb.unitary(hs, np.full((N, 1), J), h, 2, "foh")
    assert abs(hb.fidelity(V, SWAP) - 1.0) < 1e-13
    # exp(i J t / 4) [cos(J t / 2) I - i sin(J t / 2) SWAP] at J t = pi / 2
    V2 = hb.unitary(hs, np.full((N, 1), J), h / 2, 1, "zoh")
    t = np.pi / 2 / J
    ref = np.exp(1j * J * t / 4) * (np.cos(J * t / 2) * np.eye(4) - 1j * np.sin(J * t / 2) * SWAP)
    assert np.allclose(V2, ref, atol=1e-13)


def test_expm_action_against_scipy():
    rng = np.random.default_rng(7)
    A = (rng.standard_normal((30, 30)) + 1j * rng.standard_normal((30, 30))) * 0.4
    X = rng.standard_normal((30, 3)) + 0j
    nrm = float(np.abs(A).sum(axis=0).max())
    assert nrm > 4            # several halvings
    got = hb.expm_action(lambda Y: A @ Y, nrm, X)
    ref = scipy.linalg.expm(A) @ X
    assert np.linalg.norm(got - ref) < 1e-12 * np.linalg.norm(ref)


def test_omega_action_and_columns_match_dense_path():
    cfg = synth.small_case(405, n_slices=4, dt=1e-3)
    amps = np.asarray(cfg["amps"], float)
    sysm = oracle.System.from_cfg(cfg)
    for order, hold in ((2, "foh"), (1, "zoh")):
        om = oracle.slice_omega(sysm.liouv, amps, 2, cfg["dt"], order, hold)
        apply, bound = hb.omega_action(sysm, amps, 2, cfg["dt"], order, hold)
        assert np.allclose(apply(np.eye(64)), om, atol=1e-15)
        assert bound >= float(np.abs(om).sum(axis=0).max())
        U = oracle.propagate(sysm.omegas(amps, cfg["dt"], order, hold))
        cols = [0, 9, 27, 63]
        got = hb.propagator_columns(sysm, amps, cfg["dt"], order, hold, cols)
        assert np.linalg.norm(got - U[:, cols]) < 1e-12 * np.linalg.norm(U[:, cols])
