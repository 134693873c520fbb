"""Pins of the oracle's logical-subspace scores (Sec. III-C, Eq. 16-17) and of
its adjoint for a general score of U, against closed forms, the spin algebra of
the encoding (Sec. II-A, Eq. 2-3) and finite differences."""
import numpy as np
import pytest

import oracle
from oracle import logical as lg
import synth
from helpers import oracle_system


def haar2(seed):
    return synth.haar_unitary(np.random.default_rng(seed), 2)


def total_spin():
    S = [sum(oracle.spin_op(oracle.pauli(a), i, 3) for i in range(3)) / 2 for a in "xyz"]
    return S, sum(s @ s for s in S)


def test_encoding_is_an_orthonormal_spin_half_doublet():
    phi = np.stack(lg.logical_states(), axis=1)
    assert np.allclose(phi.conj().T @ phi, np.eye(2), atol=1e-15)
    S, S2 = total_spin()
    for k in range(2):
        assert np.allclose(S[2] @ phi[:, k], 0.5 * phi[:, k], atol=1e-14)          # S_z = +1/2
        assert np.allclose(S2 @ phi[:, k], 0.75 * phi[:, k], atol=1e-14)           # S = 1/2
    # 0_L = |u>_2 (x) singlet of spins 1 and 3: S_1 . S_3 = -3/4 on it, +1/4 on 1_L
    S13 = sum(oracle.spin_op(oracle.pauli(a), 0, 3) @ oracle.spin_op(oracle.pauli(a), 2, 3)
              for a in "xyz") / 4
    assert np.allclose(S13 @ phi[:, 0], -0.75 * phi[:, 0], atol=1e-14)
    assert np.allclose(S13 @ phi[:, 1], 0.25 * phi[:, 1], atol=1e-14)


@pytest.mark.parametrize("proj", ["populations", "operators"])
def test_projectors_are_orthonormal(proj):
    P = lg.populations_projector() if proj == "populations" else lg.operator_projector()
    assert np.allclose(P.conj().T @ P, np.eye(P.shape[1]), atol=1e-15)
    assert np.allclose(lg.projection(np.eye(64), P), np.eye(P.shape[1]), atol=1e-15)


def test_projection_of_a_logical_gate_closed_forms():
    V = haar2(3)
    U = oracle.superop_of_unitary(lg.embed(V))
    Pi_pop = lg.projection(U, lg.populations_projector())
    # Tr(rho_k W rho_l W^dag) = |<k|V|l>|^2
    assert np.allclose(Pi_pop, np.abs(V) ** 2, atol=1e-14)
    Pi_op = lg.projection(U, lg.operator_projector())
    assert np.allclose(Pi_op, np.kron(V.conj(), V), atol=1e-14)


def test_logical_process_fidelity_closed_form():
    V, W = haar2(4), haar2(5)
    U = oracle.superop_of_unitary(lg.embed(W))
    F, _ = lg.score(U, lg.operator_projector(), lg.gate_target(V), "linear")
    assert abs(F - abs(np.trace(V.conj().T @ W)) ** 2 / 4.0) < 1e-14
    F1, _ = lg.score(U, lg.operator_projector(), lg.gate_target(W), "linear")
    assert abs(F1 - 1.0) < 1e-14
    L0, _ = lg.score(U, lg.populations_projector(), lg.populations_target(W), "projected")
    assert L0 < 1e-28


@pytest.mark.parametrize("kind,proj", [("projected", "populations"), ("projected", "operators"),
                                       ("linear", "operators")])
def test_seed_is_the_derivative(kind, proj):
    rng = np.random.default_rng(6)
    P = lg.populations_projector() if proj == "populations" else lg.operator_projector()
    U0 = (rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))) / 8
    T = (rng.standard_normal((P.shape[1],) * 2) + 1j * rng.standard_normal((P.shape[1],) * 2))
    E = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    _, M = lg.score(U0, P, T, kind)
    h = 1e-4
    fd = (lg.score(U0 + h * E, P, T, kind)[0] - lg.score(U0 - h * E, P, T, kind)[0]) / (2 * h)
    assert abs(fd - np.real(np.trace(M @ E))) < 1e-8 * max(1.0, abs(fd))


def test_seed_adjoint_reproduces_the_fidelity_adjoint():
    cfg = synth.small_case(8, n_slices=6, dt=2.5e-4)
    osys = oracle_system(cfg)
    amps = cfg["amps"]
    ST = oracle.superop_of_unitary(cfg["U_target"])
    seed = lambda U: (float(np.real(np.trace(ST.conj().T @ U))) / 64.0, ST.conj().T / 64.0)
    F0, g0 = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    F1, g1 = oracle.grad_adjoint_seed(osys, amps, cfg["dt"], 2, "foh", seed)
    assert abs(F0 - F1) < 1e-15 and np.allclose(g0, g1, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kind,proj", [("projected", "populations"), ("linear", "operators")])
def test_seed_adjoint_matches_finite_differences(kind, proj):
    cfg = synth.small_case(9, n_slices=5, dt=2.5e-4)
    osys = oracle_system(cfg)
    amps = cfg["amps"]
    P = lg.populations_projector() if proj == "populations" else lg.operator_projector()
    T = lg.populations_target(haar2(10)) if proj == "populations" else lg.gate_target(haar2(10))
    f = lambda a: lg.score(oracle.propagate(osys.omegas(a, cfg["dt"], 2, "foh")), P, T, kind)[0]
    _, g = oracle.grad_adjoint_seed(osys, amps, cfg["dt"], 2, "foh", lambda U: lg.score(U, P, T, kind))
    h = 1e-3
    for m, c in [(0, 0), (2, 1), (4, 0)]:
        e = np.zeros_like(amps)
        e[m, c] = h
        fd = (f(amps + e) - f(amps - e)) / (2 * h)
        assert abs(fd - g[m, c]) < 1e-6 * max(1.0, abs(fd)), (m, c, fd, g[m, c])


def test_seed_adjoint_at_sampled_rows_matches_full():
    cfg = synth.small_case(12, n_slices=9, dt=2.5e-4)
    osys = oracle_system(cfg)
    P, T = lg.populations_projector(), lg.populations_target(haar2(13))
    fn = lambda U: lg.score(U, P, T, "projected")
    v0, g0 = oracle.grad_adjoint_seed(osys, cfg["amps"], cfg["dt"], 2, "foh", fn)
    v1, g1 = oracle.grad_adjoint_seed_at(osys, cfg["amps"], cfg["dt"], 2, "foh", fn, [0, 4, 8])
    assert v0 == v1
    for r in (0, 4, 8):
        assert np.allclose(g1[r], g0[r], rtol=1e-13, atol=1e-16)
