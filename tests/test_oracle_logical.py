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


# ------------------------------------------------ state-level reference
def test_uhlmann_closed_forms():
    from oracle import states as st
    rng = np.random.default_rng(20)
    psi = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    phi = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    psi /= np.linalg.norm(psi)
    phi /= np.linalg.norm(phi)
    F = st.uhlmann(np.outer(psi, psi.conj()) + 0 * 1e-300, np.outer(phi, phi.conj()))
    assert abs(F - abs(np.vdot(psi, phi)) ** 2) < 1e-8          # sqrtm of a rank-1 matrix
    p = rng.random(8); p /= p.sum()
    q = rng.random(8); q /= q.sum()
    assert abs(st.uhlmann(np.diag(p), np.diag(q)) - np.sum(np.sqrt(p * q)) ** 2) < 1e-13
    rho = st.random_density(8, rng)
    assert abs(st.uhlmann(rho, rho) - 1.0) < 1e-12


def test_rk4_state_constant_control_is_the_exponential():
    from oracle import states as st
    cfg = synth.small_case(21, n_slices=4)
    osys = oracle_system(cfg)
    u = np.array([2 * np.pi * 7.0, 2 * np.pi * 3.0])
    rho0 = st.random_density(8, np.random.default_rng(22))
    T = 0.05
    ref = oracle.unvec(sla_expm(T * osys.liouv(u)) @ oracle.vec(rho0), 8)
    e1 = np.abs(st.rk4_state(osys, lambda t: u, T, 200, rho0) - ref).max()
    e2 = np.abs(st.rk4_state(osys, lambda t: u, T, 400, rho0) - ref).max()
    assert e2 < 1e-10 and 12.0 < e1 / e2 < 20.0     # fourth order: halving h divides by 16


def sla_expm(A):
    import scipy.linalg
    return scipy.linalg.expm(A)
