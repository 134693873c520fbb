"""Pins of the oracle's Hubbard model (Eq. 1): fermionic algebra, symmetries,
closed forms of the diagonal and of the two-site exchange, and the closed-system
reduction of its superoperator propagator."""
import numpy as np

import oracle
from oracle import hubbard as hu
from oracle import hilbert as hb


def rand_coef(rng, n_dots):
    return np.concatenate([[rng.uniform(50, 80)], rng.uniform(-10, 10, n_dots), [rng.uniform(5, 15)]])


def test_canonical_anticommutation_three_dots():
    c = hu.annihilators(3)
    eye = np.eye(64)
    for a in range(6):
        for b in range(6):
            assert np.allclose(c[a] @ c[b].conj().T + c[b].conj().T @ c[a], eye * (a == b))
            assert np.allclose(c[a] @ c[b] + c[b] @ c[a], 0.0)


def test_hermitian_and_conserves_number_and_sz():
    rng = np.random.default_rng(1)
    N, Sz = hu.total_number(3), hu.total_sz(3)
    for _ in range(3):
        H = hu.hamiltonian(rng.uniform(-20, 20, 2), rand_coef(rng, 3), 3)
        assert np.allclose(H, H.conj().T)
        assert np.allclose(H @ N - N @ H, 0.0)
        assert np.allclose(H @ Sz - Sz @ H, 0.0)
    for L in hu.jump_ops(3, 100.0, 2.0):
        assert np.allclose(L @ N - N @ L, 0.0)          # no electron leaves a dot array


def test_zero_hopping_is_diagonal_closed_form():
    """t = 0: H is diagonal with sum_i [U/2 n_i (n_i - 1) + V_i n_i] + U_C sum n_i n_{i+1},
    n_i the electron count of dot i read off the basis index."""
    rng = np.random.default_rng(2)
    coef = rand_coef(rng, 3)
    U, V, UC = coef[0], coef[1:4], coef[4]
    H = hu.hamiltonian([0.0, 0.0], coef, 3)
    diag = []
    for s in range(64):
        n = [bin((s >> (2 * (2 - i))) & 3).count("1") for i in range(3)]
        diag.append(sum(0.5 * U * k * (k - 1) + v * k for k, v in zip(n, V))
                    + UC * (n[0] * n[1] + n[1] * n[2]))
    assert np.allclose(H, np.diag(diag))


def test_two_site_exchange_splitting():
    """Two dots, two electrons, no V or U_C: the singlet lies at
    (U - sqrt(U^2 + 16 t^2)) / 2, the triplet at 0, so J = E_T - E_S -> 4 t^2 / U."""
    N, Sz = hu.total_number(2), hu.total_sz(2)
    for U, t in ((60.0, 3.0), (60.0, 0.3), (10.0, 4.0)):
        H = hu.hamiltonian([t], [U, 0.0, 0.0, 0.0], 2)
        sel0 = np.where((np.abs(np.diag(N) - 2) < 1e-12) & (np.abs(np.diag(Sz)) < 1e-12))[0]
        sel1 = np.where((np.abs(np.diag(N) - 2) < 1e-12) & (np.abs(np.diag(Sz) - 1) < 1e-12))[0]
        e0 = np.linalg.eigvalsh(H[np.ix_(sel0, sel0)])
        e1 = np.linalg.eigvalsh(H[np.ix_(sel1, sel1)])
        assert np.isclose(e0[0], (U - np.sqrt(U * U + 16 * t * t)) / 2, atol=1e-12)
        assert np.allclose(e1, 0.0, atol=1e-12)
        J = e1[0] - e0[0]
        if t / U < 0.01:
            assert abs(J / (4 * t * t / U) - 1) < 1e-3


def test_single_electron_hopping():
    N = hu.total_number(2)
    t, V = 7.0, 2.5
    H = hu.hamiltonian([t], [30.0, V, V, 4.0], 2)
    sel = np.where(np.abs(np.diag(N) - 1) < 1e-12)[0]
    e = np.linalg.eigvalsh(H[np.ix_(sel, sel)])
    assert np.allclose(e, [V - t, V - t, V + t, V + t])


def test_closed_reduction_and_adjoint():
    """Two dots (superoperator 256 x 256): the Hilbert reduction equals the
    superoperator route, and its adjoint equals central differences."""
    rng = np.random.default_rng(3)
    coef = rand_coef(rng, 2)
    amps = rng.uniform(0, 20, (5, 1))
    dt = 5e-3
    sup = hu.HubbardSystem(2, coef)
    hil = hu.HubbardHilbert(2, coef)
    S = oracle.propagate(sup.omegas(amps, dt, 2, "foh"))
    V = hb.unitary(hil, amps, dt, 2, "foh")
    assert np.linalg.norm(hb.superop(V) - S) < 1e-11 * np.linalg.norm(S)
    Ut = np.linalg.qr(rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16)))[0]
    F, g = hb.grad(hil, amps, dt, 2, "foh", Ut)
    assert abs(F - oracle.fidelity(S, Ut)[0]) < 1e-13
    fd = hb.grad_fd(hil, amps, dt, 2, "foh", Ut, np.arange(amps.size), h=1e-4)
    assert np.linalg.norm(g.reshape(-1) - fd) < 1e-6 * np.linalg.norm(fd)


def test_dissipative_trace_preservation():
    rng = np.random.default_rng(4)
    sysm = hu.HubbardSystem(2, rand_coef(rng, 2), T1=100.0, T2=2.0)
    om = oracle.slice_omega(sysm.liouv, rng.uniform(0, 20, (3, 1)), 1, 5e-3, 2, "foh")
    S = oracle.expm_taylor(om)
    vI = np.eye(16).T.reshape(-1)
    assert np.allclose(vI @ S, vI, atol=1e-13)


def test_jump_operators_on_one_dot():
    """One dot: the spin flip maps |up> to |down> / sqrt(T1) and annihilates
    |0>, |down>, |up down>; the dephasing operator is diag(0, 1, -1, 0) / sqrt(T2)."""
    L1, L2 = hu.jump_ops(1, 4.0, 9.0)
    ref1 = np.zeros((4, 4))
    ref1[2, 1] = 0.5
    assert np.allclose(L1, ref1)
    assert np.allclose(L2, np.diag([0, 1, -1, 0]) / 3.0)
