"""The real representation behind the FP32 default (`basis="hermitian"`),
pinned on the oracle's own operators, on the CPU.

In the orthonormal basis of Hermitian operators |k><k|, (|k><l| + |l><k|)/sqrt 2
and i(|l><k| - |k><l|)/sqrt 2 every superoperator that maps Hermitian matrices
to Hermitian matrices is a real matrix. The library relies on this for the
Liouvillian of Eq. 8, its Magnus commutators, the slice exponentials and their
products (Eq. 14-15) and the target channel of the process fidelity; these
tests check each of those facts on the oracle's operators, the unitarity of
the change of basis, the invariance of the fidelity trace, and the two
identities the logical score uses (its projector and the real part of its
seed)."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import synth
from helpers import hermitian_basis_change, oracle_system
from oracle.liouville import liouvillian


def rand_herm(rng, d):
    X = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    return (X + X.conj().T) / 2


def rand_cplx(rng, d):
    return rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))


def to_real(S, T):
    return T @ S @ T.conj().T


@pytest.mark.parametrize("d", [2, 3, 4, 8])
def test_change_of_basis_is_unitary(d):
    T = hermitian_basis_change(d)
    assert np.allclose(T @ T.conj().T, np.eye(d * d), atol=1e-15)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_liouvillian_and_its_commutators_are_real(d):
    rng = np.random.default_rng(10 + d)
    T = hermitian_basis_change(d)
    L1 = liouvillian(rand_herm(rng, d), [rand_cplx(rng, d), rand_cplx(rng, d)])
    L2 = liouvillian(rand_herm(rng, d), [rand_cplx(rng, d)])
    for S in (L1, L2, L1 @ L2 - L2 @ L1, expm(0.1 * L1), expm(0.1 * L2) @ expm(0.1 * L1)):
        R = to_real(S, T)
        assert np.abs(R.imag).max() <= 1e-12 * max(1.0, np.abs(R).max())
    # a map that does not preserve Hermiticity is not real there
    A = rand_cplx(rng, d)
    assert np.abs(to_real(np.kron(np.eye(d), A), T).imag).max() > 1e-3


def test_spin_chain_propagator_real_and_recovered():
    """The oracle's 3-spin propagator of a short pulse: real in the basis of
    Hermitian operators, and T^dag R T gives it back."""
    cfg = synth.small_case(7, n_slices=12, dt=2.5e-4)
    osys = oracle_system(cfg)
    S = oracle.propagate(osys.omegas(cfg["amps"], cfg["dt"], 2, "foh"))
    T = hermitian_basis_change(8)
    R = to_real(S, T)
    assert np.abs(R.imag).max() <= 1e-13
    assert np.allclose(T.conj().T @ R.real @ T, S, atol=1e-13)


def test_fidelity_trace_invariant():
    """F = Re Tr(S_T^dag S) / d^2 with S_T = conj(U) (x) U, and
    Tr(R_T^T R) with R_T = T S_T T^dag real: the same number."""
    rng = np.random.default_rng(3)
    d = 4
    T = hermitian_basis_change(d)
    U = synth.haar_unitary(rng, d)
    ST = np.kron(U.conj(), U)
    S = expm(0.2 * liouvillian(rand_herm(rng, d), [rand_cplx(rng, d) * 0.3]))
    RT, R = to_real(ST, T), to_real(S, T)
    assert np.abs(RT.imag).max() <= 1e-13
    F_col = np.trace(ST.conj().T @ S).real / d ** 2
    F_real = np.trace(RT.real.T @ R.real) / d ** 2
    assert abs(F_col - F_real) <= 1e-14
    # the seed the real path stores: T S_T^dag T^dag = R_T^T
    assert np.allclose(to_real(ST.conj().T, T), RT.T, atol=1e-13)


def test_logical_projector_and_seed_identities():
    """P^dag U P = (T P)^dag R (T P) for U = T^dag R T, and for a real change
    dR of R: Re Tr(M dU) = Tr(Re(T M T^dag) dR) for any complex seed M."""
    rng = np.random.default_rng(5)
    d, L = 4, 3
    n = d * d
    T = hermitian_basis_change(d)
    S = expm(0.3 * liouvillian(rand_herm(rng, d), [rand_cplx(rng, d) * 0.2]))
    R = to_real(S, T).real
    P = rng.normal(size=(n, L)) + 1j * rng.normal(size=(n, L))
    TP = T @ P
    assert np.allclose(P.conj().T @ S @ P, TP.conj().T @ R @ TP, atol=1e-12)
    M = rand_cplx(rng, n)
    dR = rng.normal(size=(n, n))
    dU = T.conj().T @ dR @ T
    lhs = np.trace(M @ dU).real
    rhs = np.trace(to_real(M, T).real @ dR)
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
