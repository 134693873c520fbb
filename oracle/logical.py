"""Logical-subspace scores of the pulse optimiser (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Encoding (Sec. II-A, Eq. 2 and 3) in the 3-spin basis of ``oracle.model``
(spin 1 the most significant factor, up = index 0):
    |0_L> = (|uud> - |duu>) / sqrt 2,
    |1_L> = (2 |udu> - |uud> - |duu>) / sqrt 6.
The paper states the encoding for a 64-dimensional Hubbard space and prints
basis indices that fit no ordering of it; here the encoding is written out in
the 8-dimensional spin space the propagator uses.

A projector P (n x L, n = d^2) has the column-stacked vectors vec(O_k) of L
logical operators as columns:
    populations (the paper's P, Sec. III-C): O_0 = rho_0, O_1 = rho_1 with
        rho_k = |k_L><k_L|;
    operator basis: O_{a + 2b} = |a_L><b_L| (a, b in {0, 1}), which carries the
        whole logical channel.
Pi = P^dag U P is the L x L projection of Eq. 16. Two scores of Pi:
    "projected": ||Pi - T||_F^2, the Frobenius loss of Eq. 17 with ||A||_F^2 =
        Tr(A^dag A) (the printed transpose read as the conjugate transpose);
    "linear":    Re Tr(T^dag Pi) / L, which for the operator basis and
        T = conj(V) (x) V is the process fidelity of the logical gate V.
Each score s(U) has dS = Re Tr(M dU) for the seed M returned with it, which
is what the adjoint needs (``propagator.grad_adjoint_seed``).
"""
import numpy as np

from .liouville import vec


def logical_states():
    """(phi_0, phi_1) as length-8 complex vectors."""
    e = np.eye(8, dtype=complex)
    uud, udu, duu = e[1], e[2], e[4]
    phi0 = (uud - duu) / np.sqrt(2.0)
    phi1 = (2.0 * udu - uud - duu) / np.sqrt(6.0)
    return phi0, phi1


def populations_projector():
    """n x 2: vec(rho_0), vec(rho_1)."""
    phi = logical_states()
    return np.stack([vec(np.outer(p, p.conj())) for p in phi], axis=1)


def operator_projector():
    """n x 4: column a + 2 b is vec(|a_L><b_L|)."""
    phi = logical_states()
    cols = [None] * 4
    for a in range(2):
        for b in range(2):
            cols[a + 2 * b] = vec(np.outer(phi[a], phi[b].conj()))
    return np.stack(cols, axis=1)


def embed(V):
    """8 x 8 unitary acting as the 2 x 2 V on span{phi_0, phi_1} (logical basis)
    and as the identity on its orthogonal complement."""
    B = np.stack(logical_states(), axis=1)          # 8 x 2
    return B @ V @ B.conj().T + (np.eye(8) - B @ B.conj().T)


def populations_target(V):
    """T_kl = |<k_L| V |l_L>|^2: Pi of the ideal gate for the population projector."""
    return np.abs(np.asarray(V)) ** 2 + 0j


def gate_target(V):
    """conj(V) (x) V in the operator basis a + 2 b: Pi of the ideal gate."""
    V = np.asarray(V, dtype=complex)
    return np.kron(V.conj(), V)


def projection(U, P):
    """Pi = P^dag U P (Eq. 16)."""
    return P.conj().T @ U @ P


def score(U, P, T, kind):
    """(value, seed M) with d value = Re Tr(M dU)."""
    Pi = projection(U, P)
    L = P.shape[1]
    if kind == "projected":
        D = Pi - T
        value = float(np.real(np.trace(D.conj().T @ D)))
        M = 2.0 * P @ D.conj().T @ P.conj().T
    elif kind == "linear":
        value = float(np.real(np.trace(T.conj().T @ Pi))) / L
        M = P @ T.conj().T @ P.conj().T / L
    else:
        raise ValueError(kind)
    return value, M
