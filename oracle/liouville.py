"""Superoperator form of the Lindblad equation (oracle), Eq. 7-8.

Column-stacking vectorisation: vec(rho)[i + d*j] = rho[i, j], so that
vec(A X B) = (B^T (x) A) vec(X). With it Eq. 8 reads

  L = -i (I (x) H - H^T (x) I)
      + sum_k [ conj(L_k) (x) L_k - 1/2 I (x) L_k^dag L_k - 1/2 (L_k^dag L_k)^T (x) I ].
"""
import numpy as np


def vec(rho):
    """Column-stacking vectorisation."""
    return np.asarray(rho).T.reshape(-1)


def unvec(v, d):
    return np.asarray(v).reshape(d, d).T


def lift_hamiltonian(H):
    """-i (I (x) H - H^T (x) I), the Hamiltonian part of Eq. 8."""
    d = H.shape[0]
    I = np.eye(d, dtype=complex)
    return -1j * (np.kron(I, H) - np.kron(H.T, I))


def liouvillian(H, Ls):
    """Eq. 8 for a Hamiltonian H and a list of jump operators Ls."""
    d = H.shape[0]
    I = np.eye(d, dtype=complex)
    out = lift_hamiltonian(H)
    for L in Ls:
        LdL = L.conj().T @ L
        out = out + np.kron(L.conj(), L) - 0.5 * np.kron(I, LdL) \
            - 0.5 * np.kron(LdL.T, I)
    return out
