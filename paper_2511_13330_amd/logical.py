"""Logical qubit of the three-spin exchange-only encoding (Sec. II-A, Eq. 2
and 3) and the projectors of the logical-subspace scores (Sec. III-C,
Eq. 16-17), as host arrays for System.logical_score_and_grad.

Basis of the 8-dimensional spin space: spin 1 is the most significant factor
and |up> has index 0, so |uud> = 1, |udu> = 2, |duu> = 4. Superoperators act on
column-stacked density matrices, vec(rho)[i + 8 j] = rho[i][j].
"""
import numpy as np

UUD, UDU, DUU = 1, 2, 4


def states():
    """|0_L> = (|uud> - |duu>) / sqrt 2, |1_L> = (2 |udu> - |uud> - |duu>) / sqrt 6."""
    z = np.zeros((2, 8), dtype=np.complex128)
    z[0, UUD], z[0, DUU] = 1 / np.sqrt(2), -1 / np.sqrt(2)
    z[1, UDU], z[1, UUD], z[1, DUU] = 2 / np.sqrt(6), -1 / np.sqrt(6), -1 / np.sqrt(6)
    return z


def _colvec(M):
    return np.asarray(M).reshape(-1, order="F")


def population_projector():
    """[64, 2]: vec(rho_0), vec(rho_1) (the projection of Eq. 16)."""
    z = states()
    return np.stack([_colvec(np.outer(z[k], z[k].conj())) for k in range(2)], axis=1)


def operator_projector():
    """[64, 4]: column a + 2 b is vec(|a_L><b_L|) (the whole logical channel)."""
    z = states()
    cols = {a + 2 * b: _colvec(np.outer(z[a], z[b].conj())) for a in range(2) for b in range(2)}
    return np.stack([cols[k] for k in range(4)], axis=1)


def population_target(V):
    """Pi of the ideal logical gate V (2 x 2) under the population projector."""
    return np.abs(np.asarray(V, dtype=np.complex128)) ** 2 + 0j


def gate_target(V):
    """conj(V) (x) V: Pi of the ideal gate V under the operator projector."""
    V = np.asarray(V, dtype=np.complex128)
    return np.kron(V.conj(), V)
