"""Spin-chain operators (oracle).

Conventions: spin 1 is the most significant Kronecker factor; |0> = up with
sigma_z = +1; sigma_minus = [[0, 0], [1, 0]] maps up to down; S_i = sigma_i / 2.
The Hamiltonian follows the three-electron exchange model: exchange couplings
S_c . S_{c+1} between neighbours as the controls (the paper's tunable inter-dot
terms, Sec. II-A) and static Zeeman terms (B_i / 2) sigma_z_i. Jump operators are
op / sqrt(T) as in the paper's Lindblad background (Sec. II-B, after Eq. 6):
sigma_minus_i / sqrt(T1) and sigma_z_i / sqrt(T2) for every spin.
"""
import numpy as np


def pauli(name):
    if name == "x":
        return np.array([[0, 1], [1, 0]], dtype=complex)
    if name == "y":
        return np.array([[0, -1j], [1j, 0]], dtype=complex)
    if name == "z":
        return np.array([[1, 0], [0, -1]], dtype=complex)
    if name == "m":  # sigma_minus: up (index 0) -> down (index 1)
        return np.array([[0, 0], [1, 0]], dtype=complex)
    if name == "i":
        return np.eye(2, dtype=complex)
    raise ValueError(name)


def spin_op(op, i, n_spins):
    """op acting on spin i (0-based) of an n-spin chain, identity elsewhere."""
    out = np.array([[1.0 + 0j]])
    for k in range(n_spins):
        out = np.kron(out, op if k == i else np.eye(2, dtype=complex))
    return out


def exchange_terms(n_spins):
    """H_c = S_c . S_{c+1} = (1/4) sum_a sigma^a_c sigma^a_{c+1}, c = 0..n-2."""
    terms = []
    for c in range(n_spins - 1):
        h = np.zeros((2 ** n_spins,) * 2, dtype=complex)
        for a in "xyz":
            h += spin_op(pauli(a), c, n_spins) @ spin_op(pauli(a), c + 1, n_spins)
        terms.append(h / 4.0)
    return terms


def zeeman_terms(n_spins):
    """Z_i = sigma_z_i / 2."""
    return [spin_op(pauli("z"), i, n_spins) / 2.0 for i in range(n_spins)]


def jump_ops(n_spins, T1, T2):
    """sigma_minus_i / sqrt(T1) and sigma_z_i / sqrt(T2) per spin (skipped when
    the time is infinite)."""
    ops = []
    for i in range(n_spins):
        if np.isfinite(T1):
            ops.append(spin_op(pauli("m"), i, n_spins) / np.sqrt(T1))
        if np.isfinite(T2):
            ops.append(spin_op(pauli("z"), i, n_spins) / np.sqrt(T2))
    return ops


def hamiltonian(u, b, eps, n_spins):
    """H = sum_c eps_c u_c S_c.S_{c+1} + sum_i (b_i / 2) sigma_z_i."""
    H = np.zeros((2 ** n_spins,) * 2, dtype=complex)
    for c, hc in enumerate(exchange_terms(n_spins)):
        H += eps[c] * u[c] * hc
    for i, zi in enumerate(zeeman_terms(n_spins)):
        H += b[i] * zi
    return H
