"""Operators of the exchange-coupled spin chain, as arrays for lmag_set_system.

Spin 1 is the most significant tensor factor; |0> is spin up (sigma_z = +1);
sigma_minus maps up to down. Controls are the exchange terms S_c . S_{c+1}
(the tunable inter-dot couplings), static terms the Zeeman terms sigma_z_i / 2,
jump operators sigma_minus_i / sqrt(T1) and sigma_z_i / sqrt(T2) per spin
(the op / sqrt(T) form of the paper's Lindblad background).
"""
import numpy as np

_SX = np.array([[0, 1], [1, 0]], dtype=complex)
_SY = np.array([[0, -1j], [1j, 0]], dtype=complex)
_SZ = np.array([[1, 0], [0, -1]], dtype=complex)
_SM = np.array([[0, 0], [1, 0]], dtype=complex)


def _on(op, i, n):
    m = np.ones((1, 1), dtype=complex)
    for k in range(n):
        m = np.kron(m, op if k == i else np.eye(2))
    return m


def chain_operators(n_spins, T1=np.inf, T2=np.inf):
    """(H_static, H_ctrl, L_jump) as complex arrays [k][d][d]."""
    d = 2 ** n_spins
    ctrl = []
    for c in range(n_spins - 1):
        h = sum(_on(p, c, n_spins) @ _on(p, c + 1, n_spins) for p in (_SX, _SY, _SZ))
        ctrl.append(h / 4.0)
    static = [_on(_SZ, i, n_spins) / 2.0 for i in range(n_spins)]
    jumps = []
    for i in range(n_spins):
        if np.isfinite(T1):
            jumps.append(_on(_SM, i, n_spins) / np.sqrt(T1))
        if np.isfinite(T2):
            jumps.append(_on(_SZ, i, n_spins) / np.sqrt(T2))

    def arr(lst):
        return np.array(lst, dtype=complex).reshape(len(lst), d, d)

    return arr(static), arr(ctrl), arr(jumps)
