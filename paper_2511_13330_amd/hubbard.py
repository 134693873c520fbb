"""Operators of the Hubbard model of a linear quantum-dot array (paper Eq. 1),
as arrays for lmag_set_system.

Each dot has the states |0>, |up>, |down>, |up down> (local index
n_up + 2 n_down); dot 1 is the most significant tensor factor. The fermion
annihilators are local 4 x 4 operators dressed with the parity of the dots
before them (c_{i s} = P x ... x P x a_s x I x ... x I, P = (-1)^(n_up + n_down)),
and the down mode of a dot also carries the parity of its up mode, so that
|up down> = c+_up c+_down |0>.

Controls: the hopping terms sum_s (c+_{i s} c_{i+1, s} + h.c.) of the
neighbouring pairs (amplitudes t_{i,i+1}). Static terms, in this order: the
double-occupancy count sum_i n_i (n_i - 1) / 2 (coefficient U~), the dot
occupations n_i (coefficients V_i), the neighbour products sum_i n_i n_{i+1}
(coefficient U_C). Jump operators per dot: the spin flip |down><up| / sqrt(T1)
and the spin dephasing (n_up - n_down) / sqrt(T2).
"""
import numpy as np

_A_UP = np.zeros((4, 4), dtype=complex)
_A_UP[0, 1] = 1.0          # |up> -> |0>
_A_UP[2, 3] = 1.0          # |up down> -> |down>
_A_DN = np.zeros((4, 4), dtype=complex)
_A_DN[0, 2] = 1.0          # |down> -> |0>
_A_DN[1, 3] = -1.0         # |up down> -> -|up> (passes the up mode)
_PAR = np.diag([1.0, -1.0, -1.0, 1.0]).astype(complex)
_NUM = np.diag([0.0, 1.0, 1.0, 2.0]).astype(complex)
_FLIP = np.zeros((4, 4), dtype=complex)
_FLIP[2, 1] = 1.0          # |up> -> |down>
_SZ2 = np.diag([0.0, 1.0, -1.0, 0.0]).astype(complex)


def _site(ops, n_dots):
    """Tensor product over the dots of ops[i] (identity where None)."""
    m = np.ones((1, 1), dtype=complex)
    for i in range(n_dots):
        m = np.kron(m, ops[i] if ops[i] is not None else np.eye(4))
    return m


def _annihilator(i, spin, n_dots):
    ops = [_PAR] * i + [_A_UP if spin == 0 else _A_DN] + [None] * (n_dots - i - 1)
    return _site(ops, n_dots)


def _local(op, i, n_dots):
    return _site([op if k == i else None for k in range(n_dots)], n_dots)


def hubbard_operators(n_dots, T1=np.inf, T2=np.inf):
    """(H_static, H_ctrl, L_jump) as complex arrays [k][d][d], d = 4^n_dots."""
    d = 4 ** n_dots
    ctrl = []
    for i in range(n_dots - 1):
        h = np.zeros((d, d), dtype=complex)
        for s in (0, 1):
            a, b = _annihilator(i, s, n_dots), _annihilator(i + 1, s, n_dots)
            h += a.conj().T @ b + b.conj().T @ a
        ctrl.append(h)
    n = [_local(_NUM, i, n_dots) for i in range(n_dots)]
    double = sum(_local(np.diag([0.0, 0.0, 0.0, 1.0]).astype(complex), i, n_dots)
                 for i in range(n_dots))
    static = [double] + n + [sum((n[i] @ n[i + 1] for i in range(n_dots - 1)),
                                 np.zeros((d, d), dtype=complex))]
    jumps = []
    for i in range(n_dots):
        if np.isfinite(T1):
            jumps.append(_local(_FLIP, i, n_dots) / np.sqrt(T1))
        if np.isfinite(T2):
            jumps.append(_local(_SZ2, i, n_dots) / np.sqrt(T2))

    def arr(lst):
        return np.array(lst, dtype=complex).reshape(len(lst), d, d)

    return arr(static), arr(ctrl), arr(jumps)


def hubbard_system(n_dots, T1=np.inf, T2=np.inf, **kw):
    """A System for the dot array: static coefficients per item are
    (U~, V_1, ..., V_N, U_C), controls the hopping amplitudes."""
    from .system import System
    hs, hc, lj = hubbard_operators(n_dots, T1, T2)
    return System(hs, hc, lj, **kw)
