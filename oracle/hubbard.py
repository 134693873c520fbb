"""Hubbard model of a linear array of quantum dots (oracle), Eq. 1.

H = sum_i [ (U~/2) n_i (n_i - 1) + V_i n_i ] + U_C sum_<ij> n_i n_j
    + sum_<ij> t_ij sum_sigma ( c+_{i sigma} c_{j sigma} + c+_{j sigma} c_{i sigma} )

over nearest-neighbour pairs <ij> = (i, i+1) of the array. Every dot has the
four states |0>, |up>, |down>, |up down> (local index n_up + 2 n_down); dot 1 is
the most significant factor of the 4^N product basis. The 2N fermionic modes
are ordered (1 up, 1 down, 2 up, 2 down, ...). The annihilator c_k is built
entry by entry from the occupation bits of the basis states: it empties mode k
with the sign (-1)^(number of occupied modes before k) (Jordan-Wigner), so that
|up down> = c+_up c+_down |0> on every dot.

Controls are the hopping amplitudes t_ij (one per neighbour pair). The static
terms are, in this order, sum_i n_i (n_i - 1) / 2 (coefficient U~), n_i for
every dot (coefficient V_i) and sum_<ij> n_i n_j (coefficient U_C). Jump
operators per dot, in the spirit of the paper's op/sqrt(T) (Sec. II-B): the
spin flip c+_{i down} c_{i up} / sqrt(T1) (relaxation, keeps the electron
number) and (n_{i up} - n_{i down}) / sqrt(T2) (dephasing of the dot's spin).
"""
import numpy as np

from .propagator import System
from .hilbert import HilbertSystem


def _occ(state, n_dots):
    """Occupation bits of the 2 n_dots modes, in mode order."""
    bits = []
    for i in range(n_dots):
        loc = (state >> (2 * (n_dots - 1 - i))) & 3
        bits += [loc & 1, (loc >> 1) & 1]
    return bits


def _index(bits, n_dots):
    s = 0
    for i in range(n_dots):
        s = 4 * s + bits[2 * i] + 2 * bits[2 * i + 1]
    return s


def annihilators(n_dots):
    """c_k for every mode k = 2 i + sigma (sigma 0 = up, 1 = down)."""
    dim = 4 ** n_dots
    ops = []
    for k in range(2 * n_dots):
        c = np.zeros((dim, dim), dtype=complex)
        for s in range(dim):
            bits = _occ(s, n_dots)
            if not bits[k]:
                continue
            sign = (-1) ** sum(bits[:k])
            nb = list(bits)
            nb[k] = 0
            c[_index(nb, n_dots), s] = sign
        ops.append(c)
    return ops


def number_ops(n_dots):
    c = annihilators(n_dots)
    n_mode = [ck.conj().T @ ck for ck in c]
    return [n_mode[2 * i] + n_mode[2 * i + 1] for i in range(n_dots)], n_mode


def pairs(n_dots):
    return [(i, i + 1) for i in range(n_dots - 1)]


def hopping_terms(n_dots):
    """sum_sigma (c+_{i s} c_{j s} + c+_{j s} c_{i s}) for every neighbour pair."""
    c = annihilators(n_dots)
    out = []
    for i, j in pairs(n_dots):
        h = np.zeros_like(c[0])
        for s in (0, 1):
            a, b = c[2 * i + s], c[2 * j + s]
            h += a.conj().T @ b + b.conj().T @ a
        out.append(h)
    return out


def static_terms(n_dots):
    """[sum_i n_i (n_i - 1) / 2, n_1, ..., n_N, sum_<ij> n_i n_j]."""
    n, _ = number_ops(n_dots)
    eye = np.eye(4 ** n_dots, dtype=complex)
    onsite = sum(0.5 * ni @ (ni - eye) for ni in n)
    coulomb = sum((n[i] @ n[j] for i, j in pairs(n_dots)), np.zeros_like(eye))
    return [onsite] + list(n) + [coulomb]


def jump_ops(n_dots, T1, T2):
    c = annihilators(n_dots)
    _, nm = number_ops(n_dots)
    ops = []
    for i in range(n_dots):
        up, dn = 2 * i, 2 * i + 1
        if np.isfinite(T1):
            ops.append(c[dn].conj().T @ c[up] / np.sqrt(T1))
        if np.isfinite(T2):
            ops.append((nm[up] - nm[dn]) / np.sqrt(T2))
    return ops


def total_number(n_dots):
    n, _ = number_ops(n_dots)
    return sum(n)


def total_sz(n_dots):
    _, nm = number_ops(n_dots)
    return 0.5 * sum(nm[2 * i] - nm[2 * i + 1] for i in range(n_dots))


def hamiltonian(t, coef, n_dots):
    """H of Eq. 1 for hopping amplitudes t [pairs] and static coefficients
    coef = (U~, V_1..V_N, U_C)."""
    H = sum(ti * h for ti, h in zip(t, hopping_terms(n_dots)))
    return H + sum(ci * s for ci, s in zip(coef, static_terms(n_dots)))


class HubbardSystem(System):
    """The Hubbard array as an oracle system: controls t_ij (scaled by eps),
    static coefficients (U~, V_i, U_C), the dots' jump operators."""

    def __init__(self, n_dots, coef, T1=np.inf, T2=np.inf, eps=None):
        self.n_dots = n_dots
        self.d = 4 ** n_dots
        self.n_ctrl = n_dots - 1
        self.B = np.asarray(coef, dtype=float)
        self.eps = np.ones(self.n_ctrl) if eps is None else np.asarray(eps, float)
        self.Hc = hopping_terms(n_dots)
        self.Hs = static_terms(n_dots)
        self.Ls = jump_ops(n_dots, T1, T2)

    def H(self, u):
        H = np.zeros((self.d, self.d), dtype=complex)
        for c, hc in enumerate(self.Hc):
            H += self.eps[c] * u[c] * hc
        for i, hs in enumerate(self.Hs):
            H += self.B[i] * hs
        return H


class HubbardHilbert(HubbardSystem):
    """The closed Hubbard array with the Hilbert-space generator -i H(t)
    (the closed-system reduction of the hilbert module)."""

    def __init__(self, n_dots, coef, eps=None):
        super().__init__(n_dots, coef, np.inf, np.inf, eps)

    liouv = HilbertSystem.liouv
    ctrl_generator = HilbertSystem.ctrl_generator
