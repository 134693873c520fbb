"""Closed systems in Hilbert space, and the action of a slice exponential on a
few vectors (oracle) -- references for superoperators too large for the dense
FP64 path.

Closed-system reduction. Without jump operators the generator of Eq. 8 is
Lift(H) = -i (I (x) H - H^T (x) I), and Lift(H) vec(rho) = vec(a rho - rho a)
with a = -i H: the lift is ad_a, which is linear in a and a Lie-algebra
homomorphism ([ad_a, ad_b] = ad_[a,b]). The Magnus exponent of a slice (Eq. 13
and the Gauss-Legendre commutator term) built from L(t) = ad_{a(t)} is therefore
ad of the exponent omega_n built by the same rule from a(t) = -i H(t), and
exp(ad_omega) rho = V rho V^dag with V = exp(omega) (omega is anti-Hermitian).
So the superoperator propagator of a closed system is conj(V) (x) V with
V = V_N ... V_1 (Eq. 15 in Hilbert space, d x d matrices only), and the process
fidelity against S_T = conj(U_T) (x) U_T is |Tr(U_T^dag V)|^2 / d^2.

Action of a slice exponential. exp(Omega_n) X for a block X of a few columns,
with Omega_n applied through its definition, (h/2)(A_1 + A_2) Y plus
(sqrt(3) h^2 / 12)(A_2 (A_1 Y) - A_1 (A_2 Y)), so that no n x n product is
formed; the exponential is the Taylor series of exp(Omega / 2^s) applied 2^s
times, with s from a bound on ||Omega||_1.
"""
import numpy as np

from .magnus import node_controls, SQ3
from .propagator import System, propagate, grad_adjoint_seed, grad_adjoint_seed_at


class HilbertSystem(System):
    """The spin chain of System without jump operators, with the Hilbert-space
    generator a(t) = -i H(t) in place of its lift."""

    def __init__(self, n_spins, B, eps=None):
        super().__init__(n_spins, B, np.inf, np.inf, eps)

    @classmethod
    def from_cfg(cls, cfg, eps=None, dB=None):
        B = np.asarray(cfg["B"], float)
        if dB is not None:
            B = B + np.asarray(dB, float)
        return cls(cfg["n_spins"], B, eps)

    def liouv(self, u):
        return -1j * self.H(u)

    def ctrl_generator(self, c):
        return -1j * self.Hc[c]


def unitary(hsys, amps, dt, order, hold):
    """V = V_N ... V_1 with V_n = exp(omega_n)."""
    return propagate(hsys.omegas(np.asarray(amps, float), dt, order, hold))


def superop(V):
    """conj(V) (x) V: the column-stacking superoperator of rho -> V rho V^dag."""
    return np.kron(V.conj(), V)


def fidelity(V, U_target):
    """|Tr(U_T^dag V)|^2 / d^2, the process fidelity of the channel of V."""
    d = V.shape[0]
    t = np.trace(U_target.conj().T @ V)
    return float(abs(t) ** 2) / (d * d)


def _seed(U_target):
    d = U_target.shape[0]

    def seed(V):
        # F = |t|^2 / d^2, t = Tr(U_T^dag V): dF = Re Tr((2 conj(t) / d^2) U_T^dag dV)
        t = np.trace(U_target.conj().T @ V)
        return float(abs(t) ** 2) / (d * d), (2.0 * np.conj(t) / (d * d)) * U_target.conj().T
    return seed


def grad(hsys, amps, dt, order, hold, U_target):
    """(F, dF/du) of the closed system: the adjoint of grad_adjoint_seed with
    the Hilbert-space slices and the fidelity's seed."""
    return grad_adjoint_seed(hsys, amps, dt, order, hold, _seed(U_target))


def grad_at(hsys, amps, dt, order, hold, U_target, slices):
    return grad_adjoint_seed_at(hsys, amps, dt, order, hold, _seed(U_target), slices)


def grad_fd(hsys, amps, dt, order, hold, U_target, coords, h=1e-4):
    """Central differences of the closed-system fidelity at flat indices coords."""
    amps = np.asarray(amps, float)
    out = np.zeros(len(coords))
    for i, flat in enumerate(coords):
        m, c = divmod(int(flat), amps.shape[1])
        up = amps.copy(); up[m, c] += h
        dn = amps.copy(); dn[m, c] -= h
        out[i] = (fidelity(unitary(hsys, up, dt, order, hold), U_target)
                  - fidelity(unitary(hsys, dn, dt, order, hold), U_target)) / (2.0 * h)
    return out


def _norm1(A):
    return float(np.max(np.sum(np.abs(A), axis=0)))


def omega_action(system, amps, n, dt, order, hold):
    """(apply, bound): apply(Y) = Omega_n Y from the node matrices, and an upper
    bound of ||Omega_n||_1 from their norms."""
    ua, ub = node_controls(np.asarray(amps, float), n, hold)
    A1, A2 = system.liouv(ua), system.liouv(ub)
    k = SQ3 * dt * dt / 12.0
    n1, n2 = _norm1(A1), _norm1(A2)

    def apply(Y):
        out = 0.5 * dt * (A1 @ Y + A2 @ Y)
        if order == 2:
            out = out + k * (A2 @ (A1 @ Y) - A1 @ (A2 @ Y))
        return out

    bound = 0.5 * dt * (n1 + n2) + (2.0 * k * n1 * n2 if order == 2 else 0.0)
    return apply, bound


def expm_action(apply, bound, X):
    """exp(A) X for A given by apply(Y) = A Y and bound >= ||A||_1: the Taylor
    series of exp(A / 2^s), ||A / 2^s||_1 <= 1/2, applied 2^s times; terms are
    added until one is below 1e-18 of the partial sum (max column 1-norm)."""
    X = np.asarray(X, dtype=complex)
    s = 0
    if bound > 0.5:
        s = int(np.ceil(np.log2(bound / 0.5)))
    scale = 2.0 ** (-s)
    for _ in range(2 ** s):
        total = X.copy()
        term = X.copy()
        for k in range(1, 80):
            term = scale * apply(term) / k
            total = total + term
            if _norm1(term) <= 1e-18 * _norm1(total):
                break
        X = total
    return X


def propagator_columns(system, amps, dt, order, hold, cols):
    """Columns cols of U = S_N ... S_1: the slice exponentials applied in turn to
    the unit vectors e_j."""
    amps = np.asarray(amps, float)
    n = system.d ** 2
    X = np.zeros((n, len(cols)), dtype=complex)
    X[np.asarray(cols), np.arange(len(cols))] = 1.0
    for k in range(amps.shape[0]):
        apply, bound = omega_action(system, amps, k, dt, order, hold)
        X = expm_action(apply, bound, X)
    return X
