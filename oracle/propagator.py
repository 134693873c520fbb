"""Propagator, fidelity and gradient (oracle), Eq. 9-15.

U = S_N ... S_1 with S_n = exp(Omega_n), later slices on the left (Eq. 15),
evaluated as a plain sequential left multiplication.

Process fidelity: F = Re Tr(S_T^dag U) / d^2 with S_T = conj(U_T) (x) U_T, the
column-stacking superoperator of the target unitary.

Gradient (exact adjoint of the discretised method): with prefixes
X_n = S_n ... S_1 (X_0 = I) and suffixes Y_n = S_T^dag S_N ... S_{n+1}
(Y_N = S_T^dag), F = Re Tr(S_n M_n) / d^2 with M_n = X_{n-1} Y_n, so

  dF = Re Tr(L(Omega_n, dOmega_n) M_n) / d^2 = Re Tr(K_n dOmega_n) / d^2,
  K_n = L(Omega_n, M_n)

by the adjoint identity Tr(M L(A, E)) = Tr(L(A, M) E). dOmega_n / du is formed
explicitly from the node matrices (no basis expansion).
"""
import numpy as np

from .model import exchange_terms, zeeman_terms, jump_ops, hamiltonian
from .liouville import liouvillian, lift_hamiltonian
from .magnus import (node_controls, gl2_nodes, slice_omega, SQ3, node_controls3, gl3_nodes,
                     order6_terms, comm, SQ15)
from .expm import expm_taylor, frechet_block


class System:
    """Spin chain with exchange controls, Zeeman fields b and per-coupling
    control scales eps (quasi-static J noise; 1 when absent)."""

    def __init__(self, n_spins, B, T1=np.inf, T2=np.inf, eps=None):
        self.n_spins = n_spins
        self.d = 2 ** n_spins
        self.n_ctrl = n_spins - 1
        self.B = np.asarray(B, dtype=float)
        self.eps = np.ones(self.n_ctrl) if eps is None else np.asarray(eps, float)
        self.Hc = exchange_terms(n_spins)
        self.Ls = jump_ops(n_spins, T1, T2)

    @classmethod
    def from_cfg(cls, cfg, dissipative=True, eps=None, dB=None):
        B = np.asarray(cfg["B"], float)
        if dB is not None:
            B = B + np.asarray(dB, float)
        T1, T2 = (cfg["T1"], cfg["T2"]) if dissipative else (np.inf, np.inf)
        return cls(cfg["n_spins"], B, T1, T2, eps)

    def H(self, u):
        return hamiltonian(u, self.B, self.eps, self.n_spins)

    def liouv(self, u):
        return liouvillian(self.H(u), self.Ls)

    def ctrl_generator(self, c):
        """d L / d (eps_c u_c): the lifted control term of Eq. 8."""
        return lift_hamiltonian(self.Hc[c])

    def omegas(self, amps, dt, order, hold):
        return [slice_omega(self.liouv, amps, n, dt, order, hold)
                for n in range(amps.shape[0])]

    def domega(self, amps, n, dt, order, hold):
        """dOmega_n / d u_{m,c} as a dict {(m, c): matrix}."""
        if order == 6:
            return self._domega6(amps, n, dt, hold)
        N = amps.shape[0]
        ua, ub = node_controls(amps, n, hold)
        A1, A2 = self.liouv(ua), self.liouv(ub)
        if hold == "zoh":
            w = {n: (1.0, 1.0)}
        else:
            l1, l2 = gl2_nodes()
            if n + 1 < N:
                w = {n: (1.0 - l1, 1.0 - l2), n + 1: (l1, l2)}
            else:
                w = {n: (1.0, 1.0)}
        out = {}
        for m, (w1, w2) in w.items():
            for c in range(self.n_ctrl):
                G = self.eps[c] * self.ctrl_generator(c)
                d1, d2 = w1 * G, w2 * G
                dom = 0.5 * dt * (d1 + d2)
                if order == 2:
                    k = SQ3 * dt * dt / 12.0
                    dom = dom + k * ((d2 @ A1 - A1 @ d2) + (A2 @ d1 - d1 @ A2))
                out[(m, c)] = dom
        return out


def _domega6(self, amps, n, dt, hold):
    """dOmega_n / d u_{m,c} of the sixth-order scheme by the product rule on
    its commutators, with dB_k / d u_{m,c} = w_k(m) eps_c G_c (G_c the control
    generator, w_k(m) the weight of row m in the control value at node k)."""
    N = amps.shape[0]
    u1, u2, u3 = node_controls3(amps, n, hold)
    Bs = [self.liouv(u) for u in (u1, u2, u3)]
    a1, a2, a3, C1, W, C2, X, Y = order6_terms(*Bs, dt)
    lam = gl3_nodes()
    if hold == "zoh" or n + 1 >= N:
        w = {n: (1.0, 1.0, 1.0)}
    else:
        w = {n: tuple(1.0 - l for l in lam), n + 1: lam}
    out = {}
    for m, wk in w.items():
        for c in range(self.n_ctrl):
            G = self.eps[c] * self.ctrl_generator(c)
            dB1, dB2, dB3 = (wk[k] * G for k in range(3))
            da1 = dt * dB2
            da2 = (SQ15 * dt / 3.0) * (dB3 - dB1)
            da3 = (10.0 * dt / 3.0) * (dB3 - 2.0 * dB2 + dB1)
            dC1 = comm(da1, a2) + comm(a1, da2)
            dW = 2.0 * da3 + dC1
            dC2 = -(comm(da1, W) + comm(a1, dW)) / 60.0
            dX = -20.0 * da1 - da3 + dC1
            dY = da2 + dC2
            out[(m, c)] = da1 + da3 / 12.0 + (comm(dX, Y) + comm(X, dY)) / 240.0
    return out


System._domega6 = _domega6


def slice_products(omegas):
    return [expm_taylor(om) for om in omegas]


def propagate(omegas):
    """U = S_N ... S_1 by sequential left multiplication."""
    n = omegas[0].shape[0]
    U = np.eye(n, dtype=complex)
    for om in omegas:
        U = expm_taylor(om) @ U
    return U


def superop_of_unitary(V):
    """Column-stacking superoperator of rho -> V rho V^dag."""
    return np.kron(V.conj(), V)


def fidelity(U, U_target):
    """(Re, Im) of Tr(S_T^dag U) / d^2."""
    d = U_target.shape[0]
    ST = superop_of_unitary(U_target)
    z = np.trace(ST.conj().T @ U) / (d * d)
    return float(z.real), float(z.imag)


def grad_adjoint(system, amps, dt, order, hold, U_target):
    """(F, dF/du) with dF/du shaped like amps."""
    amps = np.asarray(amps, dtype=float)
    N = amps.shape[0]
    d = system.d
    oms = system.omegas(amps, dt, order, hold)
    S = slice_products(oms)
    n = oms[0].shape[0]
    X = [np.eye(n, dtype=complex)]
    for k in range(N):
        X.append(S[k] @ X[-1])
    ST = superop_of_unitary(U_target)
    F = float(np.real(np.trace(ST.conj().T @ X[N]))) / (d * d)
    Y = ST.conj().T
    grad = np.zeros_like(amps)
    for k in range(N - 1, -1, -1):
        # Y currently holds Y_{k+1} in the 1-based notation above (slice k is
        # the (k+1)-th); M = X_k Y
        M = X[k] @ Y
        K = frechet_block(oms[k], M)
        for (m, c), dom in system.domega(amps, k, dt, order, hold).items():
            grad[m, c] += float(np.real(np.trace(K @ dom))) / (d * d)
        Y = Y @ S[k]
    return F, grad


def grad_adjoint_seed(system, amps, dt, order, hold, seed_fn):
    """(s, ds/du) for a score s(U) of the total propagator: seed_fn(U) returns
    (s, M) with ds = Re Tr(M dU); the adjoint runs as in grad_adjoint with the
    suffix started from M instead of S_T^dag / d^2."""
    amps = np.asarray(amps, dtype=float)
    N = amps.shape[0]
    oms = system.omegas(amps, dt, order, hold)
    S = slice_products(oms)
    n = oms[0].shape[0]
    X = [np.eye(n, dtype=complex)]
    for k in range(N):
        X.append(S[k] @ X[-1])
    value, Y = seed_fn(X[N])
    grad = np.zeros_like(amps)
    for k in range(N - 1, -1, -1):
        M = X[k] @ Y
        K = frechet_block(oms[k], M)
        for (m, c), dom in system.domega(amps, k, dt, order, hold).items():
            grad[m, c] += float(np.real(np.trace(K @ dom)))
        Y = Y @ S[k]
    return value, grad


def grad_fd(system, amps, dt, order, hold, U_target, coords, h=1e-4):
    """Central differences of F at flat indices coords of amps (float64)."""
    amps = np.asarray(amps, dtype=float)
    out = np.zeros(len(coords))
    for i, flat in enumerate(coords):
        m, c = divmod(int(flat), amps.shape[1])
        up = amps.copy(); up[m, c] += h
        dn = amps.copy(); dn[m, c] -= h
        fu = fidelity(propagate(system.omegas(up, dt, order, hold)), U_target)[0]
        fd = fidelity(propagate(system.omegas(dn, dt, order, hold)), U_target)[0]
        out[i] = (fu - fd) / (2.0 * h)
    return out


def rk4_propagator(system, amps, dt, hold, steps_per_slice):
    """Classical RK4 on dU/dt = L(t) U (Eq. 9, U(0) = 1) with the same control
    interpolation as the slices; every RK4 step lies inside one slice."""
    amps = np.asarray(amps, dtype=float)
    N = amps.shape[0]
    n = system.d ** 2
    U = np.eye(n, dtype=complex)
    hs = dt / steps_per_slice

    def u_at(k, frac):
        if hold == "zoh":
            return amps[k]
        u1 = amps[k + 1] if k + 1 < N else amps[k]
        return amps[k] + frac * (u1 - amps[k])

    for k in range(N):
        for j in range(steps_per_slice):
            f0 = j / steps_per_slice
            fm = (j + 0.5) / steps_per_slice
            f1 = (j + 1.0) / steps_per_slice
            L0 = system.liouv(u_at(k, f0))
            Lm = system.liouv(u_at(k, fm))
            L1 = system.liouv(u_at(k, f1))
            k1 = L0 @ U
            k2 = Lm @ (U + 0.5 * hs * k1)
            k3 = Lm @ (U + 0.5 * hs * k2)
            k4 = L1 @ (U + hs * k3)
            U = U + (hs / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return U


def grad_adjoint_at(system, amps, dt, order, hold, U_target, slices):
    """dF/du restricted to the rows in `slices` (exact adjoint). The prefix and
    suffix chains run over all slices; the Frechet derivative K_k is formed only
    for the slices whose Omega depends on a requested row (k and k-1 for FOH)."""
    amps = np.asarray(amps, dtype=float)
    N = amps.shape[0]
    d = system.d
    want = set(int(s) for s in slices)
    need = set()
    for s in want:
        need.add(s)
        if hold == "foh" and s > 0:
            need.add(s - 1)
    oms = system.omegas(amps, dt, order, hold)
    S = slice_products(oms)
    n = oms[0].shape[0]
    X = [np.eye(n, dtype=complex)]
    for k in range(N):
        X.append(S[k] @ X[-1])
    ST = superop_of_unitary(U_target)
    F = float(np.real(np.trace(ST.conj().T @ X[N]))) / (d * d)
    Y = ST.conj().T
    out = {s: np.zeros(amps.shape[1]) for s in want}
    for k in range(N - 1, -1, -1):
        if k in need:
            K = frechet_block(oms[k], X[k] @ Y)
            for (m, c), dom in system.domega(amps, k, dt, order, hold).items():
                if m in want:
                    out[m][c] += float(np.real(np.trace(K @ dom))) / (d * d)
        Y = Y @ S[k]
    return F, out


def grad_adjoint_seed_at(system, amps, dt, order, hold, seed_fn, slices):
    """grad_adjoint_seed restricted to the rows in `slices` (as grad_adjoint_at)."""
    amps = np.asarray(amps, dtype=float)
    N = amps.shape[0]
    want = set(int(s) for s in slices)
    need = set()
    for s in want:
        need.add(s)
        if hold == "foh" and s > 0:
            need.add(s - 1)
    oms = system.omegas(amps, dt, order, hold)
    S = slice_products(oms)
    n = oms[0].shape[0]
    X = [np.eye(n, dtype=complex)]
    for k in range(N):
        X.append(S[k] @ X[-1])
    value, Y = seed_fn(X[N])
    out = {s: np.zeros(amps.shape[1]) for s in want}
    for k in range(N - 1, -1, -1):
        if k in need:
            K = frechet_block(oms[k], X[k] @ Y)
            for (m, c), dom in system.domega(amps, k, dt, order, hold).items():
                if m in want:
                    out[m][c] += float(np.real(np.trace(K @ dom)))
        Y = Y @ S[k]
    return value, out


def grad_fd_cached(system, amps, dt, order, hold, U_target, coords, h=1e-4):
    """Central differences of F, like grad_fd, for long pulses: a change of row
    m only changes the slices m-1 and m (FOH) or m (ZOH), so F(u +- h e) is the
    trace of (suffix) (changed slices) (prefix) with the unchanged prefix and
    suffix products of Eq. 15 computed once."""
    amps = np.asarray(amps, dtype=float)
    N = amps.shape[0]
    d = system.d
    oms = system.omegas(amps, dt, order, hold)
    S = slice_products(oms)
    n = oms[0].shape[0]
    X = [np.eye(n, dtype=complex)]
    for k in range(N):
        X.append(S[k] @ X[-1])
    ST = superop_of_unitary(U_target)
    Ys = [None] * (N + 1)
    Y = ST.conj().T
    Ys[N] = Y
    for k in range(N - 1, -1, -1):
        Y = Y @ S[k]
        Ys[k] = Y          # Ys[k] = S_T^dag S_{N-1} ... S_k
    out = np.zeros(len(coords))
    for i, flat in enumerate(coords):
        m, c = divmod(int(flat), amps.shape[1])
        lo = m - 1 if (hold == "foh" and m > 0) else m
        vals = []
        for sgn in (1.0, -1.0):
            a2 = amps.copy()
            a2[m, c] += sgn * h
            mid = np.eye(n, dtype=complex)
            for k in range(lo, m + 1):
                mid = expm_taylor(slice_omega(system.liouv, a2, k, dt, order, hold)) @ mid
            vals.append(float(np.real(np.trace(Ys[m + 1] @ mid @ X[lo]))) / (d * d))
        out[i] = (vals[0] - vals[1]) / (2.0 * h)
    return out
