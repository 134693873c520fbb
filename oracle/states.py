"""State-level reference for the accuracy study of the propagator (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper checks its Magnus propagator by evolving a random initial density
matrix with it and with an ODE solver, and scoring the two final states by the
Uhlmann fidelity as the number of slices grows (Sec. IV, Fig. 3). Here the ODE
solver is classical RK4 on the vectorised Lindblad equation d vec(rho)/dt =
L(u(t)) vec(rho) (Eq. 8 and 9) with a control given as a function of time, in
FP64.
"""
import numpy as np
import scipy.linalg as sla

from .liouville import vec, unvec


def rk4_state(system, u_fn, T, steps, rho0):
    """rho(T) by RK4 with `steps` equal steps; u_fn(t) -> control vector."""
    v = vec(np.asarray(rho0, dtype=complex))
    h = T / steps
    for k in range(steps):
        t = k * h
        L0 = system.liouv(u_fn(t))
        Lm = system.liouv(u_fn(t + 0.5 * h))
        L1 = system.liouv(u_fn(t + h))
        k1 = L0 @ v
        k2 = Lm @ (v + 0.5 * h * k1)
        k3 = Lm @ (v + 0.5 * h * k2)
        k4 = L1 @ (v + h * k3)
        v = v + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return unvec(v, system.d)


def uhlmann(rho, sigma):
    """F(rho, sigma) = (Tr sqrt(sqrt(rho) sigma sqrt(rho)))^2 (both Hermitian PSD)."""
    s = sla.sqrtm(np.asarray(rho, dtype=complex))
    m = sla.sqrtm(s @ np.asarray(sigma, dtype=complex) @ s)
    return float(np.real(np.trace(m)) ** 2)


def random_density(d, rng):
    """A full-rank random density matrix: G G^dag / Tr, G complex Ginibre."""
    G = rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))
    R = G @ G.conj().T
    return R / np.trace(R).real
