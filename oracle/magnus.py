"""Magnus slice exponents (oracle), Eq. 13 and its second-order extension.

Within slice n = [t_n, t_n + h] the controls are either held constant (ZOH,
u(t) = u_n) or interpolated linearly (FOH, u(t) = u_n + (t - t_n)/h (u_{n+1} - u_n),
with u_N taken equal to u_{N-1} for the last slice). The two Gauss-Legendre
nodes are tau_{1,2} = t_n + (1/2 -/+ sqrt(3)/6) h and A_k = L(tau_k).

* First order (Eq. 13): Omega_n = int_slice L(t) dt. L is affine in u and u is
  at most linear in t, so the two-point rule (h/2)(A_1 + A_2) is this integral
  exactly.
* Second order: Omega_n = (h/2)(A_1 + A_2) + (sqrt(3) h^2 / 12) [A_2, A_1], the
  fourth-order Magnus integrator for dU/dt = L(t) U. For ZOH, A_1 = A_2 and the
  commutator vanishes.
"""
import numpy as np

SQ3 = np.sqrt(3.0)


def gl2_nodes():
    """Fractions lambda_k of the slice at which the two nodes sit."""
    return 0.5 - SQ3 / 6.0, 0.5 + SQ3 / 6.0


def node_controls(amps, n, hold):
    """Control values at the two Gauss-Legendre nodes of slice n."""
    N = amps.shape[0]
    u0 = amps[n]
    if hold == "zoh":
        return u0.copy(), u0.copy()
    u1 = amps[n + 1] if n + 1 < N else amps[n]
    l1, l2 = gl2_nodes()
    return u0 + l1 * (u1 - u0), u0 + l2 * (u1 - u0)


def slice_omega(liouv, amps, n, dt, order, hold):
    """Omega_n from a callable liouv(u) -> L (the full Eq. 8 matrix)."""
    ua, ub = node_controls(amps, n, hold)
    A1 = liouv(ua)
    A2 = liouv(ub)
    om = 0.5 * dt * (A1 + A2)
    if order == 2:
        om = om + (SQ3 * dt * dt / 12.0) * (A2 @ A1 - A1 @ A2)
    elif order != 1:
        raise ValueError("order must be 1 or 2")
    return om


def slice_omegas(liouv, amps, dt, order, hold):
    return [slice_omega(liouv, amps, n, dt, order, hold)
            for n in range(amps.shape[0])]
