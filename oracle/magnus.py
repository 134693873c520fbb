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
* Order 6: the sixth-order Magnus integrator on the three Gauss-Legendre nodes
  c_{1,2,3} = 1/2 - sqrt(15)/10, 1/2, 1/2 + sqrt(15)/10 (Blanes, Casas and Ros,
  BIT 40 (2000); the same scheme extends the paper's slice average, Eq. 13, to
  longer slices). With B_k = L(t_n + c_k h),
    a1 = h B_2, a2 = (sqrt(15) h / 3)(B_3 - B_1), a3 = (10 h / 3)(B_3 - 2 B_2 + B_1),
    C1 = [a1, a2], C2 = -(1/60) [a1, 2 a3 + C1],
    Omega_n = a1 + a3 / 12 + (1/240) [-20 a1 - a3 + C1, a2 + C2].
  When the L(t) commute, Omega_n is the three-point Gauss-Legendre quadrature
  h (5 B_1 + 8 B_2 + 5 B_3) / 18 of the slice integral.
"""
import numpy as np

SQ3 = np.sqrt(3.0)
SQ15 = np.sqrt(15.0)


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


def gl3_nodes():
    """Fractions of the slice at which the three nodes of order 6 sit."""
    return 0.5 - SQ15 / 10.0, 0.5, 0.5 + SQ15 / 10.0


def node_controls3(amps, n, hold):
    """Control values at the three Gauss-Legendre nodes of slice n."""
    N = amps.shape[0]
    u0 = amps[n]
    if hold == "zoh":
        return u0.copy(), u0.copy(), u0.copy()
    u1 = amps[n + 1] if n + 1 < N else amps[n]
    return tuple(u0 + lam * (u1 - u0) for lam in gl3_nodes())


def comm(X, Y):
    return X @ Y - Y @ X


def order6_terms(B1, B2, B3, dt):
    """(a1, a2, a3, C1, W, C2, X, Y) of the sixth-order scheme, W = 2 a3 + C1,
    X = -20 a1 - a3 + C1, Y = a2 + C2; Omega = a1 + a3/12 + [X, Y]/240."""
    a1 = dt * B2
    a2 = (SQ15 * dt / 3.0) * (B3 - B1)
    a3 = (10.0 * dt / 3.0) * (B3 - 2.0 * B2 + B1)
    C1 = comm(a1, a2)
    W = 2.0 * a3 + C1
    C2 = -comm(a1, W) / 60.0
    X = -20.0 * a1 - a3 + C1
    Y = a2 + C2
    return a1, a2, a3, C1, W, C2, X, Y


def slice_omega(liouv, amps, n, dt, order, hold):
    """Omega_n from a callable liouv(u) -> L (the full Eq. 8 matrix)."""
    if order == 6:
        u1, u2, u3 = node_controls3(amps, n, hold)
        a1, a2, a3, C1, W, C2, X, Y = order6_terms(liouv(u1), liouv(u2), liouv(u3), dt)
        return a1 + a3 / 12.0 + comm(X, Y) / 240.0
    ua, ub = node_controls(amps, n, hold)
    A1 = liouv(ua)
    A2 = liouv(ub)
    om = 0.5 * dt * (A1 + A2)
    if order == 2:
        om = om + (SQ3 * dt * dt / 12.0) * (A2 @ A1 - A1 @ A2)
    elif order != 1:
        raise ValueError("order must be 1, 2 or 6")
    return om


def slice_omegas(liouv, amps, dt, order, hold):
    return [slice_omega(liouv, amps, n, dt, order, hold)
            for n in range(amps.shape[0])]
