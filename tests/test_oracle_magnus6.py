"""Pins of the oracle's sixth-order Magnus slices (three Gauss-Legendre nodes):
global convergence order 6 against a fine RK4 integration of Eq. 9 (with the
fourth-order scheme's order 4 beside it), the commuting case in closed form,
piecewise-constant controls, and its derivative against central differences."""
import numpy as np
import scipy.linalg

import oracle

SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], complex)


def coarse_pulse(rng):
    c = rng.uniform(0, 2 * np.pi * 20, (5, 1))
    c[4] = c[3]          # the last slice holds its value: the function is the same at every k
    return c


def subdivided(coarse, k):
    return np.array([coarse[s] + (coarse[s + 1] - coarse[s]) * j / k
                     for s in range(len(coarse) - 1) for j in range(k)])


def test_convergence_orders_against_rk4():
    """A fixed piecewise-linear pulse over 80 ns on two dissipative spins, each
    of its 4 segments cut into k = 1, 2, 4 first-order-hold slices: the error of
    the sixth-order scheme falls as k^-6, that of the fourth-order (second-order
    Magnus) scheme as k^-4."""
    rng = np.random.default_rng(3)
    sysm = oracle.System(2, [2 * np.pi * 8, -2 * np.pi * 5], T1=50.0, T2=2.0)
    coarse = coarse_pulse(rng)
    T = 0.08
    ref = oracle.rk4_propagator(sysm, subdivided(coarse, 1), T / 4, "foh", 512)
    e6, e2 = [], []
    for k in (1, 2, 4):
        a = subdivided(coarse, k)
        h = T / len(a)
        e6.append(np.linalg.norm(oracle.propagate(sysm.omegas(a, h, 6, "foh")) - ref))
        e2.append(np.linalg.norm(oracle.propagate(sysm.omegas(a, h, 2, "foh")) - ref))
    s6 = np.log2(np.array(e6[:-1]) / np.array(e6[1:]))
    s2 = np.log2(np.array(e2[:-1]) / np.array(e2[1:]))
    assert np.all((s6 > 5.7) & (s6 < 6.4)), s6
    assert np.all((s2 > 3.8) & (s2 < 4.3)), s2


def test_commuting_generators_give_the_exact_integral():
    """Two spins, no fields, one exchange control: L(t) = J(t) Lift(S1.S2)
    commute at all times, so every commutator vanishes and the slice exponent is
    the three-point Gauss-Legendre rule, exact for the linear J of first-order
    hold: U = expm(Lift(S1.S2) int J dt); at int J dt = pi the channel is SWAP."""
    sysm = oracle.System(2, [0.0, 0.0])
    rng = np.random.default_rng(4)
    amps = rng.uniform(0, 50, (6, 1))
    h = 3e-3
    U = oracle.propagate(sysm.omegas(amps, h, 6, "foh"))
    u_ext = np.concatenate([amps[:, 0], amps[-1:, 0]])
    integral = h * np.sum(0.5 * (u_ext[:-1] + u_ext[1:]))
    G = oracle.lift_hamiltonian(oracle.exchange_terms(2)[0])
    assert np.allclose(U, scipy.linalg.expm(integral * G), atol=1e-13)
    J = np.full((8, 1), 2 * np.pi * 5.0)
    hs = np.pi / (2 * np.pi * 5.0) / 8
    F, _ = oracle.fidelity(oracle.propagate(sysm.omegas(J, hs, 6, "foh")), SWAP)
    assert abs(F - 1.0) < 1e-13


def test_piecewise_constant_controls_reduce_to_first_order():
    cfg_sys = oracle.System(3, [1.0, -2.0, 3.0], T1=100.0, T2=2.0)
    amps = np.random.default_rng(5).uniform(0, 100, (4, 2))
    for n in range(4):
        o6 = oracle.slice_omega(cfg_sys.liouv, amps, n, 2e-3, 6, "zoh")
        o1 = oracle.slice_omega(cfg_sys.liouv, amps, n, 2e-3, 1, "zoh")
        assert np.allclose(o6, o1, atol=1e-14)


def test_adjoint_against_central_differences():
    sysm = oracle.System(3, [3.0, -20.0, 41.0], T1=100.0, T2=2.0, eps=np.array([1.01, 0.98]))
    rng = np.random.default_rng(6)
    amps = rng.uniform(5, 120, (5, 2))
    Ut = np.linalg.qr(rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)))[0]
    h = 4e-3
    _, g = oracle.grad_adjoint(sysm, amps, h, 6, "foh", Ut)
    fd = oracle.grad_fd(sysm, amps, h, 6, "foh", Ut, np.arange(amps.size), h=1e-4)
    assert np.linalg.norm(g.reshape(-1) - fd) < 1e-6 * np.linalg.norm(fd)


def _rk4_generic(A, h, steps):
    n = A(0.0).shape[0]
    U = np.eye(n, dtype=complex)
    dt = h / steps
    for j in range(steps):
        t = j * dt
        k1 = A(t) @ U
        k2 = A(t + dt / 2) @ (U + dt / 2 * k1)
        k3 = A(t + dt / 2) @ (U + dt / 2 * k2)
        k4 = A(t + dt) @ (U + dt * k3)
        U = U + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return U


def test_local_order_seven_for_a_quadratic_generator():
    """The scheme on a generic (non-commuting, quadratic in time) generator
    A(t) = P0 + t P1 + t^2 P2, where all of a1, a2, a3 and both commutator levels
    contribute: the one-slice error against a fine RK4 falls as h^7."""
    from oracle.magnus import order6_terms, gl3_nodes, comm
    rng = np.random.default_rng(8)
    P = [rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)) for _ in range(3)]
    P[1] *= 6.0
    P[2] *= 30.0
    A = lambda t: P[0] + t * P[1] + t * t * P[2]
    errs = []
    for h in (0.2, 0.1):
        B = [A(c * h) for c in gl3_nodes()]
        a1, a2, a3, C1, W, C2, X, Y = order6_terms(*B, h)
        assert np.linalg.norm(a3) > 1e-3 * np.linalg.norm(a1)
        om = a1 + a3 / 12.0 + comm(X, Y) / 240.0
        errs.append(np.linalg.norm(scipy.linalg.expm(om) - _rk4_generic(A, h, 2000)))
    slope = np.log2(errs[0] / errs[1])
    assert 6.6 < slope < 7.4, (errs, slope)
