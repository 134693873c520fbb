"""State-level accuracy of the propagator (the paper's Fig. 3 experiment, Sec.
IV): a random initial density matrix is evolved by the GPU propagator of N
slices and by the oracle's RK4 integration of the Lindblad equation with the
smooth control, and the two final states are compared by the Uhlmann fidelity
as N grows. Second-order Magnus with first-order-hold controls converges at
fourth order in the infidelity (second order in the state), first-order
Magnus with piecewise-constant controls at second order."""
import numpy as np
import pytest

import oracle
from oracle import states as ost
import synth
from helpers import oracle_system, lib_system

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

T_TOTAL = 0.256          # us
NS = (8, 16, 32, 64, 128, 256, 512, 1024)


def pulse(t):
    A = synth.A_MAX
    return np.array([A * (0.5 + 0.35 * np.sin(2 * np.pi * t / T_TOTAL + 0.3)),
                     A * (0.5 + 0.35 * np.sin(4 * np.pi * t / T_TOTAL + 1.1))])


@pytest.fixture(scope="module")
def reference():
    cfg = synth.small_case(61, n_slices=8)
    rho0 = ost.random_density(8, np.random.default_rng(62))
    ref = ost.rk4_state(oracle_system(cfg), pulse, T_TOTAL, 16384, rho0)
    return cfg, rho0, ref


def study(cfg, rho0, ref, prec, order, hold):
    sysm = lib_system(cfg, prec, order, hold)
    dt_ = torch.float32 if prec == "f32" else torch.float64
    out = []
    for N in NS:
        h = T_TOTAL / N
        amps = np.stack([pulse(n * h) for n in range(N)])
        a = torch.tensor(amps, dtype=dt_, device="cuda").contiguous()
        U = sysm.propagate(a, [N], h, static_coef=np.asarray(cfg["B"])[None, :]).cpu().numpy()[0]
        rho = oracle.unvec(U.astype(np.complex128) @ oracle.vec(rho0), 8)
        rho = 0.5 * (rho + rho.conj().T)
        out.append(1.0 - ost.uhlmann(ref, rho))
    return np.array(out)


def orders(err):
    return np.log2(err[:-1] / err[1:])


def test_accuracy_study(reference):
    cfg, rho0, ref = reference
    e2 = study(cfg, rho0, ref, "f64", 2, "foh")
    e1 = study(cfg, rho0, ref, "f64", 1, "zoh")
    e2s = study(cfg, rho0, ref, "f32", 2, "foh")
    print("\nN      1-F (order 2, FOH, FP64)  1-F (order 1, ZOH, FP64)  1-F (order 2, FOH, FP32)")
    for N, a, b, c in zip(NS, e2, e1, e2s):
        print(f"{N:5d}  {a:.3e}                 {b:.3e}                 {c:.3e}")
    print("observed orders (FOH, ZOH):", np.round(orders(e2), 2), np.round(orders(e1), 2))
    assert np.all(np.diff(e2[:6]) < 0) and np.all(np.diff(e1) < 0)
    assert np.median(orders(e2)[1:5]) > 3.0
    assert np.median(orders(e1)[1:6]) > 1.5
    assert e2[-1] < 1e-8 and e2s[-1] < 1e-6
