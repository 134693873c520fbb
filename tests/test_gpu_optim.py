"""The optimiser row: Adam + projection kernel against the oracle step, and a
refine run on a reachable target."""
import numpy as np
import pytest

import oracle
import synth
from helpers import lib_system, oracle_system, rounded, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_adam_kernel_matches_oracle(prec):
    from paper_2511_13330_amd import spin_chain_system
    s = spin_chain_system(3, precision=prec, magnus_order=1, hold="zoh")
    rng = np.random.default_rng(3)
    rows = 1000
    th = rng.uniform(0, 10, (rows, 2)); m = np.zeros_like(th); v = np.zeros_like(th)
    active = rng.random(rows) < 0.8
    dt = torch.float32 if prec == "f32" else torch.float64
    T = lambda x: torch.tensor(x, dtype=dt, device="cuda").contiguous()
    tth, tm, tv = T(th), T(m), T(v)
    act = torch.tensor(active.astype(np.uint8), device="cuda")
    for t in range(1, 6):
        g = rng.standard_normal((rows, 2)) * 3
        gq = g.astype(np.float32).astype(np.float64) if prec == "f32" else g
        s.adam_project(tth, T(g), tm, tv, t, 0.7, grad_scale=-1.0, lo=0.0, hi=10.0,
                       row_active=act)
        th, m, v = oracle.adam_project(th, gq, m, v, t, 0.7, grad_scale=-1.0, lo=0.0, hi=10.0,
                                       active=active)
        if prec == "f32":
            th, m, v = [x.astype(np.float32).astype(np.float64) for x in (th, m, v)]
    tol = 1e-5 if prec == "f32" else 1e-13
    assert np.allclose(tth.cpu().numpy(), th, rtol=tol, atol=tol)
    assert np.allclose(tm.cpu().numpy(), m, rtol=tol, atol=tol)


def test_refine_step_equals_oracle_adam_on_oracle_gradient():
    from paper_2511_13330_amd.optim import refine
    cfg = synth.small_case(41, n_slices=20)
    sysm = lib_system(cfg, chunk=6)
    a0 = rounded(cfg["amps"], "f32")
    amps = torch.tensor(a0, dtype=torch.float32, device="cuda")
    out = refine(sysm, amps, [20], cfg["dt"], cfg["U_target"], max_steps=1, amax=synth.A_MAX,
                 static_coef=np.asarray(cfg["B"])[None, :])
    F0, g0 = oracle.grad_adjoint(oracle_system(cfg), a0, cfg["dt"], 2, "foh", cfg["U_target"])
    th, _, _ = oracle.adam_project(a0, g0, 0 * a0, 0 * a0, 1, 0.01 * synth.A_MAX,
                                   grad_scale=-1.0, lo=0.0, hi=synth.A_MAX)
    assert abs(out["history"][0] - F0) < 1e-7
    # first Adam step moves every free coordinate by ~lr * sign(g); compare positions
    assert np.allclose(amps.cpu().numpy(), th, atol=1e-4 * synth.A_MAX)


def test_refine_reaches_reachable_target():
    # closed system; the target is the propagator of a reference pulse (reachable);
    # the start is the reference scaled by 0.6 (F about 0.87)
    from paper_2511_13330_amd.optim import refine
    import scipy.linalg as sla
    cfg = synth.small_case(43, n_slices=96, dt=2.5e-4)
    osys = oracle_system(cfg, dissipative=False)
    ref = cfg["amps"]
    UH = np.eye(8, dtype=complex)
    for n in range(96):   # midpoint rule of the FOH pulse: accurate to O(h^2)
        UH = sla.expm(-1j * cfg["dt"] * osys.H(0.5 * (ref[n] + ref[min(n + 1, 95)]))) @ UH
    sysm = lib_system(cfg, dissipative=False, chunk=16)
    amps = torch.tensor(0.6 * ref, dtype=torch.float32, device="cuda")
    out = refine(sysm, amps, [96], cfg["dt"], UH, max_steps=40, amax=synth.A_MAX, lr=2.0,
                 static_coef=np.asarray(cfg["B"])[None, :])
    h = out["history"]
    assert h[0] < 0.9
    assert out["reached"][0] > 0 and max(h) >= 0.999
