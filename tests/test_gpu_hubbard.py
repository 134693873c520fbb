"""The Hubbard model of three quantum dots (Eq. 1; 64 states, superoperator
4096 x 4096 -- the paper's measured problem size) and of two dots (256 x 256)
through the block-tiled path, FP32, against the oracle's Hubbard model:
the closed system through the Hilbert-space reduction (propagator, F, every
gradient coordinate, also over a whole 128-slice pulse under a 64 GB workspace
budget), the dissipative system by sampled propagator columns and, for two
dots, element by element with the gradient."""
import numpy as np
import pytest

import oracle
from oracle import hilbert as hb
from oracle import hubbard as hu
import synth
from helpers import rounded, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def lib_hubbard(cfg, n_dots, dissipative, **kw):
    from paper_2511_13330_amd import hubbard_system
    T1, T2 = (cfg["T1"], cfg["T2"]) if dissipative else (np.inf, np.inf)
    return hubbard_system(n_dots, T1, T2, precision="f32", magnus_order=2, hold="foh", **kw)


def run(sysm, cfg, amps, coef, want_grad=True, propagate=True):
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(coef)[None, :]
    N = len(amps)
    U = None
    if propagate:
        U = sysm.propagate(a, [N], cfg["dt"], static_coef=b).cpu().numpy()[0].astype(complex)
    F, g = sysm.fidelity_and_grad(a, [N], cfg["dt"], cfg["U_target"], static_coef=b,
                                  want_grad=want_grad)
    return U, F.item(), (g.cpu().numpy().astype(float) if g is not None else None)


def test_three_dots_closed_two_slices():
    cfg = synth.hubbard3()
    amps = rounded(cfg["amps"][:2], "f32")
    U, F, g = run(lib_hubbard(cfg, 3, False), cfg, amps, cfg["coef"])
    hil = hu.HubbardHilbert(3, cfg["coef"])
    V = hb.unitary(hil, amps, cfg["dt"], 2, "foh")
    assert rel(U, hb.superop(V)) <= 1e-4
    F_ref, g_ref = hb.grad(hil, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F - F_ref) <= 1e-6
    assert rel(g, g_ref) <= 1e-3
    fd = hb.grad_fd(hil, amps, cfg["dt"], 2, "foh", cfg["U_target"], np.arange(amps.size))
    assert rel(g.reshape(-1), fd) <= 1e-3


def test_three_dots_dissipative_sampled_columns():
    cfg = synth.hubbard3()
    amps = rounded(cfg["amps"][:2], "f32")
    U, F, _ = run(lib_hubbard(cfg, 3, True), cfg, amps, cfg["coef"], want_grad=False)
    vI = np.eye(64).T.reshape(-1)
    assert np.abs(vI @ U - vI).max() < 1e-4
    cols = np.random.default_rng(8).choice(4096, 8, replace=False)
    cols[0] = 1 + 64 * 1          # |up><up| on dot 3's single-electron state
    ref = hb.propagator_columns(hu.HubbardSystem(3, cfg["coef"], cfg["T1"], cfg["T2"]), amps,
                                cfg["dt"], 2, "foh", list(cols))
    assert rel(U[:, cols], ref) <= 2e-5


def test_three_dots_closed_full_pulse_under_64_GB():
    cfg = synth.hubbard3()
    amps = rounded(cfg["amps"], "f32")
    sysm = lib_hubbard(cfg, 3, False, workspace_bytes_max=64 << 30)
    U, F, g = run(sysm, cfg, amps, cfg["coef"])
    assert sysm.last_plan()["recompute"] == 1
    hil = hu.HubbardHilbert(3, cfg["coef"])
    F_ref, g_ref = hb.grad(hil, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F - F_ref) <= 1e-6
    assert rel(g, g_ref) <= 1e-3
    V = hb.unitary(hil, amps, cfg["dt"], 2, "foh")
    assert rel(U, hb.superop(V)) <= 1e-4


def test_two_dots_dissipative_element_by_element():
    cfg = synth.hubbard3(seed=6, n_slices=16)
    coef = np.concatenate([cfg["coef"][:3], cfg["coef"][4:]])     # U~, V_1, V_2, U_C
    amps = rounded(cfg["amps"][:, :1], "f32")
    Ut = synth.haar_unitary(np.random.default_rng(9), 16)
    cfg2 = {**cfg, "U_target": Ut}
    U, F, g = run(lib_hubbard(cfg2, 2, True, chunk_slices=5), cfg2, amps, coef)
    osys = hu.HubbardSystem(2, coef, cfg["T1"], cfg["T2"])
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) <= 2e-5
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", Ut)
    assert abs(F - F_ref) <= 1e-6
    assert rel(g, g_ref) <= 1e-3
