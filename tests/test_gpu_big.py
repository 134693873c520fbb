"""Block-tiled path (superoperators larger than one 64x64 tile): 4 spins,
256 x 256 superoperator, FP32, against the FP64 oracle; full-size 4-spin
configuration through invariants."""
import numpy as np
import pytest

import oracle
import synth
from helpers import oracle_system, lib_system, rounded, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(cfg, amps, chunk=0, want_grad=True, dissipative=True):
    sysm = lib_system(cfg, "f32", cfg["order"], cfg["hold"], chunk=chunk, dissipative=dissipative)
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    N = len(amps)
    U = sysm.propagate(a, [N], cfg["dt"], static_coef=b).cpu().numpy()[0].astype(complex)
    F, g = sysm.fidelity_and_grad(a, [N], cfg["dt"], cfg["U_target"], static_coef=b,
                                  want_grad=want_grad)
    return sysm, U, F.cpu().numpy()[0], (g.cpu().numpy().astype(float) if g is not None else None)


@pytest.mark.parametrize("chunk", [0, 3])
def test_four_spin_small_matches_oracle(chunk):
    cfg = synth.small_case(71, n_spins=4, n_slices=12, dt=2.5e-4)
    amps = rounded(cfg["amps"], "f32")
    sysm, U, F, g = run(cfg, amps, chunk)
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) < 2e-5
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F - F_ref) < 1e-6
    assert rel(g, g_ref) < 1e-3


def test_four_spin_with_squarings():
    # 1 ns slices of large amplitudes push ||Omega||_1 above theta_3: s > 0
    cfg = synth.small_case(72, n_spins=4, n_slices=6, dt=4e-3)
    amps = rounded(cfg["amps"], "f32")
    sysm, U, F, g = run(cfg, amps, 2)
    hist = sysm.selection_histogram()
    assert hist[1, 1:].sum() > 0   # Pade-3 with squarings
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) < 1e-4
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F - F_ref) < 1e-6
    assert rel(g, g_ref) < 1e-3


def test_four_spin_full_size_invariants():
    cfg = synth.config3_four()
    amps = rounded(cfg["amps"], "f32")
    sysm, U, F, g = run(cfg, amps)
    d = 16
    vI = np.eye(d).T.reshape(-1)
    # trace preservation holds for any slice count (up to FP32 rounding)
    assert np.abs(vI @ U - vI).max() < 1e-3
    # Hermiticity preservation: S[(i,j),(k,l)] = conj(S[(j,i),(l,k)])
    P = np.zeros((d * d, d * d))
    for i in range(d):
        for j in range(d):
            P[j + d * i, i + d * j] = 1.0
    assert np.linalg.norm(U - (P @ U @ P).conj()) < 1e-3 * np.linalg.norm(U)
    assert 0.0 <= F <= 1.0 and np.all(np.isfinite(g))
    # the first slices' gradient against the oracle on a truncated pulse is
    # covered by the small cases; here the sampled gradient must be finite and
    # the propagator a contraction in the trace norm sense
    assert np.linalg.norm(U, 2) < 1.5


def test_five_spin_propagator_and_fidelity():
    # superoperator 1024 x 1024 (16 x 16 tiles per side), two slices
    cfg = synth.small_case(73, n_spins=5, n_slices=2, dt=2.5e-4)
    amps = rounded(cfg["amps"], "f32")
    sysm, U, F, _ = run(cfg, amps, want_grad=False)
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) < 2e-5
    F_ref, _ = oracle.fidelity(U_ref, cfg["U_target"])
    assert abs(F - F_ref) < 1e-6


def test_four_spin_high_fidelity_closed_system():
    """F near 1 on the block-tiled path: 1024 slices of 0.25 ns, target = the
    oracle's own closed-system propagator (|up up up up> spans a one-dimensional
    S_z sector, so the top-left d x d block is the unitary up to a phase)."""
    cfg = synth.small_case(72, n_spins=4, n_slices=1024, dt=2.5e-4)
    amps = rounded(cfg["amps"], "f32")
    osys = oracle_system(cfg, dissipative=False)
    S_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    d = cfg["d"]
    tgt = S_ref[:d, :d] / np.abs(np.linalg.det(S_ref[:d, :d])) ** (1.0 / d)
    F_ref, _ = oracle.fidelity(S_ref, tgt)
    assert F_ref > 1 - 1e-12
    sysm, U, F, _ = run({**cfg, "U_target": tgt}, amps, want_grad=False, dissipative=False)
    assert rel(U, S_ref) < 1e-4
    assert abs(F - F_ref) <= 1e-6
