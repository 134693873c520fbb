"""Parity of the HIP path with the FP64 oracle, through the C ABI.

Small cases span several chunks with a ragged tail and are compared element by
element; the full-size configurations compare the whole propagator and F, and
the gradient on sampled rows."""
import numpy as np
import pytest

import oracle
import synth
from helpers import oracle_system, lib_system, rounded, rel, hermitian_basis_change

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def to_dev(a, sysm):
    return torch.tensor(np.asarray(a), dtype=sysm.rdtype, device="cuda").contiguous()


def lib_fid(sysm, cfg, amps, want_grad=True, **kw):
    F, g = sysm.fidelity_and_grad(to_dev(amps, sysm), [len(amps)], cfg["dt"], cfg["U_target"],
                                  static_coef=np.asarray(cfg["B"])[None, :], want_grad=want_grad,
                                  **kw)
    return F.cpu().numpy(), (g.cpu().numpy().astype(np.float64) if g is not None else None)


# ----------------------------------------------------------- small cases
@pytest.mark.parametrize("prec,order,hold,chunk,basis", [
    ("f64", 1, "zoh", 7, "column"), ("f64", 2, "foh", 6, "column"), ("f32", 2, "foh", 7, "hermitian"),
    ("f32", 2, "foh", 7, "column"), ("f32", 1, "zoh", 0, "hermitian"), ("f32", 1, "zoh", 0, "column")])
def test_small_propagator_and_fidelity(prec, order, hold, chunk, basis):
    cfg = synth.small_case(100 + chunk, n_slices=40, dt=2.5e-4 if order == 2 else 1e-3)
    sysm = lib_system(cfg, prec, order, hold, chunk=chunk, basis=basis)
    amps = rounded(cfg["amps"], prec)
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], order, hold))
    U = sysm.propagate(to_dev(amps, sysm), [40], cfg["dt"],
                       static_coef=np.asarray(cfg["B"])[None, :]).cpu().numpy()[0]
    tol = 1e-12 if prec == "f64" else 2e-6
    assert rel(U, U_ref) < tol
    F_ref, _ = oracle.fidelity(U_ref, cfg["U_target"])
    F, _ = lib_fid(sysm, cfg, amps, want_grad=False)
    assert abs(F[0] - F_ref) < (1e-13 if prec == "f64" else 1e-7)


@pytest.mark.parametrize("prec,order,hold,chunk,basis", [
    ("f64", 2, "foh", 7, "column"), ("f64", 1, "zoh", 5, "column"), ("f32", 2, "foh", 7, "hermitian"),
    ("f32", 2, "foh", 7, "column")])
def test_small_gradient(prec, order, hold, chunk, basis):
    cfg = synth.small_case(200 + chunk, n_slices=30, dt=2.5e-4 if order == 2 else 1e-3)
    sysm = lib_system(cfg, prec, order, hold, chunk=chunk, basis=basis)
    amps = rounded(cfg["amps"], prec)
    osys = oracle_system(cfg)
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], order, hold, cfg["U_target"])
    F, g = lib_fid(sysm, cfg, amps)
    assert abs(F[0] - F_ref) < (1e-12 if prec == "f64" else 1e-7)
    assert rel(g, g_ref) < (1e-9 if prec == "f64" else 1e-4)


def test_padded_tiles_both_bases():
    """Two spins (d = 4): the superoperator fills the top-left 16 x 16 of a
    64 x 64 tile. In the basis of Hermitian operators the padding maps to
    itself; propagator, fidelity and gradient agree with the oracle in both
    bases."""
    cfg = synth.small_case(502, n_spins=2, n_slices=35, dt=2.5e-4)
    amps = rounded(cfg["amps"], "f32")
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    for basis in ("hermitian", "column"):
        sysm = lib_system(cfg, "f32", 2, "foh", chunk=6, basis=basis)
        U = sysm.propagate(to_dev(amps, sysm), [35], cfg["dt"],
                           static_coef=np.asarray(cfg["B"])[None, :]).cpu().numpy()[0]
        assert rel(U, U_ref) < 2e-6, basis
        F, g = lib_fid(sysm, cfg, amps)
        assert abs(F[0] - F_ref) < 1e-7, basis
        assert rel(g, g_ref) < 1e-4, basis


def test_zoh_second_order_equals_first_order():
    cfg = synth.small_case(7, n_slices=20, dt=1e-3)
    amps = cfg["amps"]
    s1 = lib_system(cfg, "f64", 1, "zoh", chunk=6)
    s2 = lib_system(cfg, "f64", 2, "zoh", chunk=6)
    b = np.asarray(cfg["B"])[None, :]
    U1 = s1.propagate(to_dev(amps, s1), [20], 1e-3, static_coef=b).cpu().numpy()
    U2 = s2.propagate(to_dev(amps, s2), [20], 1e-3, static_coef=b).cpu().numpy()
    assert rel(U2, U1) < 1e-13


# --------------------------------------------------- closed forms on the GPU
def test_gpu_rabi_single_spin():
    from paper_2511_13330_amd import System
    sx = np.array([[0, 1], [1, 0]], complex)
    sz = np.array([[1, 0], [0, -1]], complex)
    s = System([sz / 2], [sx / 2], [], precision="f64", magnus_order=1, hold="zoh", chunk_slices=3)
    W, N, h = 2 * np.pi * 3.0, 10, 0.037
    U = s.propagate(torch.full((N, 1), W, dtype=torch.float64, device="cuda"), [N], h,
                    static_coef=[[0.0]]).cpu().numpy()[0]
    t = N * h
    V = np.cos(W * t / 2) * np.eye(2) - 1j * np.sin(W * t / 2) * sx
    assert np.allclose(U, np.kron(V.conj(), V), atol=1e-12)


def test_gpu_two_spin_swap():
    from paper_2511_13330_amd import spin_chain_system
    SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], complex)
    s = spin_chain_system(2, precision="f64", magnus_order=2, hold="foh", chunk_slices=4)
    J, N = 2 * np.pi * 5.0, 16
    h = np.pi / J / N
    F, _ = s.fidelity_and_grad(torch.full((N, 1), J, dtype=torch.float64, device="cuda"), [N], h,
                               SWAP, static_coef=[[0.0, 0.0]], want_grad=False)
    assert abs(F.item() - 1.0) < 1e-12


# ------------------------------------------------------ full configurations
def test_config0_full_fp64():
    cfg = synth.config0()
    sysm = lib_system(cfg)
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(cfg["amps"], cfg["dt"], 1, "zoh"))
    U = sysm.propagate(to_dev(cfg["amps"], sysm), [100], cfg["dt"],
                       static_coef=np.asarray(cfg["B"])[None, :]).cpu().numpy()[0]
    assert rel(U, U_ref) < 1e-12
    F_ref, _ = oracle.fidelity(U_ref, cfg["U_target"])
    F, _ = lib_fid(sysm, cfg, cfg["amps"], want_grad=False)
    assert abs(F[0] - F_ref) < 1e-12


@pytest.fixture(scope="module", params=["hermitian", "column"])
def config1_run(request):
    cfg = synth.config1()
    sysm = lib_system(cfg, basis=request.param)
    amps = rounded(cfg["amps"], "f32")
    F, g = lib_fid(sysm, cfg, amps)
    U = sysm.propagate(to_dev(amps, sysm), [4096], cfg["dt"],
                       static_coef=np.asarray(cfg["B"])[None, :]).cpu().numpy()[0]
    assert sysm.basis == request.param
    return cfg, amps, F, g, U, sysm


def test_config1_propagator_and_fidelity(config1_run):
    cfg, amps, F, g, U, sysm = config1_run
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) <= 1e-4
    F_ref, _ = oracle.fidelity(U_ref, cfg["U_target"])
    assert abs(F[0] - F_ref) <= 1e-6
    hist = sysm.selection_histogram()
    # the propagate call: s = 0 everywhere, Pade-3 exactly for the slices whose
    # exponent's 1-norm in the kernel's basis exceeds theta_2 (up to slices at
    # the threshold within FP32 rounding)
    oms = osys.omegas(amps, cfg["dt"], 2, "foh")
    if sysm.basis == "hermitian":
        T = hermitian_basis_change(8)
        oms = [(T @ o @ T.conj().T).real for o in oms]
    norms = np.array([np.abs(o).sum(axis=0).max() for o in oms])
    above = int((norms > 8.093024022188482e-2).sum())   # theta_2 of the FP32 degree choice
    assert hist[:2, 0].sum() == 4096 and abs(int(hist[1, 0]) - above) <= 2, (above, hist[:2, 0])


def test_config1_gradient_sampled(config1_run):
    cfg, amps, F, g, U, sysm = config1_run
    osys = oracle_system(cfg)
    coords = np.asarray(cfg["fd_coords"])
    rows = sorted(set(int(c) // 2 for c in coords))
    _, g_at = oracle.grad_adjoint_at(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"], rows)
    ours = np.array([g[int(c) // 2, int(c) % 2] for c in coords])
    adj = np.array([g_at[int(c) // 2][int(c) % 2] for c in coords])
    assert rel(ours, adj) <= 1e-3
    fd = oracle.grad_fd_cached(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"], coords, h=1e-4)
    assert rel(ours, fd) <= 1e-3


def test_config1_long_chunks():
    """256-slice chunks, the length the automatic rule picks at the benchmark
    size: longer FP32 adjoint chains per chunk, fewer chunk totals to scan."""
    cfg = synth.config1()
    sysm = lib_system(cfg, chunk=256)
    amps = rounded(cfg["amps"], "f32")
    F, g = lib_fid(sysm, cfg, amps)
    assert sysm.last_plan()["chunk_slices"] == 256
    U = sysm.propagate(to_dev(amps, sysm), [4096], cfg["dt"],
                       static_coef=np.asarray(cfg["B"])[None, :]).cpu().numpy()[0]
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) <= 1e-4
    coords = np.asarray(cfg["fd_coords"])
    rows = sorted(set(int(c) // 2 for c in coords))
    F_ref, g_at = oracle.grad_adjoint_at(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"], rows)
    assert abs(F[0] - F_ref) <= 1e-6
    ours = np.array([g[int(c) // 2, int(c) % 2] for c in coords])
    adj = np.array([g_at[int(c) // 2][int(c) % 2] for c in coords])
    assert rel(ours, adj) <= 1e-3


def test_config1_high_fidelity_closed_system():
    """F near 1 is where rounding along the 4096-slice chain shows most (the
    error of F is first order in any non-unitary drift of the product). The
    target is the oracle's own closed-system propagator of the same pulse: the
    |up up up> state spans a one-dimensional S_z sector, so the top-left d x d
    block of the superoperator is the unitary up to a global phase."""
    cfg = synth.config1()
    amps = rounded(cfg["amps"], "f32")
    osys = oracle_system(cfg, dissipative=False)
    S_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    d = 8
    tgt = S_ref[:d, :d] / np.abs(np.linalg.det(S_ref[:d, :d])) ** (1.0 / d)
    F_ref, _ = oracle.fidelity(S_ref, tgt)
    assert F_ref > 1 - 1e-12
    sysm = lib_system(cfg, dissipative=False)
    S = sysm.propagate(to_dev(amps, sysm), [4096], cfg["dt"],
                       static_coef=np.asarray(cfg["B"])[None, :]).cpu().numpy()[0]
    assert rel(S, S_ref) <= 1e-4
    F, _ = lib_fid(sysm, {**cfg, "U_target": tgt}, amps, want_grad=False)
    assert abs(F[0] - F_ref) <= 1e-6
    # gradient near (not at) the optimum, F about 0.995
    rng = np.random.default_rng(11)
    a2 = rounded(amps + rng.normal(0.0, 0.05 * synth.A_MAX, amps.shape), "f32")
    F2, g2 = lib_fid(sysm, {**cfg, "U_target": tgt}, a2)
    coords = np.asarray(cfg["fd_coords"])
    rows = sorted(set(int(c) // 2 for c in coords))
    F2_ref, g_at = oracle.grad_adjoint_at(osys, a2, cfg["dt"], 2, "foh", tgt, rows)
    assert 0.9 < F2_ref < 1 - 1e-4
    assert abs(F2[0] - F2_ref) <= 1e-6
    ours = np.array([g2[int(c) // 2, int(c) % 2] for c in coords])
    adj = np.array([g_at[int(c) // 2][int(c) % 2] for c in coords])
    assert rel(ours, adj) <= 1e-3


# ------------------------------------------- scale-and-square path (s > 0)
@pytest.mark.parametrize("prec,dt,m_min,tol_F,tol_g", [
    ("f32", 1e-2, 3, 1e-7, 1e-4), ("f64", 2e-2, 7, 1e-12, 1e-9)])
def test_forced_squarings_forward_and_adjoint(prec, dt, m_min, tol_F, tol_g):
    """Slices long enough that ||Omega||_1 exceeds the largest Pade degree's
    theta (FP32: theta_3, FP64: theta_7), so every slice is scaled by 2^-s with
    s > 0 and squared back: the forward squarings D <- 2D + D^2 and the
    adjoint's squaring recurrence run in the 64 x 64 pipeline."""
    cfg = synth.small_case(300, n_slices=26, dt=dt)
    sysm = lib_system(cfg, prec, 2, "foh", chunk=6)
    amps = rounded(cfg["amps"], prec)
    osys = oracle_system(cfg)
    oms = osys.omegas(amps, dt, 2, "foh")
    theta = float(np.max([np.abs(o).sum(axis=0).max() for o in oms]))
    assert min(np.abs(o).sum(axis=0).max() for o in oms) > (0.43 if prec == "f32" else 0.96)
    U_ref = oracle.propagate(oms)
    U = sysm.propagate(to_dev(amps, sysm), [26], dt,
                       static_coef=np.asarray(cfg["B"])[None, :]).cpu().numpy()[0]
    hist = sysm.selection_histogram()
    row = {3: 1, 7: 3}[m_min]
    assert hist[row, 1:].sum() == 26 and hist[:, 0].sum() == 0, (theta, hist[:, :8])
    assert rel(U, U_ref) < (2e-6 if prec == "f32" else 1e-12)
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, dt, 2, "foh", cfg["U_target"])
    F, g = lib_fid(sysm, cfg, amps)
    assert abs(F[0] - F_ref) <= tol_F
    assert rel(g, g_ref) <= tol_g


def test_config1_gradient_all_coordinates(config1_run):
    """The whole 2 x 4096 gradient against the oracle's exact adjoint, norm-wise."""
    cfg, amps, F, g, U, sysm = config1_run
    osys = oracle_system(cfg)
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F[0] - F_ref) <= 1e-6
    assert rel(g, g_ref) <= 1e-3
