"""Block-tiled path (superoperators larger than one 64x64 tile), FP32, against
the FP64 oracle: 4 spins (256 x 256) element by element on short pulses and, at
the full 8192-slice size, through invariants and the closed-system reduction
(the superoperator of a closed system is conj(V) (x) V, V computed by the oracle
in Hilbert space); 5 spins (1024 x 1024) element by element; 6 spins
(4096 x 4096) through the closed-system reduction (propagator, F, every
gradient coordinate) and sampled propagator columns of the dissipative system."""
import numpy as np
import pytest

import oracle
from oracle import hilbert as hb
import synth
from helpers import oracle_system, lib_system, rounded, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(cfg, amps, chunk=0, want_grad=True, dissipative=True, basis="hermitian"):
    sysm = lib_system(cfg, "f32", cfg["order"], cfg["hold"], chunk=chunk, dissipative=dissipative,
                      basis=basis)
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    N = len(amps)
    U = sysm.propagate(a, [N], cfg["dt"], static_coef=b).cpu().numpy()[0].astype(complex)
    F, g = sysm.fidelity_and_grad(a, [N], cfg["dt"], cfg["U_target"], static_coef=b,
                                  want_grad=want_grad)
    return sysm, U, F.cpu().numpy()[0], (g.cpu().numpy().astype(float) if g is not None else None)


@pytest.mark.parametrize("basis", ["hermitian", "column"])
@pytest.mark.parametrize("chunk", [0, 3])
def test_four_spin_small_matches_oracle(chunk, basis):
    cfg = synth.small_case(71, n_spins=4, n_slices=12, dt=2.5e-4)
    amps = rounded(cfg["amps"], "f32")
    sysm, U, F, g = run(cfg, amps, chunk, basis=basis)
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) < 2e-5
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F - F_ref) < 1e-6
    assert rel(g, g_ref) < 1e-3


@pytest.mark.parametrize("basis", ["hermitian", "column"])
def test_four_spin_with_squarings(basis):
    # 1 ns slices of large amplitudes push ||Omega||_1 above theta_3: s > 0
    cfg = synth.small_case(72, n_spins=4, n_slices=6, dt=4e-3)
    amps = rounded(cfg["amps"], "f32")
    sysm, U, F, g = run(cfg, amps, 2, basis=basis)
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


def test_four_spin_full_size_closed_system():
    """All 8192 slices of the 4-spin configuration without dissipation: the
    whole 256 x 256 propagator against conj(V) (x) V and F against
    |Tr(U_T^dag V)|^2 / d^2."""
    cfg = synth.config3_four()
    amps = rounded(cfg["amps"], "f32")
    V = hb.unitary(hb.HilbertSystem.from_cfg(cfg), amps, cfg["dt"], 2, "foh")
    sysm, U, F, _ = run(cfg, amps, want_grad=False, dissipative=False)
    assert rel(U, hb.superop(V)) <= 1e-4
    assert abs(F - hb.fidelity(V, cfg["U_target"])) <= 1e-6


def test_four_spin_closed_gradient_all_coordinates():
    """Every gradient coordinate (3 controls x 2048 slices of the 4-spin pulse)
    against the oracle's Hilbert-space adjoint, norm-wise."""
    cfg = synth.config3_four()
    amps = rounded(cfg["amps"][:2048], "f32")
    F_ref, g_ref = hb.grad(hb.HilbertSystem.from_cfg(cfg), amps, cfg["dt"], 2, "foh",
                           cfg["U_target"])
    sysm, U, F, g = run(cfg, amps, dissipative=False)
    assert abs(F - F_ref) <= 1e-6
    assert rel(g, g_ref) <= 1e-3


def test_four_spin_dissipative_512_slices():
    """The dissipative 4-spin system on the first 512 slices of its pulse: the
    whole propagator and F against the dense oracle, the gradient on sampled
    rows against the oracle's adjoint."""
    cfg = synth.config3_four()
    amps = rounded(cfg["amps"][:512], "f32")
    osys = oracle_system(cfg)
    sysm, U, F, g = run(cfg, amps)
    rows = [0, 1, 137, 300, 510, 511]
    F_ref, g_at = oracle.grad_adjoint_at(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"], rows)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) <= 1e-4
    assert abs(F - F_ref) <= 1e-6
    ours = np.concatenate([g[r] for r in rows])
    ref = np.concatenate([g_at[r] for r in rows])
    assert rel(ours, ref) <= 1e-3


@pytest.fixture(scope="module")
def six_closed():
    cfg = synth.config3_six()
    amps = rounded(cfg["amps"][:2], "f32")
    sysm, U, F, g = run(cfg, amps, dissipative=False)
    return cfg, amps, U, F, g


def test_six_spin_closed_propagator_and_fidelity(six_closed):
    """6 spins (superoperator 4096 x 4096), two 1 ns slices, FOH second order:
    the whole propagator against conj(V) (x) V and F against the reduction."""
    cfg, amps, U, F, g = six_closed
    V = hb.unitary(hb.HilbertSystem.from_cfg(cfg), amps, cfg["dt"], 2, "foh")
    assert rel(U, hb.superop(V)) <= 1e-4
    assert abs(F - hb.fidelity(V, cfg["U_target"])) <= 1e-6


def test_six_spin_closed_gradient(six_closed):
    """All 2 x 5 gradient coordinates against the reduction's adjoint and its
    FP64 central differences."""
    cfg, amps, U, F, g = six_closed
    hs = hb.HilbertSystem.from_cfg(cfg)
    F_ref, g_ref = hb.grad(hs, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert rel(g, g_ref) <= 1e-3
    fd = hb.grad_fd(hs, amps, cfg["dt"], 2, "foh", cfg["U_target"], np.arange(amps.size))
    assert rel(g.reshape(-1), fd) <= 1e-3


def test_six_spin_dissipative_sampled_columns():
    """The dissipative 6-spin propagator of two 1 ns slices: eight sampled
    columns against the oracle's slice-exponential action (Omega_n applied
    through the dense Eq. 8 node matrices), and trace preservation of the
    whole propagator."""
    cfg = synth.config3_six()
    amps = rounded(cfg["amps"][:2], "f32")
    sysm, U, F, _ = run(cfg, amps, want_grad=False)
    d = 64
    vI = np.eye(d).T.reshape(-1)
    assert np.abs(vI @ U - vI).max() < 1e-4
    cols = np.random.default_rng(6).choice(d * d, 8, replace=False)
    cols[0] = 0                                   # |0><0|: populations
    ref = hb.propagator_columns(oracle_system(cfg), amps, cfg["dt"], 2, "foh", list(cols))
    assert rel(U[:, cols], ref) <= 2e-5


def test_four_spin_recompute_bitwise_equal_to_stored():
    """Under a workspace budget too small for every slice's matrices, the
    block-tiled adjoint runs in slice windows and re-runs each window's
    forward instead of storing it: propagator, F and gradient are bitwise those
    of the stored path (same chunk length), with squarings in some slices."""
    cfg = synth.small_case(74, n_spins=4, n_slices=30, dt=2e-3)
    amps = rounded(cfg["amps"], "f32")
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    out = {}
    for name, budget in (("stored", 0), ("recompute", 100 << 20)):
        sysm = lib_system(cfg, "f32", 2, "foh", chunk=4, workspace_bytes_max=budget)
        F, g = sysm.fidelity_and_grad(a, [30], cfg["dt"], cfg["U_target"], static_coef=b)
        plan = sysm.last_plan()
        hist = sysm.selection_histogram()
        U = sysm.propagate(a, [30], cfg["dt"], static_coef=b)
        out[name] = (F, g, U, plan, hist)
    Fs, gs, Us, ps, hs = out["stored"]
    Fr, gr, Ur, pr, hr = out["recompute"]
    assert ps["recompute"] == 0 and ps["waves"] == 1
    assert pr["recompute"] == 1 and pr["waves"] > 1 and pr["workspace_bytes"] <= 100 << 20
    assert hs[1, 0] > 0 and hs[1, 1:].sum() > 0        # slices with and without squarings
    assert torch.equal(Fs, Fr) and torch.equal(gs, gr) and torch.equal(Us, Ur)
    osys = oracle_system(cfg)
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(Fs.item() - F_ref) < 1e-6
    assert rel(gs.cpu().numpy().astype(float), g_ref) < 1e-3


def test_six_spin_full_pulse_under_64_GB():
    """The 6-spin configuration (4096 x 4096 superoperator, 128 slices of
    1 ns, five controls) without dissipation, forward and adjoint under a
    64 GB workspace budget (storing every slice's matrices would need about
    190 GB): the adjoint recomputes the forward window by window. Propagator,
    F and all 640 gradient coordinates against the Hilbert-space reduction."""
    cfg = synth.config3_six()
    amps = rounded(cfg["amps"], "f32")
    sysm = lib_system(cfg, "f32", 2, "foh", dissipative=False, workspace_bytes_max=64 << 30)
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    F, g = sysm.fidelity_and_grad(a, [128], cfg["dt"], cfg["U_target"], static_coef=b)
    plan = sysm.last_plan()
    assert plan["recompute"] == 1 and plan["workspace_bytes"] <= 64 << 30
    hs = hb.HilbertSystem.from_cfg(cfg)
    F_ref, g_ref = hb.grad(hs, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F.item() - F_ref) <= 1e-6
    assert rel(g.cpu().numpy().astype(float), g_ref) <= 1e-3
    U = sysm.propagate(a, [128], cfg["dt"], static_coef=b).cpu().numpy()[0].astype(complex)
    V = hb.unitary(hs, amps, cfg["dt"], 2, "foh")
    assert rel(U, hb.superop(V)) <= 1e-4


def _tuning_line(path, d, total, chunk, variant, basis="column"):
    b = int(np.floor(np.log2(total)))
    tag = "h" if basis == "hermitian" else ""
    with open(path, "w") as f:
        f.write('{"key": "p32%s_o2_d%d_s%d", "chunk": %d, "variant": %d, "ms": 0.0}\n'
                % (tag, d, b, chunk, variant))


@pytest.mark.parametrize("basis,variant", [("column", v) for v in range(9)] +
                         [("hermitian", v) for v in (0, 1, 2, 5, 7)])
def test_four_spin_product_kernels_match_oracle(basis, variant, tmp_path):
    """Each product kernel of the block-tiled path (register-B tiles with the
    16x16x4 MFMA; a quadrant per wave with 16x16x4; a quadrant per wave with
    32x32x2; a quadrant per wave with split-bf16 operands on the 16x16x32 bf16
    MFMA; two output tiles per eight-wave workgroup; register-B tiles with each
    product on one XCD; register-B tiles at three workgroups per CU, without and
    with the XCD grouping; register-B tiles with the A tiles double-buffered in
    LDS by direct global-to-LDS loads; in the real Hermitian-operator basis the
    real 64 x 64 kernel without and with the XCD grouping and the real 128 x 128
    kernel), selected through a tuning
    line: propagator, F and gradient against the oracle, with squarings in some
    slices."""
    cfg = synth.small_case(75, n_spins=4, n_slices=14, dt=2e-3)
    amps = rounded(cfg["amps"], "f32")
    sysm = lib_system(cfg, "f32", 2, "foh", basis=basis)
    path = tmp_path / "tune.jsonl"
    _tuning_line(path, 16, 14, 4, variant, basis)
    sysm.load_tuning(str(path))
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    U = sysm.propagate(a, [14], cfg["dt"], static_coef=b).cpu().numpy()[0].astype(complex)
    F, g = sysm.fidelity_and_grad(a, [14], cfg["dt"], cfg["U_target"], static_coef=b)
    assert sysm.last_plan()["chunk_slices"] == 4
    osys = oracle_system(cfg)
    U_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    assert rel(U, U_ref) < 2e-5
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F.item() - F_ref) < 1e-6
    assert rel(g.cpu().numpy().astype(float), g_ref) < 1e-3


def test_block_tiled_autotune_picks_a_kernel():
    cfg = synth.small_case(76, n_spins=4, n_slices=256, dt=2.5e-4)
    amps = rounded(cfg["amps"], "f32")
    sysm = lib_system(cfg, "f32", 2, "foh")
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    chunk, variant, ms = sysm.autotune(a, [256], cfg["dt"], cfg["U_target"], static_coef=b, reps=1)
    assert 0 <= variant < 9 and chunk >= 1 and ms > 0
    F, g = sysm.fidelity_and_grad(a, [256], cfg["dt"], cfg["U_target"], static_coef=b)
    assert sysm.last_plan()["chunk_slices"] == chunk
    F_ref, _ = oracle.fidelity(oracle.propagate(oracle_system(cfg).omegas(amps, cfg["dt"], 2, "foh")),
                               cfg["U_target"])
    assert abs(F.item() - F_ref) < 1e-6


def test_four_spin_noise_groups_match_oracle_means():
    """Block-tiled path with quasi-static noise: two candidates x two noise
    samples (field offsets, control scales), grouped per candidate."""
    cfg = synth.small_case(77, n_spins=4, n_slices=10, dt=2.5e-4)
    rng = np.random.default_rng(5)
    amps = [rounded(cfg["amps"], "f32"), rounded(rng.uniform(0, synth.A_MAX, (7, 3)), "f32")]
    dB = rng.normal(0, 2 * np.pi, (2, 4))
    eps = rng.normal(1, 0.01, (2, 3))
    flat = np.concatenate(amps)
    ns, off, static, scale, groups = [], [], [], [], []
    for c, o in ((0, 0), (1, 10)):
        for s in range(2):
            ns.append(len(amps[c])); off.append(o); groups.append(c)
            static.append(np.asarray(cfg["B"]) + dB[s]); scale.append(eps[s])
    sysm = lib_system(cfg, "f32", 2, "foh", chunk=3)
    F, g = sysm.fidelity_and_grad(torch.tensor(flat, dtype=torch.float32, device="cuda"), ns,
                                  cfg["dt"], cfg["U_target"], slice_offset=off,
                                  static_coef=np.array(static), ctrl_scale=np.array(scale),
                                  groups=groups)
    F = F.cpu().numpy(); g = g.cpu().numpy().astype(float)
    for c, o in ((0, 0), (1, 10)):
        Fs, gs = [], []
        for s in range(2):
            osys = oracle_system(cfg, eps=eps[s], dB=dB[s])
            f, gk = oracle.grad_adjoint(osys, amps[c], cfg["dt"], 2, "foh", cfg["U_target"])
            Fs.append(f); gs.append(gk)
        assert abs(F[c] - np.mean(Fs)) < 1e-6
        assert rel(g[o:o + len(amps[c])], np.mean(gs, axis=0)) < 1e-3


def test_block_tiled_output_at_unaligned_address():
    """The propagator written to a caller's buffer that starts 8 bytes past a
    16-byte boundary (the elementwise kernels then take their one-element
    path) equals the one written to an aligned buffer, bit for bit."""
    import ctypes
    from paper_2511_13330_amd._lib import lib, check
    cfg = synth.small_case(77, n_spins=4, n_slices=5, dt=2.5e-4)
    amps = rounded(cfg["amps"], "f32")
    sysm = lib_system(cfg, "f32", 2, "foh")
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    st = np.asarray(cfg["B"])[None, :]
    U = sysm.propagate(a, [5], cfg["dt"], static_coef=st)
    b, keep, n_items, _ = sysm._batch(a, [5], None, cfg["dt"], st, None, None)
    n = U.shape[-1]
    buf = torch.zeros(n * n + 1, dtype=torch.complex64, device="cuda")
    view = buf[1:]
    assert view.data_ptr() % 16 == 8
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(lib().lmag_propagate(sysm._ctx, ctypes.byref(b), ctypes.c_void_p(view.data_ptr()), stream),
          sysm._ctx)
    del keep
    torch.cuda.synchronize()
    assert torch.equal(view.view(1, n, n), U)
    assert buf[0].item() == 0


def test_hermitian_and_column_bases_agree():
    """The two representations of the block-tiled path on one 4-spin pulse of
    64 slices: propagator, F and gradient agree to FP32 rounding, and the real
    one uses half the workspace."""
    cfg = synth.small_case(79, n_spins=4, n_slices=64, dt=1e-3)
    amps = rounded(cfg["amps"], "f32")
    out = {}
    for basis in ("hermitian", "column"):
        sysm, U, F, g = run(cfg, amps, 8, basis=basis)
        out[basis] = (U, F, g, sysm.last_plan()["workspace_bytes"])
    (Uh, Fh, gh, wh), (Uc, Fc, gc, wc) = out["hermitian"], out["column"]
    assert rel(Uh, Uc) < 2e-5
    assert abs(Fh - Fc) < 1e-6
    assert rel(gh, gc) < 1e-4
    assert wh < 0.6 * wc
