"""Batched calls through the C ABI: uneven slice counts, quasi-static noise
groups, autograd, determinism, streams and argument errors."""
import numpy as np
import pytest

import oracle
import synth
from helpers import oracle_system, lib_system, rounded, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def small_robust(seed=5, n_cand=3, n_noise=4, n_min=9, n_max=23):
    return synth.config2(seed, n_cand=n_cand, n_noise=n_noise, n_min=n_min, n_max=n_max)


def test_uneven_items_match_single_calls():
    cfg = small_robust()
    sysm = lib_system(cfg, chunk=4)
    amps = [rounded(a, "f32") for a in cfg["amps_per_cand"]]
    flat = torch.tensor(np.concatenate(amps), dtype=torch.float32, device="cuda")
    ns = [len(a) for a in amps]
    b = np.tile(np.asarray(cfg["B"])[None, :], (len(ns), 1))
    F, g = sysm.fidelity_and_grad(flat, ns, cfg["dt"], cfg["U_target"], static_coef=b)
    off = np.concatenate([[0], np.cumsum(ns)[:-1]])
    osys = oracle_system(cfg)
    for i, a in enumerate(amps):
        F1, g1 = sysm.fidelity_and_grad(torch.tensor(a, dtype=torch.float32, device="cuda"),
                                        [ns[i]], cfg["dt"], cfg["U_target"],
                                        static_coef=b[:1])
        assert torch.equal(F[i:i + 1], F1)
        assert torch.equal(g[off[i]:off[i] + ns[i]], g1)
        Fr, gr = oracle.grad_adjoint(osys, a, cfg["dt"], 2, "foh", cfg["U_target"])
        assert abs(F1.item() - Fr) < 1e-7
        assert rel(g1.cpu().numpy(), gr) < 1e-4


def test_noise_groups_match_oracle_means():
    cfg = small_robust(n_cand=2, n_noise=3)
    sysm = lib_system(cfg, chunk=5)
    amps = [rounded(a, "f32") for a in cfg["amps_per_cand"]]
    flat = np.concatenate(amps)
    ns_c = [len(a) for a in amps]
    off_c = np.concatenate([[0], np.cumsum(ns_c)[:-1]])
    n_noise = cfg["dB"].shape[0]
    # items = candidate x noise sample, sharing the candidate's amplitude rows
    ns, off, static, scale, groups = [], [], [], [], []
    for c in range(len(amps)):
        for s in range(n_noise):
            ns.append(ns_c[c]); off.append(off_c[c]); groups.append(c)
            static.append(np.asarray(cfg["B"]) + cfg["dB"][s])
            scale.append(cfg["eps"][s])
    F, g = sysm.fidelity_and_grad(torch.tensor(flat, dtype=torch.float32, device="cuda"), ns,
                                  cfg["dt"], cfg["U_target"], slice_offset=off,
                                  static_coef=np.array(static), ctrl_scale=np.array(scale),
                                  groups=groups)
    F = F.cpu().numpy(); g = g.cpu().numpy()
    for c in range(len(amps)):
        Fs, gs = [], []
        for s in range(n_noise):
            osys = oracle_system(cfg, eps=cfg["eps"][s], dB=cfg["dB"][s])
            Fr, gr = oracle.grad_adjoint(osys, amps[c], cfg["dt"], 2, "foh", cfg["U_target"])
            Fs.append(Fr); gs.append(gr)
        assert abs(F[c] - np.mean(Fs)) < 1e-7
        assert rel(g[off_c[c]:off_c[c] + ns_c[c]], np.mean(gs, axis=0)) < 1e-4


def test_pulse_fidelity_autograd():
    from paper_2511_13330_amd import PulseFidelity
    cfg = synth.small_case(31, n_slices=16)
    sysm = lib_system(cfg, chunk=5)
    amps = torch.tensor(rounded(cfg["amps"], "f32"), dtype=torch.float32, device="cuda",
                        requires_grad=True)
    F = PulseFidelity.apply(amps, sysm, [16], cfg["dt"], cfg["U_target"],
                            {"static_coef": np.asarray(cfg["B"])[None, :]})
    loss = 3.0 * (1.0 - F).sum()
    loss.backward()
    _, g = oracle.grad_adjoint(oracle_system(cfg), amps.detach().cpu().numpy().astype(float),
                               cfg["dt"], 2, "foh", cfg["U_target"])
    assert rel(amps.grad.cpu().numpy(), -3.0 * g) < 1e-4


def test_bitwise_determinism_and_stream():
    cfg = synth.small_case(32, n_slices=50)
    sysm = lib_system(cfg, chunk=7)
    amps = torch.tensor(rounded(cfg["amps"], "f32"), dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    F1, g1 = sysm.fidelity_and_grad(amps, [50], cfg["dt"], cfg["U_target"], static_coef=b)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        F2, g2 = sysm.fidelity_and_grad(amps, [50], cfg["dt"], cfg["U_target"], static_coef=b,
                                        stream=st)
    st.synchronize()
    assert torch.equal(F1, F2) and torch.equal(g1, g2)


def test_argument_errors_leave_outputs_untouched():
    from paper_2511_13330_amd import LmagError
    cfg = synth.small_case(33, n_slices=8)
    sysm = lib_system(cfg)
    amps = torch.zeros((8, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(LmagError, match="INVALID"):
        sysm.fidelity_and_grad(amps, [8], -1.0, cfg["U_target"])
    with pytest.raises(LmagError, match="INVALID"):
        sysm.fidelity_and_grad(amps, [8], 1e-3, cfg["U_target"], target_of_item=[3])
    with pytest.raises(ValueError):
        sysm.fidelity_and_grad(amps, [9], 1e-3, cfg["U_target"])
    with pytest.raises(LmagError, match="INVALID"):
        sysm.fidelity_and_grad(amps, [4, 4], 1e-3, cfg["U_target"], slice_offset=[0, 4],
                               groups=[0, 0])


def test_nan_amplitudes_propagate_to_F():
    cfg = synth.small_case(34, n_slices=8)
    sysm = lib_system(cfg)
    a = rounded(cfg["amps"], "f32").copy()
    a[3, 1] = np.nan
    F, g = sysm.fidelity_and_grad(torch.tensor(a, dtype=torch.float32, device="cuda"), [8],
                                  cfg["dt"], cfg["U_target"],
                                  static_coef=np.asarray(cfg["B"])[None, :])
    assert torch.isnan(F).all()


def test_benchmark_batch_plan_and_consistency():
    """The benchmark's batch, 64 config-1 pulses: the automatic chunk length is
    256 slices (about four chunks per workgroup), and each pulse's F and
    gradient equal those of the same pulse evaluated alone."""
    B = 64
    cfg = synth.config1_batch(B)
    sysm = lib_system(cfg)
    amps = cfg["amps_batch"].astype(np.float32)
    st = np.tile(np.asarray(cfg["B"])[None, :], (B, 1))
    a = torch.tensor(amps.reshape(B * 4096, 2), device="cuda")
    F, g = sysm.fidelity_and_grad(a, [4096] * B, cfg["dt"], cfg["U_target"], static_coef=st)
    plan = sysm.last_plan()
    assert plan["total_slices"] == B * 4096 and plan["chunk_slices"] == 256
    F = F.cpu().numpy()
    g = g.cpu().numpy().reshape(B, 4096, 2).astype(np.float64)
    for i in (0, 17, 63):
        Fi, gi = sysm.fidelity_and_grad(torch.tensor(amps[i], device="cuda"), [4096], cfg["dt"],
                                        cfg["U_target"], static_coef=st[:1])
        assert abs(F[i] - Fi.cpu().numpy()[0]) <= 1e-6
        assert rel(g[i], gi.cpu().numpy().astype(np.float64)) <= 1e-4


def test_two_streams_different_inputs_back_to_back():
    """Two calls with different inputs on two streams, issued back to back with
    no host synchronisation: they share the context's workspace, so the second
    waits on the device for the first; each equals the same call made alone."""
    cfg_a = synth.small_case(35, n_slices=4096)
    cfg_b = synth.small_case(36, n_slices=300)
    sysm = lib_system(cfg_a, chunk=16)
    runs = []
    for cfg in (cfg_a, cfg_b):
        a = torch.tensor(rounded(cfg["amps"], "f32"), dtype=torch.float32, device="cuda")
        runs.append((a, [cfg["n_slices"]], cfg["dt"], cfg["U_target"],
                     np.asarray(cfg["B"])[None, :]))
    ref = [sysm.fidelity_and_grad(a, n, dt, U, static_coef=b) for a, n, dt, U, b in runs]
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for s in (s1, s2):
        s.wait_stream(torch.cuda.current_stream())
    out = []
    for s, (a, n, dt, U, b) in zip((s1, s2), runs):
        with torch.cuda.stream(s):
            out.append(sysm.fidelity_and_grad(a, n, dt, U, static_coef=b, stream=s))
    torch.cuda.synchronize()
    for (F, g), (Fr, gr) in zip(out, ref):
        assert torch.equal(F, Fr) and torch.equal(g, gr)


def test_overlapping_items_rejected_only_with_gradient():
    from paper_2511_13330_amd import LmagError
    cfg = synth.small_case(37, n_slices=16)
    sysm = lib_system(cfg, chunk=4)
    a = torch.tensor(rounded(cfg["amps"], "f32"), dtype=torch.float32, device="cuda")
    b = np.tile(np.asarray(cfg["B"])[None, :], (2, 1))
    with pytest.raises(LmagError, match="INVALID"):
        sysm.fidelity_and_grad(a, [10, 10], cfg["dt"], cfg["U_target"], slice_offset=[0, 5],
                               static_coef=b)
    F, _ = sysm.fidelity_and_grad(a, [10, 10], cfg["dt"], cfg["U_target"], slice_offset=[0, 5],
                                  static_coef=b, want_grad=False)
    for i, o in enumerate((0, 5)):
        Fi, _ = sysm.fidelity_and_grad(a[o:o + 10].contiguous(), [10], cfg["dt"], cfg["U_target"],
                                       static_coef=b[:1], want_grad=False)
        assert F[i].item() == Fi.item()


def test_rows_outside_items_get_zero_gradient():
    """Rows of amps that no item reads (here NaN) get a zero gradient from the
    binding and from the autograd backward."""
    from paper_2511_13330_amd import PulseFidelity
    cfg = synth.small_case(38, n_slices=20)
    sysm = lib_system(cfg, chunk=4)
    a = rounded(cfg["amps"], "f32").copy()
    a[[0, 1, 10, 11, 18, 19]] = np.nan
    amps = torch.tensor(a, dtype=torch.float32, device="cuda", requires_grad=True)
    b = np.tile(np.asarray(cfg["B"])[None, :], (2, 1))
    opts = {"slice_offset": [2, 12], "static_coef": b}
    F, g = sysm.fidelity_and_grad(amps.detach(), [8, 6], cfg["dt"], cfg["U_target"], **opts)
    assert torch.isfinite(F).all()
    outside = [0, 1, 10, 11, 18, 19]
    assert torch.count_nonzero(g[outside]) == 0
    F2 = PulseFidelity.apply(amps, sysm, [8, 6], cfg["dt"], cfg["U_target"], opts)
    (1.0 - F2).sum().backward()
    assert torch.isfinite(amps.grad).all()
    assert torch.count_nonzero(amps.grad[outside]) == 0
    assert torch.equal(amps.grad[2:10], -g[2:10])
