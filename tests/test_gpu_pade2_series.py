"""FP32 Padé-2 slices evaluate r_2(A) by its power series cut at degree 4 (the
default inverse variant). The Neumann/Gauss-Jordan variant forms r_2 = q_2^{-1} p_2
instead. At the full 4096-slice pulse both must give the same propagator,
fidelity and gradient to FP32 accuracy, and the series path must cover the
Padé-2 slices."""
import json

import numpy as np
import pytest

import oracle
import synth
from helpers import lib_system, oracle_system, rounded, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 4096


def _system(cfg, variant, tmp_path, basis, dissipative=True):
    sysm = lib_system(cfg, dissipative=dissipative, basis=basis)
    key = f"p32{'h' if basis == 'hermitian' else ''}_o2_d8_s{int(np.floor(np.log2(N)))}"
    f = tmp_path / f"tune{variant}.jsonl"
    f.write_text(json.dumps({"key": key, "chunk": 16, "inverse": variant, "ms": 1.0}) + "\n")
    sysm.load_tuning(f)
    return sysm


@pytest.mark.parametrize("basis", ["hermitian", "column"])
def test_series_and_inverse_forms_agree(tmp_path, basis):
    cfg = synth.config1()
    amps = rounded(cfg["amps"], "f32")
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    out = {}
    for v in (0, 2):
        sysm = _system(cfg, v, tmp_path, basis)
        S = sysm.propagate(a, [N], cfg["dt"], static_coef=b).cpu().numpy()[0]
        F, g = sysm.fidelity_and_grad(a, [N], cfg["dt"], cfg["U_target"], static_coef=b)
        assert sysm.last_plan()["chunk_slices"] == 16
        out[v] = (S, F.item(), g.cpu().numpy(), sysm.selection_histogram())
    hist = out[0][3]
    # Padé-2 slices dominate this workload (in the real basis the 1-norms are
    # larger and about 7 % of the slices take Padé-3)
    assert hist[0].sum() >= (0.9 if basis == "hermitian" else 0.99) * hist.sum()
    assert (hist == out[2][3]).all()            # the (m, s) choice does not depend on the variant
    assert rel(out[0][0], out[2][0]) <= 5e-6
    assert abs(out[0][1] - out[2][1]) <= 2e-7
    assert rel(out[0][2], out[2][2]) <= 1e-5


@pytest.mark.parametrize("basis", ["hermitian", "column"])
def test_series_form_at_unit_fidelity(tmp_path, basis):
    # closed system, target = the oracle's own propagator (F = 1), where a
    # non-unitary drift of the slice map shows first order in F
    cfg = synth.config1()
    amps = rounded(cfg["amps"], "f32")
    osys = oracle_system(cfg, dissipative=False)
    S_ref = oracle.propagate(osys.omegas(amps, cfg["dt"], 2, "foh"))
    d = 8
    tgt = S_ref[:d, :d] / np.abs(np.linalg.det(S_ref[:d, :d])) ** (1.0 / d)
    F_ref, _ = oracle.fidelity(S_ref, tgt)
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    for v in (0, 2):
        sysm = _system(cfg, v, tmp_path, basis, dissipative=False)
        F, _ = sysm.fidelity_and_grad(a, [N], cfg["dt"], tgt, static_coef=b)
        assert abs(F.item() - F_ref) <= 1e-6, (v, F.item() - F_ref)
