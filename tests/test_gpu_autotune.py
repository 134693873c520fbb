"""Autotuner of the persistent slice kernels: picks a (chunk, inverse) pair that
the next untuned-size call uses, records it, and every variant keeps parity."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from helpers import lib_system, oracle_system, rounded, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_autotune_choice_is_used_and_keeps_parity(tmp_path, monkeypatch):
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("LMAG_TUNE_CACHE", str(cache))
    cfg = synth.small_case(61, n_slices=256)
    amps = rounded(cfg["amps"], "f32")
    sysm = lib_system(cfg)
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    C, inv, ms = sysm.autotune(a, [256], cfg["dt"], cfg["U_target"], static_coef=b, reps=1)
    assert C >= 1 and inv in (0, 1, 2) and ms > 0
    F, g = sysm.fidelity_and_grad(a, [256], cfg["dt"], cfg["U_target"], static_coef=b)
    assert sysm.last_plan()["chunk_slices"] == C
    Fr, gr = oracle.grad_adjoint(oracle_system(cfg), amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F.item() - Fr) < 1e-6 and rel(g.cpu().numpy(), gr) < 1e-4
    line = json.loads(cache.read_text().strip().splitlines()[-1])
    assert line["chunk"] == C and line["variant"] == inv
    fresh = lib_system(cfg)
    fresh.load_tuning(cache)
    fresh.fidelity_and_grad(a, [256], cfg["dt"], cfg["U_target"], static_coef=b)
    assert fresh.last_plan()["chunk_slices"] == C


@pytest.mark.parametrize("basis", ["hermitian", "column"])
@pytest.mark.parametrize("inverse", [0, 1, 2])
def test_each_inverse_variant_keeps_parity(tmp_path, inverse, basis):
    # 0: power series / Neumann / Gauss-Jordan chosen per slice; 1: Gauss-Jordan;
    # 2: Neumann or Gauss-Jordan. Forced through a tuning line for this size.
    cfg = synth.small_case(62, n_slices=48)
    amps = rounded(cfg["amps"], "f32")
    total = 48
    key = f"p32{'h' if basis == 'hermitian' else ''}_o2_d8_s{int(np.floor(np.log2(total)))}"
    f = tmp_path / "t.jsonl"
    f.write_text(json.dumps({"key": key, "chunk": 7, "inverse": inverse, "ms": 1.0}) + "\n")
    sysm = lib_system(cfg, basis=basis)
    sysm.load_tuning(f)
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    F, g = sysm.fidelity_and_grad(a, [total], cfg["dt"], cfg["U_target"],
                                  static_coef=np.asarray(cfg["B"])[None, :])
    assert sysm.last_plan()["chunk_slices"] == 7
    Fr, gr = oracle.grad_adjoint(oracle_system(cfg), amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F.item() - Fr) < 1e-7 and rel(g.cpu().numpy(), gr) < 1e-4
