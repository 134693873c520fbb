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
    assert C >= 1 and inv in (0, 1) and ms > 0
    F, g = sysm.fidelity_and_grad(a, [256], cfg["dt"], cfg["U_target"], static_coef=b)
    assert sysm.last_plan()["chunk_slices"] == C
    Fr, gr = oracle.grad_adjoint(oracle_system(cfg), amps, cfg["dt"], 2, "foh", cfg["U_target"])
    assert abs(F.item() - Fr) < 1e-6 and rel(g.cpu().numpy(), gr) < 1e-4
    line = json.loads(cache.read_text().strip().splitlines()[-1])
    assert line["chunk"] == C and line["inverse"] == inv
    fresh = lib_system(cfg)
    fresh.load_tuning(cache)
    fresh.fidelity_and_grad(a, [256], cfg["dt"], cfg["U_target"], static_coef=b)
    assert fresh.last_plan()["chunk_slices"] == C
