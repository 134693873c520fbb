"""Workspace budget: waves of items and the recompute mode of the adjoint give
bitwise the same results as the unconstrained call (same chunking)."""
import numpy as np
import pytest

import synth
from helpers import lib_system, rounded

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(cfg, amps, ns, budget, chunk, prec="f32"):
    sysm = lib_system(cfg, prec, chunk=chunk, workspace_bytes_max=budget)
    b = np.tile(np.asarray(cfg["B"])[None, :], (len(ns), 1))
    dt = torch.float32 if prec == "f32" else torch.float64
    F, g = sysm.fidelity_and_grad(torch.tensor(amps, dtype=dt, device="cuda"), ns, cfg["dt"],
                                  cfg["U_target"], static_coef=b)
    return F.cpu().numpy(), g.cpu().numpy(), sysm.last_plan()


def test_waves_match_single_call():
    cfg = synth.small_case(51, n_slices=200)
    amps = rounded(cfg["amps"], "f32")
    ns = [40] * 5
    F0, g0, p0 = run(cfg, amps, ns, 0, 4)
    F1, g1, p1 = run(cfg, amps, ns, 16 << 20, 4)
    assert p0["waves"] == 1 and p1["waves"] > 1
    assert np.array_equal(F0, F1) and np.array_equal(g0, g1)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_recompute_matches_stored(prec):
    cfg = synth.small_case(52, n_slices=600)
    amps = rounded(cfg["amps"], prec)
    F0, g0, p0 = run(cfg, amps, [600], 0, 2, prec)
    budget = 100 << 20 if prec == "f32" else 200 << 20
    F1, g1, p1 = run(cfg, amps, [600], budget, 2, prec)
    assert p0["recompute"] == 0 and p1["recompute"] == 1
    assert p1["grid"] < p0["grid"]
    assert p0["sparse_support"] > 0   # compact K_n^T shares the tiles the recompute reads
    assert np.array_equal(F0, F1) and np.array_equal(g0, g1)


def test_budget_too_small_is_nomem():
    from paper_2511_13330_amd import LmagError
    cfg = synth.small_case(53, n_slices=64)
    with pytest.raises(LmagError, match="NOMEM"):
        run(cfg, rounded(cfg["amps"], "f32"), [64], 1 << 20, 8)
