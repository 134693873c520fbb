"""The entry point that allocates nothing (lmag_fidelity_and_grad_noalloc)
against lmag_fidelity_and_grad, through the C ABI: two calls in a row, the
second with a smaller batch, each equal to the allocating call on the same
inputs; a batch over the fixed scratch is rejected before any launch."""
import numpy as np
import pytest

import synth
from helpers import lib_system, rounded

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _inputs(cfg, n_items, prec):
    a = np.concatenate([rounded(np.roll(cfg["amps"], 3 * i, axis=0), prec) for i in range(n_items)])
    rdt = torch.float32 if prec == "f32" else torch.float64
    amps = torch.tensor(a, dtype=rdt, device="cuda")
    b = torch.tensor(np.tile(np.asarray(cfg["B"])[None, :], (n_items, 1)), dtype=torch.float64,
                     device="cuda")
    UT = torch.tensor(cfg["U_target"], dtype=torch.complex128, device="cuda")
    return amps, [cfg["n_slices"]] * n_items, b, UT


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_allocating_call_twice(prec):
    cfg = synth.small_case(61, n_slices=40)
    sysm = lib_system(cfg, prec, 2, "foh", chunk=16)
    for n_items in (3, 1):        # the second call is smaller
        amps, ns, b, UT = _inputs(cfg, n_items, prec)
        F_ref, g_ref = sysm.fidelity_and_grad(amps, ns, cfg["dt"], UT, static_coef=b)
        F = torch.full((n_items,), float("nan"), dtype=torch.float64, device="cuda")
        g = torch.full_like(amps, float("nan"))
        sysm.fidelity_and_grad_noalloc(amps, ns, cfg["dt"], UT, F, g, static_coef=b)
        torch.cuda.synchronize()
        assert torch.equal(F, F_ref)
        assert torch.equal(g, g_ref)
        # F only
        F2 = torch.zeros_like(F)
        sysm.fidelity_and_grad_noalloc(amps, ns, cfg["dt"], UT, F2, None, static_coef=b)
        assert torch.equal(F2, F_ref)


def test_noalloc_rejects_batch_over_scratch():
    from paper_2511_13330_amd import LmagError
    cfg = synth.small_case(62, n_slices=2048)
    sysm = lib_system(cfg, "f32", 2, "foh")
    amps, ns, b, UT = _inputs(cfg, 1, "f32")
    F = torch.full((1,), -7.0, dtype=torch.float64, device="cuda")
    g = torch.full_like(amps, -7.0)
    with pytest.raises(LmagError, match="INVALID"):
        sysm.fidelity_and_grad_noalloc(amps, ns, cfg["dt"], UT, F, g, static_coef=b)
    torch.cuda.synchronize()
    assert (F == -7.0).all() and (g == -7.0).all()
