"""The learned proposal's gain: trained on pairs from the plain optimiser, its
proposals refined by the plain method reach F >= 0.999 more often and in fewer
iterations than a cold start on the same held-out targets."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_proposal_beats_cold_start():
    from paper_2511_13330_amd.proposal import run_experiment
    r = run_experiment(n_train=2000, n_test=256, epochs=15, refine_steps=40, log=lambda s: None)
    p, c = r["proposal_refine"], r["cold_start"]
    assert r["train_loss_last"] < r["train_loss_first"]
    assert p["mean_F_start"] > c["mean_F_start"]
    assert p["fraction_F_ge_0999"] > c["fraction_F_ge_0999"]
    assert p["median_iterations_to_0999"] < c["median_iterations_to_0999"]
