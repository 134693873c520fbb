"""Host-only checks of bench.py: it refuses more than one GPU, and its
algorithmic flop counts per slice are the products the kernels run."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

M = 8.0 * 64 ** 3   # one complex 64 x 64 x 64 product in real flops


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_flops_per_slice():
    # forward, Padé-2 by its degree-4 series: A^2, the series product, the chain
    assert bench.forward_flops_per_slice(2, 0) == 3 * M
    # forward, Padé-3 with s squarings: A^2, U, an n x n solve (4/3), D, s
    # squarings, the chain
    assert bench.forward_flops_per_slice(3, 2) == (2 + 2 + 4.0 / 3.0 + 1) * M
    # backward: M_n, Z update, 2 pi_m for the Frechet derivative, 2 more, 2 per squaring
    assert bench.backward_flops_per_slice(2, 0) == 6 * M
    assert bench.backward_flops_per_slice(3, 1) == 10 * M


def test_flops_from_histogram():
    h = np.zeros((4, 64), dtype=np.int64)
    h[0, 0] = 10   # m = 2, s = 0
    h[1, 3] = 2    # m = 3, s = 3
    f = bench.flops_from_hist(h, bench.forward_flops_per_slice)
    assert f == 10 * 3 * M + 2 * (2 + 3 + 4.0 / 3.0 + 1) * M


def test_pooled_cpu_baseline_is_the_oracle_adjoint():
    """The benchmark's CPU baseline runs the oracle's per-slice steps in a
    process pool; its F and gradient are those of oracle.grad_adjoint."""
    import oracle
    import synth
    cfg = synth.small_case(77, n_slices=37)
    cb, F, g = bench.cpu_baseline(cfg)
    amps = cfg["amps"].astype(np.float32).astype(np.float64)
    F_ref, g_ref = oracle.grad_adjoint(oracle.System.from_cfg(cfg), amps, cfg["dt"], 2, "foh",
                                       cfg["U_target"])
    assert abs(F - F_ref) < 1e-14
    assert np.allclose(g, g_ref, rtol=1e-12, atol=1e-16)
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0
