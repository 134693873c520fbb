"""A system whose superoperator is not a power-of-two number of tiles: d = 24,
n = 576 = 9 x 64 (nine tile rows; the two-tile kernel and the XCD grouping
fall back where their shape conditions fail), with random Hermitian static and
control terms and two jump operators, through every block-tiled product
kernel in both representations, element by element against the oracle (propagator, F and the whole
gradient), with slices at Pade degree 2 and 3 and with squarings."""
import numpy as np
import pytest

import oracle
from helpers import rounded, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

D = 24


def hermitian(rng, scale):
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    H = (X + X.conj().T) / 2
    return scale * H / np.linalg.norm(H, 2)


def case(seed=91, n_slices=8, dt=2e-3):
    rng = np.random.default_rng(seed)
    Hs = [hermitian(rng, 2 * np.pi * 10) for _ in range(2)]
    Hc = [hermitian(rng, 2 * np.pi * 20) for _ in range(2)]
    Ls = []
    for rate in (0.5, 0.2):
        X = np.triu(rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D)), 1)
        Ls.append(np.sqrt(rate) * X / np.linalg.norm(X, 2))
    coef = rng.uniform(-0.1, 0.1, 2)
    # weak controls in the first half, strong in the second: Pade degree 2 on
    # the first slices, degree 3 with squarings on the last
    amps = rng.uniform(0.0, 0.01, (n_slices, 2))
    amps[n_slices // 2:] = rng.uniform(0.5, 1.0, (n_slices - n_slices // 2, 2))
    X = rng.standard_normal((D, D)) + 1j * rng.standard_normal((D, D))
    Q, R = np.linalg.qr(X)
    UT = Q * (np.diag(R) / np.abs(np.diag(R)))
    return Hs, Hc, Ls, coef, amps, dt, UT


class Generic(oracle.System):
    """Oracle system with given static terms (coefficients per item), control
    terms and jump operators."""

    def __init__(self, Hs, Hc, Ls, coef):
        self.d = D
        self.n_ctrl = len(Hc)
        self.B = np.asarray(coef, float)
        self.eps = np.ones(self.n_ctrl)
        self.Hc, self.Hs, self.Ls = Hc, Hs, Ls

    def H(self, u):
        H = np.zeros((D, D), dtype=complex)
        for c, hc in enumerate(self.Hc):
            H += self.eps[c] * u[c] * hc
        for i, hs in enumerate(self.Hs):
            H += self.B[i] * hs
        return H


@pytest.fixture(scope="module")
def reference():
    Hs, Hc, Ls, coef, amps, dt, UT = case()
    amps = rounded(amps, "f32")
    osys = Generic(Hs, Hc, Ls, coef)
    U_ref = oracle.propagate(osys.omegas(amps, dt, 2, "foh"))
    F_ref, g_ref = oracle.grad_adjoint(osys, amps, dt, 2, "foh", UT)
    return (Hs, Hc, Ls, coef, amps, dt, UT), U_ref, F_ref, g_ref


@pytest.mark.parametrize("basis,variant", [("column", v) for v in (0, 4, 5, 6, 7, 8)] +
                         [("hermitian", v) for v in (0, 1, 2, 5, 7)])
def test_nine_tile_rows_every_product_kernel(reference, basis, variant, tmp_path):
    from paper_2511_13330_amd.system import System
    (Hs, Hc, Ls, coef, amps, dt, UT), U_ref, F_ref, g_ref = reference
    sysm = System(Hs, Hc, Ls, precision="f32", magnus_order=2, hold="foh", basis=basis)
    N = len(amps)
    with open(tmp_path / "tune.jsonl", "w") as f:
        f.write('{"key": "p32%s_o2_d%d_s%d", "chunk": 3, "variant": %d, "ms": 0.0}\n'
                % ("h" if basis == "hermitian" else "", D, int(np.floor(np.log2(N))), variant))
    sysm.load_tuning(str(tmp_path / "tune.jsonl"))
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    st = np.asarray(coef)[None, :]
    U = sysm.propagate(a, [N], dt, static_coef=st).cpu().numpy()[0].astype(complex)
    hist = sysm.selection_histogram()
    # m = 3 with s > 0 on the strong slices; in column stacking the weak ones sit
    # at m = 2 (the 1-norm, and so the selection, depends on the representation)
    assert hist[1, 1:].sum() > 0
    if basis == "column":
        assert hist[0].sum() > 0
    assert rel(U, U_ref) < 1e-4
    F, g = sysm.fidelity_and_grad(a, [N], dt, UT, static_coef=st)
    assert abs(F.item() - F_ref) < 1e-6
    assert rel(g.cpu().numpy().astype(float), g_ref) < 1e-3
