"""Unit tests of the register-tile primitives through the C ABI debug entry
points: complex 64x64 products, the Gauss-Jordan inverse and the scaled Pade
exponential, against numpy / scipy on the same inputs."""
import numpy as np
import pytest
import scipy.linalg as sla

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TDT = {"f32": torch.complex64, "f64": torch.complex128}
TOL = {"f32": 2e-6, "f64": 1e-13}


@pytest.fixture(scope="module")
def ctx_system():
    from paper_2511_13330_amd import spin_chain_system
    return spin_chain_system(3, precision="f32", magnus_order=1, hold="zoh")


def rnd(rng, scale=1.0):
    return scale * (rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64)))


def dev(x, prec):
    return torch.tensor(x, dtype=TDT[prec], device="cuda")


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("trans", [False, True])
def test_tile_gemm(ctx_system, prec, trans):
    rng = np.random.default_rng(1)
    A, B = rnd(rng), rnd(rng)
    C = ctx_system.debug_tile_gemm(dev(A, prec), dev(B, prec), transA=trans, precision=prec)
    ref = (A.T if trans else A) @ B
    err = np.linalg.norm(C.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < TOL[prec], err


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_tile_inverse(ctx_system, prec):
    rng = np.random.default_rng(2)
    R = rnd(rng)
    A = np.eye(64) + 0.4 * R / np.abs(R).sum(0).max()      # ||I - A||_1 = 0.4
    C = ctx_system.debug_tile_inverse(dev(A, prec), precision=prec).cpu().numpy()
    ref = np.linalg.inv(A)
    err = np.linalg.norm(C - ref) / np.linalg.norm(ref)
    assert err < 5 * TOL[prec], err


@pytest.mark.parametrize("prec,norm,m,s", [
    ("f32", 0.05, 2, 0), ("f32", 0.08, 2, 0), ("f32", 0.4, 3, 0), ("f32", 3.0, 3, 3),
    ("f64", 0.01, 3, 0), ("f64", 0.2, 5, 0), ("f64", 0.9, 7, 0), ("f64", 6.0, 7, 3)])
def test_tile_expm(ctx_system, prec, norm, m, s):
    rng = np.random.default_rng(3)
    A = rnd(rng)
    A *= norm / np.abs(A).sum(0).max()
    C, ms = ctx_system.debug_tile_expm(dev(A, prec), precision=prec)
    ref = sla.expm(A)
    err = np.linalg.norm(C.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert tuple(ms.cpu().numpy().tolist()) == (m, s)
    assert err < (20 * TOL[prec] * (1 + s)), err


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("n,batch", [(128, 3), (256, 5), (1024, 2), (4096, 1)])
def test_block_product_kernels(ctx_system, variant, n, batch):
    """Every block-tiled product kernel against an FP64 product of the same
    FP32 inputs (a kernel whose shape condition fails runs kernel 0)."""
    g = torch.Generator(device="cuda").manual_seed(1000 + n + variant)
    A = torch.randn(batch, n, n, dtype=torch.complex64, device="cuda", generator=g)
    B = torch.randn(batch, n, n, dtype=torch.complex64, device="cuda", generator=g)
    C = ctx_system.debug_block_gemm(A, B, variant=variant)
    ref = torch.matmul(A.to(torch.complex128), B.to(torch.complex128))
    err = (torch.linalg.matrix_norm(C.to(torch.complex128) - ref) / torch.linalg.matrix_norm(ref)).max().item()
    # FP32 accumulation over n terms: about sqrt(n) u relative (u = 6e-8)
    assert err < 4e-8 * np.sqrt(n) * 4, err
