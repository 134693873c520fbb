"""Host-only checks of the C ABI: the library loads without a GPU, exports every
symbol include/lmag.h declares, and its Pade constants satisfy their defining
properties (computed here from exact rational series, not from the library)."""
import ctypes
import os
import re
from fractions import Fraction as Fr
from math import factorial

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmag.h")


@pytest.fixture(scope="module")
def L():
    from paper_2511_13330_amd import lib
    return lib()


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lmag_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported(L):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s


def test_binding_covers_header():
    from paper_2511_13330_amd._lib import SIGNATURES
    assert sorted(SIGNATURES) == declared_symbols()


def exact_pade(m):
    return [Fr(factorial(2 * m - j) * factorial(m), factorial(2 * m) * factorial(j) * factorial(m - j))
            for j in range(m + 1)]


@pytest.mark.parametrize("m", [2, 3, 5, 7])
def test_pade_coefficients(L, m):
    b = (ctypes.c_double * (m + 1))()
    assert L.lmag_pade_coefficients(m, b) == 0
    ex = exact_pade(m)
    assert np.allclose(list(b), [float(x) for x in ex], rtol=1e-15, atol=0)
    # r_m(x) = p(x)/p(-x) agrees with exp(x) to order 2m: error ~ C x^(2m+1)
    for x in (1e-2, 2e-2):
        p = sum(float(bj) * x ** j for j, bj in enumerate(ex))
        q = sum(float(bj) * (-x) ** j for j, bj in enumerate(ex))
        assert abs(p / q - np.exp(x)) < 10 * x ** (2 * m + 1) + 1e-15


def _series_mul(a, b, K):
    out = [Fr(0)] * K
    for i, x in enumerate(a[:K]):
        if x:
            for j, y in enumerate(b[:K - i]):
                out[i + j] += x * y
    return out


def _log1p_series(a, K):
    out, p = [Fr(0)] * K, [Fr(1)] + [Fr(0)] * (K - 1)
    for k in range(1, K):
        p = _series_mul(p, a, K)
        for i in range(K):
            out[i] += Fr((-1) ** (k + 1), k) * p[i]
    return out


def backward_error_bound(m, theta, K=None):
    """h(theta)/theta with h the absolute-coefficient series of
    log(exp(-x) r_m(x)) (Higham 2005): the relative backward error bound."""
    K = K or 2 * m + 60
    b = exact_pade(m)
    p = b + [Fr(0)] * (K - len(b))
    q = [bj * (-1) ** j for j, bj in enumerate(b)] + [Fr(0)] * (K - len(b))
    lp = _log1p_series([Fr(0)] + p[1:K], K)
    lq = _log1p_series([Fr(0)] + q[1:K], K)
    c = [lp[i] - lq[i] for i in range(K)]
    c[1] -= 1
    assert all(ci == 0 for ci in c[:2 * m + 1])
    return sum(abs(float(ci)) * theta ** k for k, ci in enumerate(c)) / theta


@pytest.mark.parametrize("prec,m,u", [(32, 2, 2.0 ** -24), (32, 3, 2.0 ** -24), (64, 3, 2.0 ** -53),
                                      (64, 5, 2.0 ** -53), (64, 7, 2.0 ** -53)])
def test_theta_is_the_unit_roundoff_threshold(L, prec, m, u):
    t = ctypes.c_double()
    assert L.lmag_pade_theta(prec, m, ctypes.byref(t)) == 0
    th = t.value
    assert abs(backward_error_bound(m, th) / u - 1) < 1e-6
    assert backward_error_bound(m, th * (1 + 1e-4)) > u
    # the denominator q_m(A) stays column diagonally dominant for ||A||_1 <= theta,
    # which is why the library's Gauss-Jordan inverse needs no pivoting
    b = exact_pade(m)
    assert sum(float(bj) * th ** j for j, bj in enumerate(b) if j >= 1) < 1.0


def test_create_without_gpu_reports_device_error(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    assert L.lmag_create(ctypes.byref(ctx), 0) == -4
