"""Matrix exponential and its Frechet derivative (oracle), Eq. 14.

expm_taylor: scaling and squaring with a truncated Taylor series in float64.
The scaling exponent s makes ||A / 2^s||_1 <= 1/2; terms are added until a term
is below 1e-18 of the partial sum in 1-norm; the result is squared s times.
This is on purpose a different algorithm from the Pade approximant of the GPU.

frechet_block: the Frechet derivative L(A, E) read off the upper-right block of
exp([[A, E], [0, A]]) (the block-triangular identity).
"""
import numpy as np


def _norm1(A):
    return float(np.max(np.sum(np.abs(A), axis=0))) if A.size else 0.0


def expm_taylor(A):
    A = np.asarray(A, dtype=complex)
    n = A.shape[0]
    nrm = _norm1(A)
    s = 0
    if nrm > 0.5:
        s = int(np.ceil(np.log2(nrm / 0.5)))
    X = A / (2.0 ** s)
    I = np.eye(n, dtype=complex)
    total = I.copy()
    term = I.copy()
    for k in range(1, 80):
        term = term @ X / k
        total = total + term
        if _norm1(term) <= 1e-18 * _norm1(total):
            break
    for _ in range(s):
        total = total @ total
    return total


def frechet_block(A, E):
    """L(A, E) = d/dt exp(A + t E) at t = 0, via the 2n x 2n block matrix.
    E is normalised to the norm of A first (L is linear in E)."""
    A = np.asarray(A, dtype=complex)
    E = np.asarray(E, dtype=complex)
    n = A.shape[0]
    ne = _norm1(E)
    if ne == 0.0:
        return np.zeros_like(E)
    scale = max(_norm1(A), 1e-3) / ne
    big = np.zeros((2 * n, 2 * n), dtype=complex)
    big[:n, :n] = A
    big[n:, n:] = A
    big[:n, n:] = E * scale
    return expm_taylor(big)[:n, n:] / scale
