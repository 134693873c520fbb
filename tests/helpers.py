"""Shared test helpers: build the library system and the oracle system from the
same seeded scalars, and call the library through the binding."""
import numpy as np

import oracle


def oracle_system(cfg, dissipative=True, eps=None, dB=None):
    return oracle.System.from_cfg(cfg, dissipative=dissipative, eps=eps, dB=dB)


def lib_system(cfg, precision=None, order=None, hold=None, dissipative=True, chunk=0,
               workspace_bytes_max=0, basis="hermitian"):
    from paper_2511_13330_amd import spin_chain_system
    T1, T2 = (cfg["T1"], cfg["T2"]) if dissipative else (np.inf, np.inf)
    return spin_chain_system(cfg["n_spins"], T1, T2,
                             precision=precision or cfg["precision"],
                             magnus_order=order or cfg["order"], hold=hold or cfg["hold"],
                             chunk_slices=chunk, workspace_bytes_max=workspace_bytes_max,
                             basis=basis)


def rounded(amps, precision):
    """The amplitudes the kernel actually sees (FP32 rounding for FP32 runs)."""
    a = np.asarray(amps, dtype=np.float64)
    return a.astype(np.float32).astype(np.float64) if precision == "f32" else a


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def hermitian_basis_change(d):
    """T with (T S T^dag) real for every Hermiticity-preserving superoperator S
    in column stacking (vec(rho)[k + l d] = rho[k, l]): row k + l d is the
    coordinate on |k><k| (k = l), on (|k><l| + |l><k|) / sqrt 2 (k < l) or on
    i (|l><k| - |k><l|) / sqrt 2 (k > l)."""
    n = d * d
    T = np.zeros((n, n), dtype=complex)
    h = np.sqrt(0.5)
    for a in range(n):
        k, l = a % d, a // d
        q = l + k * d
        if k == l:
            T[a, a] = 1.0
        elif k < l:
            T[a, a], T[a, q] = h, h
        else:
            T[a, a], T[a, q] = 1j * h, -1j * h
    return T
