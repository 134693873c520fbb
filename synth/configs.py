"""Seeded workload generators (PCG64 via ``numpy.random.default_rng``).

Units: angular frequencies in rad/us, times in us (hbar = 1).

Every generator returns a plain dict of numpy arrays and scalars. The draw order
inside each generator is fixed, so a seed fully determines the workload.
"""
import numpy as np

TWO_PI = 2.0 * np.pi
A_MAX = TWO_PI * 20.0          # exchange amplitude ceiling, rad/us
B_RANGE = TWO_PI * 10.0        # Zeeman fields drawn from U[-B_RANGE, B_RANGE]
T1_US = 1000.0                 # relaxation time, us (1 ms)
T2_US = 2.0                    # dephasing time, us


def haar_unitary(rng, d):
    """Haar-random d x d unitary: QR of a complex Ginibre matrix with the
    diagonal phases of R moved into Q (Mezzadri 2007)."""
    re = rng.standard_normal((d, d))
    im = rng.standard_normal((d, d))
    z = (re + 1j * im) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return q * ph[None, :]


def _base(n_spins, n_slices, dt, order, hold, precision):
    return dict(n_spins=n_spins, d=2 ** n_spins, n_ctrl=n_spins - 1,
                n_slices=n_slices, dt=dt, order=order, hold=hold,
                precision=precision, T1=T1_US, T2=T2_US)


def config0(seed=0):
    """Three spins, 100 slices of 1 ns, ZOH first-order Magnus, FP64, forward."""
    rng = np.random.default_rng(seed)
    cfg = _base(3, 100, 1e-3, 1, "zoh", "f64")
    cfg["B"] = rng.uniform(-B_RANGE, B_RANGE, 3)
    cfg["amps"] = rng.uniform(0.0, A_MAX, (100, 2))
    cfg["U_target"] = haar_unitary(rng, 8)
    return cfg


def config1(seed=1):
    """Three spins, 4096 slices of 0.25 ns, FOH second-order Magnus, FP32,
    forward plus gradient; 32 finite-difference coordinates."""
    rng = np.random.default_rng(seed)
    cfg = _base(3, 4096, 2.5e-4, 2, "foh", "f32")
    cfg["B"] = rng.uniform(-B_RANGE, B_RANGE, 3)
    cfg["amps"] = rng.uniform(0.0, A_MAX, (4096, 2))
    cfg["U_target"] = haar_unitary(rng, 8)
    cfg["fd_coords"] = rng.choice(4096 * 2, 32, replace=False)
    return cfg


def config2(seed=2, n_cand=256, n_noise=64, n_min=512, n_max=4096):
    """Robust batch: candidates x quasi-static noise samples, uneven slice
    counts, FOH second order, FP32, shared target and nominal fields."""
    rng = np.random.default_rng(seed)
    cfg = _base(3, None, 2.5e-4, 2, "foh", "f32")
    cfg["B"] = rng.uniform(-B_RANGE, B_RANGE, 3)
    cfg["U_target"] = haar_unitary(rng, 8)
    n_sl = rng.integers(n_min, n_max + 1, n_cand)
    cfg["n_slices_per_cand"] = n_sl
    cfg["amps_per_cand"] = [rng.uniform(0.0, A_MAX, (int(n), 2)) for n in n_sl]
    cfg["dB"] = rng.normal(0.0, TWO_PI * 1.0, (n_noise, 3))
    cfg["eps"] = rng.normal(1.0, 0.01, (n_noise, 2))
    return cfg


def config3_four(seed=3):
    """Four spins (superoperator 256 x 256), 8192 slices of 0.25 ns, three
    exchange controls, FOH second order, FP32."""
    rng = np.random.default_rng(seed)
    cfg = _base(4, 8192, 2.5e-4, 2, "foh", "f32")
    cfg["B"] = rng.uniform(-B_RANGE, B_RANGE, 4)
    cfg["amps"] = rng.uniform(0.0, A_MAX, (8192, 3))
    cfg["U_target"] = haar_unitary(rng, 16)
    return cfg


def config3_six(seed=3):
    """Six spins (superoperator 4096 x 4096), 128 slices of 1 ns, five
    exchange controls, FOH second order, FP32."""
    rng = np.random.default_rng(seed + 1000)
    cfg = _base(6, 128, 1e-3, 2, "foh", "f32")
    cfg["B"] = rng.uniform(-B_RANGE, B_RANGE, 6)
    cfg["amps"] = rng.uniform(0.0, A_MAX, (128, 5))
    cfg["U_target"] = haar_unitary(rng, 64)
    return cfg


def hubbard3(seed=5, n_slices=128, dt=5e-4):
    """Hubbard model of three dots in a line (Eq. 1; 4 states per dot, Hilbert
    dimension 64, superoperator 4096 x 4096). The paper gives no parameter
    values; these are seeded synthetic draws in the units of the spin
    workloads: U~ ~ U[2pi 40, 2pi 60], V_i ~ U[-2pi 5, 2pi 5], U_C ~ U[2pi 5,
    2pi 10] (static coefficients, in the order U~, V_1, V_2, V_3, U_C) and
    hopping amplitudes t_12, t_23 ~ U[0, 2pi 10] per slice (the controls), FOH
    second order, slices of 0.5 ns, FP32, T1 = 1 ms and T2 = 2 us per dot."""
    rng = np.random.default_rng(seed)
    cfg = dict(n_dots=3, d=64, n_ctrl=2, n_slices=n_slices, dt=dt, order=2, hold="foh",
               precision="f32", T1=T1_US, T2=T2_US)
    cfg["coef"] = np.concatenate([rng.uniform(TWO_PI * 40, TWO_PI * 60, 1),
                                  rng.uniform(-TWO_PI * 5, TWO_PI * 5, 3),
                                  rng.uniform(TWO_PI * 5, TWO_PI * 10, 1)])
    cfg["amps"] = rng.uniform(0.0, TWO_PI * 10, (n_slices, 2))
    cfg["U_target"] = haar_unitary(rng, 64)
    return cfg


def config4_targets(seed=4, n=4096, n_slices=256, modes=4):
    """Learned-proposal workload: per target a nominal field vector, quasi-static
    noise scales (network inputs only) and a smooth reference pulse: for each
    control, A_MAX/2 (1 + sum_k a_k sin(pi k t / T + phi_k)) with
    sum_k |a_k| <= 1, so the pulse stays in [0, A_MAX]. The target unitary is
    the closed-system propagator of that pulse (reachable by construction); it
    is computed by whichever side consumes these draws."""
    rng = np.random.default_rng(seed)
    B = rng.uniform(-B_RANGE, B_RANGE, (n, 3))
    sigB = rng.uniform(0.0, TWO_PI * 1.0, n)
    sigJ = rng.uniform(0.0, 0.01, n)
    a = rng.uniform(-1.0, 1.0, (n, 2, modes))
    a /= np.maximum(1.0, np.abs(a).sum(axis=2, keepdims=True))
    phi = rng.uniform(0.0, TWO_PI, (n, 2, modes))
    t = (np.arange(n_slices) + 0.5) / n_slices
    k = np.arange(1, modes + 1)
    wave = np.sin(np.pi * k[None, None, :, None] * t[None, None, None, :] + phi[..., None])
    ref = 0.5 * A_MAX * (1.0 + np.einsum("ncm,ncmt->nct", a, wave))
    return dict(B=B, sigB=sigB, sigJ=sigJ, ref_amps=np.transpose(ref, (0, 2, 1)).copy(),
                n_slices=n_slices, dt=2.5e-4, d=8, n_spins=3, n_ctrl=2, order=2, hold="foh",
                precision="f32")


def small_case(seed, n_spins=3, n_slices=40, dt=2.5e-4, order=2, hold="foh",
               precision="f32", amp_max=A_MAX, T1=T1_US, T2=T2_US):
    """A small workload of the same distributions, for tests that the oracle
    must finish in seconds."""
    rng = np.random.default_rng(seed)
    cfg = _base(n_spins, n_slices, dt, order, hold, precision)
    cfg["T1"], cfg["T2"] = T1, T2
    cfg["B"] = rng.uniform(-B_RANGE, B_RANGE, n_spins)
    cfg["amps"] = rng.uniform(0.0, amp_max, (n_slices, n_spins - 1))
    cfg["U_target"] = haar_unitary(rng, 2 ** n_spins)
    return cfg


def config1_batch(n_pulses, seed=1):
    """n_pulses config-1 pulses sharing fields and target: pulse 0 is exactly
    config1(seed)'s pulse, the others are fresh draws of the same distribution."""
    cfg = config1(seed)
    rng = np.random.default_rng(seed + 7919)
    extra = rng.uniform(0.0, A_MAX, (max(0, n_pulses - 1), 4096, 2))
    cfg["amps_batch"] = np.concatenate([cfg["amps"][None], extra], axis=0)[:n_pulses]
    return cfg
