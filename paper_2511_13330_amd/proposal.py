"""Learned pulse proposal end to end: reachable targets, training pairs from the
plain optimiser, training of the proposal network, and proposal + refine
against a cold start and against the training data's mean pulse, with the
plain method as the judge and the fallback. Every numerical step runs in the
library's kernels; this module only sequences them.

Targets follow the reachable-by-construction reading of the proposal workload:
the closed-system propagator of a smooth reference pulse (0.25 ns FOH slices,
second-order Magnus) with the target's own Zeeman fields; noise scales are
network inputs only and success is judged at zero noise. The training pairs are
the plain optimiser's results started from each reference pulse perturbed by
Gaussian noise (0.3 A_max, clipped to [0, A_max]).
"""
import time

import numpy as np
import torch

from .mlp import ProposalMLP, features
from .optim import refine, cold_start
from .system import spin_chain_system


def closed_system(precision="f32", chunk=0):
    return spin_chain_system(3, np.inf, np.inf, precision=precision, magnus_order=2, hold="foh",
                             chunk_slices=chunk)


def target_unitaries(system, ref_amps, B, dt):
    """U_T of every reference pulse from the library's superoperator propagator.
    For this exchange + Zeeman chain |up up up> spans a one-dimensional S_z
    sector, so U[0][0] is a pure phase and S[i][k] = conj(U[0][0]) U[i][k] for
    i, k < d (column-stacking): the top-left d x d block of S is U_T up to a
    global phase, which the fidelity ignores."""
    n, N, nc = ref_amps.shape
    out = []
    for s in range(0, n, 2048):
        e = min(n, s + 2048)
        a = torch.tensor(ref_amps[s:e].reshape(-1, nc), dtype=system.rdtype,
                         device=system.device).contiguous()
        S = system.propagate(a, [N] * (e - s), dt, static_coef=B[s:e])
        out.append(S[:, :system.d, :system.d].to(torch.complex128).cpu().numpy())
    return np.concatenate(out)


def optimised_pulses(system, U, B, start, dt, max_steps=60, lr=2.0, amax=None, target=0.999):
    """The plain optimiser (fused forward+adjoint and Adam + projection) from
    `start`; returns the final pulses, fidelities and iterations to target."""
    n, N, nc = start.shape
    amps = torch.tensor(start.reshape(-1, nc), dtype=system.rdtype, device=system.device)
    out = refine(system, amps, [N] * n, dt, U, max_steps=max_steps, lr=lr, amax=amax,
                 target=target, static_coef=B, target_of_item=np.arange(n))
    return amps.reshape(n, N, nc), out


def propose_and_refine(system, start, n_slices, dt, U, B, refine_steps=50, fallback_steps=200,
                       lr=2.0, amax=None, target=0.999, seed=0):
    """Refine proposed pulses with the plain method, judge them with the plain
    propagator, and fall back to the plain method from a cold start where the
    proposal failed.

    start: [n, N, n_ctrl] proposals (a learned network's output, or any start).
    Every item is refined for up to refine_steps iterations (fused
    forward+adjoint and Adam + projection). Items whose final fidelity is below
    target or not finite (a non-finite proposal stays non-finite) restart from
    uniform random amplitudes in [0, amax] and are refined for up to
    fallback_steps iterations. Returns the final pulses [n, N, n_ctrl], their
    fidelities from the plain propagator, the source of each (0: proposal +
    refine, 1: fallback) and the iteration count of each path."""
    n, N, nc = start.shape
    dev = system.device
    amps = torch.as_tensor(start, dtype=system.rdtype, device=dev).reshape(-1, nc).clone()
    first = refine(system, amps, [N] * n, dt, U, max_steps=refine_steps, lr=lr, amax=amax,
                   target=target, static_coef=B, target_of_item=np.arange(n))
    F = np.asarray(first["F"], dtype=float).copy()
    fail = ~(np.isfinite(F) & (F >= target))
    source = np.zeros(n, dtype=np.int64)
    out = amps.reshape(n, N, nc)
    fb = None
    if fail.any():
        idx = np.nonzero(fail)[0]
        a2 = cold_start(len(idx), N, nc, amax if amax is not None else 1.0, seed, device=dev,
                        dtype=system.rdtype)
        fb = refine(system, a2, [N] * len(idx), dt, U[idx], max_steps=fallback_steps, lr=lr,
                    amax=amax, target=target, static_coef=B[idx], target_of_item=np.arange(len(idx)))
        out[torch.as_tensor(idx, device=dev)] = a2.reshape(len(idx), N, nc)
        F[idx] = fb["F"]
        source[idx] = 1
    return {"amps": out, "F": F, "source": source, "refine": first, "fallback": fb}


def run_experiment(n_train=20000, n_test=4096, seed=4, epochs=20, refine_steps=50, lr=2.0,
                   train_lr=1e-3, fallback_steps=200, log=print):
    """Returns a dict with the training summary and, on held-out targets, the
    fraction reaching F >= 0.999 and the time to fidelity for proposal+refine
    and for a cold start."""
    import synth
    amax = synth.A_MAX
    sysm = closed_system()
    cfg = synth.config4_targets(seed, n=n_train + n_test)
    dt, N = cfg["dt"], cfg["n_slices"]
    t0 = time.perf_counter()
    U = target_unitaries(sysm, cfg["ref_amps"], cfg["B"], dt)
    rng = np.random.default_rng(seed + 1)
    tr = slice(0, n_train)
    te = slice(n_train, n_train + n_test)
    # training pairs: the plain optimiser from a perturbed reference
    start = np.clip(cfg["ref_amps"][tr] + rng.normal(0, 0.3 * amax, cfg["ref_amps"][tr].shape),
                    0, amax)
    pulses, opt = optimised_pulses(sysm, U[tr], cfg["B"][tr], start, dt, lr=lr, amax=amax)
    ok = opt["F"] >= 0.999
    t_data = time.perf_counter() - t0
    log(f"training data: {ok.sum()}/{n_train} pairs reached F >= 0.999 in {t_data:.1f} s")
    X = torch.tensor(features(U, cfg["B"], cfg["sigB"], cfg["sigJ"]), device=sysm.device)
    Y = pulses.reshape(n_train, -1)
    net = ProposalMLP(sysm, n_in=X.shape[1], width=512, n_out=Y.shape[1], depth=4, amax=amax,
                      seed=seed)
    keep = torch.as_tensor(np.nonzero(ok)[0], device=sysm.device)
    t1 = time.perf_counter()
    hist = net.train(X[:n_train][keep], Y[keep], epochs=epochs, batch=256, lr=train_lr, seed=seed,
                     log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1

    def evaluate(start_amps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        a = start_amps.reshape(-1, 2).contiguous()
        out = refine(sysm, a, [N] * n_test, dt, U[te], max_steps=refine_steps, lr=lr, amax=amax,
                     static_coef=cfg["B"][te], target_of_item=np.arange(n_test))
        torch.cuda.synchronize()
        reached = out["reached"]
        return {"fraction_F_ge_0999": float(np.mean(reached >= 0)),
                "mean_iterations_to_0999": float(np.mean(np.where(reached >= 0, reached,
                                                                   refine_steps + 1))),
                "median_iterations_to_0999": float(np.median(np.where(reached >= 0, reached,
                                                                       refine_steps + 1))),
                "mean_F_start": out["history"][0], "mean_F_end": out["history"][-1],
                "seconds": time.perf_counter() - t, "iterations_run": out["iterations"]}

    t2 = time.perf_counter()
    prop = net.propose(X[n_train:]).reshape(n_test, N, 2)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t2
    res_prop = evaluate(prop.clone())
    res_prop["seconds"] += t_inf
    res_cold = evaluate(cold_start(n_test, N, 2, amax, seed + 2))
    # baselines that know the training data without the network: the mean of
    # the optimiser's pulses (one pulse for every target), and the constant
    # mid-range pulse
    mean_pulse = Y[keep].reshape(-1, N, 2).mean(dim=0, keepdim=True)
    res_mean = evaluate(mean_pulse.expand(n_test, N, 2).contiguous())
    res_const = evaluate(torch.full((n_test, N, 2), 0.5 * amax, dtype=sysm.rdtype,
                                    device=sysm.device))
    # the full path: proposal, refine, judgement, cold-start fallback
    full = propose_and_refine(sysm, prop, N, dt, U[te], cfg["B"][te], refine_steps=refine_steps,
                              fallback_steps=fallback_steps, lr=lr, amax=amax, seed=seed + 3)
    res_full = {"fraction_F_ge_0999": float(np.mean(full["F"] >= 0.999)),
                "n_fallback": int(full["source"].sum()),
                "fallback_reached": int(np.sum((full["source"] == 1) & (full["F"] >= 0.999)))}
    return {"n_train": n_train, "n_train_used": int(ok.sum()), "n_test": n_test,
            "train_loss_first": hist[0], "train_loss_last": hist[-1], "seconds_data": t_data,
            "seconds_train": t_train, "seconds_inference": t_inf,
            "proposal_refine": res_prop, "cold_start": res_cold, "mean_pulse": res_mean,
            "constant_pulse": res_const, "with_fallback": res_full}
