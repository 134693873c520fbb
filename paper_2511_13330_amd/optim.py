"""Plain gradient optimiser of pulse amplitudes (the paper's Adam loop,
Sec. III-C): every iteration is one fused forward+adjoint call of the library
followed by its Adam + projection kernel. The host reads the fidelity vector
once per iteration to decide which items are still active; that is the only
synchronisation."""
import numpy as np
import torch


def refine(system, amps, n_slices, dt, U_target, max_steps=50, lr=None, amax=None,
           target=0.999, static_coef=None, ctrl_scale=None, target_of_item=None,
           betas=(0.9, 0.999), eps=1e-8):
    """Ascend F from `amps` (modified in place). Returns a dict with the final
    fidelities, the iteration at which each item first reached `target`
    (-1 if never) and the per-iteration mean fidelity."""
    n_slices = np.asarray(n_slices, dtype=np.int64).reshape(-1)
    n_items = len(n_slices)
    amax = float(amax) if amax is not None else float("inf")
    lr = float(lr) if lr is not None else 0.01 * (amax if np.isfinite(amax) else 1.0)
    off = np.concatenate([[0], np.cumsum(n_slices)[:-1]])
    row_item = torch.as_tensor(np.repeat(np.arange(n_items), n_slices), device=amps.device)
    m = torch.zeros_like(amps)
    v = torch.zeros_like(amps)
    reached = np.full(n_items, -1, dtype=np.int64)
    history = []
    F = None
    for it in range(max_steps + 1):
        F, g = system.fidelity_and_grad(amps, n_slices, dt, U_target, slice_offset=off,
                                        static_coef=static_coef, ctrl_scale=ctrl_scale,
                                        target_of_item=target_of_item,
                                        want_grad=it < max_steps)
        Fh = F.cpu().numpy()            # the one host read per iteration
        history.append(float(np.nanmean(Fh)))
        newly = (reached < 0) & (Fh >= target)
        reached[newly] = it
        active = (reached < 0) & np.isfinite(Fh)
        if it == max_steps or not active.any():
            break
        act = torch.as_tensor(active.astype(np.uint8), device=amps.device)[row_item].contiguous()
        system.adam_project(amps, g, m, v, it + 1, lr, betas[0], betas[1], eps,
                            grad_scale=-1.0, lo=0.0, hi=amax, row_active=act)
    return {"F": Fh, "reached": reached, "history": history, "iterations": it}


def cold_start(n_items, n_slices, n_ctrl, amax, seed, device="cuda", dtype=torch.float32):
    """Uniform random amplitudes in [0, amax] (the plain method's start)."""
    a = np.random.default_rng(seed).uniform(0.0, amax, (n_items * n_slices, n_ctrl))
    return torch.tensor(a, dtype=dtype, device=device).contiguous()
