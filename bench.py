"""Benchmark of the differentiable Lindblad-Magnus hot path on one MI355X.

A step is one forward+gradient evaluation (Magnus coefficients, per-slice
Liouvillian + Pade exponential, chunked ordered scan, fidelity, adjoint
Frechet derivative, chain rule) of a batch of synthetic 3-spin pulses of 4096
slices (superoperator 64 x 64, FP32, FOH second-order Magnus). Inputs are
resident in HBM before the timed region starts.

Prints one JSON line: pulse evaluations per second over the whole job, the
roofline of the dominant kernel (algorithmic MFMA flops per launch over its
HIP-event duration on the stream it runs on) and the FP64 oracle timed on the
host cores on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("fwd+grad pulse evals/s (3-spin, 4096 slices) & MFMA util, "
          "|ΔF|≤1e-6 vs FP64")
PEAK_FP32_MFMA_TFLOPS = 157.3
N_SUPER = 64
M_FLOPS = 8.0 * N_SUPER ** 3          # one complex 64x64x64 product, real flops
PI_M = {2: 1, 3: 2, 5: 3, 7: 4}       # products to evaluate the Pade-m numerator/denominator


def forward_flops_per_slice(m, s):
    # m = 2 (single precision, r_2 by its degree-4 series): A^2, one product,
    # squarings, the ordered product; otherwise Pade products + squarings + one
    # n x n solve (4/3) + the ordered product (1)
    if m == 2:
        return (2.0 + s + 1.0) * M_FLOPS
    return (PI_M[m] + s + 4.0 / 3.0 + 1.0) * M_FLOPS


def backward_flops_per_slice(m, s):
    # suffix product (1) + environment product (1) + Pade Frechet derivative
    return (1.0 + 1.0 + 2 * PI_M[m] + 2.0 + 2 * s) * M_FLOPS


def flops_from_hist(hist, per_slice):
    tot = 0.0
    for mi, m in enumerate((2, 3, 5, 7)):
        for s in range(hist.shape[1]):
            if hist[mi, s]:
                tot += hist[mi, s] * per_slice(m, s)
    return tot


# ---- CPU baseline: the FP64 oracle on the host cores -------------------------
# Per-slice work (the slice exponent Omega_n, S_n = exp(Omega_n), and later the
# Frechet derivative K_n with its traces against dOmega_n/du) runs in a pool of
# single-threaded worker processes, one per host core, like the paper's one
# slice per core; the prefix and suffix products run sequentially in the
# parent. Every step is an oracle function called as it stands; the result is
# that of oracle.grad_adjoint on the same pulse.
_W = {}


def _worker_init(cfg, amps):
    from threadpoolctl import threadpool_limits
    import oracle
    threadpool_limits(1)
    _W["sys"] = oracle.System.from_cfg(cfg)
    _W["amps"] = amps
    _W["cfg"] = cfg


def _worker_slice(n):
    import oracle
    c = _W["cfg"]
    om = oracle.slice_omega(_W["sys"].liouv, _W["amps"], n, c["dt"], 2, "foh")
    return om, oracle.expm_taylor(om)


def _worker_adjoint(job):
    import oracle
    n, om, M = job
    c = _W["cfg"]
    K = oracle.frechet_block(om, M)
    d2 = float(_W["sys"].d ** 2)
    return [(m, cc, float(np.real(np.trace(K @ dom))) / d2)
            for (m, cc), dom in _W["sys"].domega(_W["amps"], n, c["dt"], 2, "foh").items()]


def cpu_baseline(cfg):
    """The FP64 oracle's forward and adjoint gradient of the whole of pulse 0
    (4096 slices), per-slice work in a process pool over the host cores."""
    import multiprocessing as mp
    import oracle
    amps = cfg["amps"].astype(np.float32).astype(np.float64)
    N = amps.shape[0]
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    workers = max(1, min(16, int(cores)))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers, initializer=_worker_init, initargs=(cfg, amps)) as pool:
        pool.map(_worker_slice, range(min(N, workers)))          # workers started and warm
        t0 = time.perf_counter()
        res = pool.map(_worker_slice, range(N), chunksize=16)
        oms = [r[0] for r in res]
        S = [r[1] for r in res]
        n = oms[0].shape[0]
        X = [np.eye(n, dtype=complex)]
        for k in range(N):
            X.append(S[k] @ X[-1])
        d = cfg["U_target"].shape[0]
        ST = oracle.superop_of_unitary(cfg["U_target"])
        F = float(np.real(np.trace(ST.conj().T @ X[N]))) / (d * d)
        Y = ST.conj().T
        jobs = [None] * N
        for k in range(N - 1, -1, -1):
            jobs[k] = (k, oms[k], X[k] @ Y)
            Y = Y @ S[k]
        parts = pool.map(_worker_adjoint, jobs[::-1], chunksize=16)   # k = N-1 .. 0
        grad = np.zeros_like(amps)
        for contrib in parts:
            for m, c, v in contrib:
                grad[m, c] += v
        elapsed = time.perf_counter() - t0
    return {"value": 1.0 / elapsed, "unit": "pulse evals/s", "cores": workers,
            "kind": "oracle",
            "sample": f"FP64 oracle fwd+grad (Taylor expm, block-triangular Frechet) of the whole "
                      f"of pulse 0 ({N} slices), {elapsed:.1f} s: per-slice work in a pool of "
                      f"{workers} single-threaded processes, prefix/suffix products sequential",
            "cpu_model": _cpu_model(), "host_cores_available": int(cores)}, F, grad


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def read_traffic(kernel, slices):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE per slice from
    committed rocprofv3 counter runs, times the slices of one launch), if the
    counters were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.json")
    if not os.path.exists(path):
        return None
    try:
        import hashlib
        with open(path) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for src in rec.get("sources", []):
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec.get("source_sha256"):
            return None
        return rec["bytes_per_slice"] * slices
    except Exception:
        return None


TRAFFIC_SOURCES = ["paper_2511_13330_amd/csrc/k_slice.hip", "paper_2511_13330_amd/csrc/tile.hpp",
                   "paper_2511_13330_amd/csrc/internal.hpp"]


def record_traffic(fetch_csv, write_csv, slices, copy_bytes):
    """Writes profiles/traffic_<kernel>.json for k_forward and k_backward from
    two rocprofv3 counter runs of this script (FETCH_SIZE, then WRITE_SIZE, in
    KiB per dispatch), each scaled by what the same counter reads for the plain
    device copy of `copy_bytes` bytes that --copy-calibration dispatches first.
    Runs on the host from the CSV files; prints a markdown table."""
    import csv
    import hashlib

    def read(path, counter):
        rows = {}
        with open(path, newline="") as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                rows.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return rows

    kib = copy_bytes / 1024.0
    out = {}
    scales = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = read(path, counter)
        copies = [v for k, vals in rows.items() if "copyBuffer" in k for v in vals]
        if not copies:
            raise SystemExit(f"{path}: no calibration copy dispatch found")
        scales[counter] = kib / max(copies)
        for name, vals in rows.items():
            for kern in ("k_forward", "k_backward", "k_omega", "k_traces", "k_omega_sparse",
                         "k_traces_sparse", "k_traces_lds"):
                if f"lmag::{kern}<" in name:
                    out.setdefault(kern, {})[counter] = float(np.mean(vals))
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    print("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | read / slice | write / slice |")
    print("|---|---|---|---|---|")
    for kern, c in sorted(out.items()):
        if "FETCH_SIZE" not in c or "WRITE_SIZE" not in c:
            continue
        fb = c["FETCH_SIZE"] * scales["FETCH_SIZE"] * 1024.0 / slices
        wb = c["WRITE_SIZE"] * scales["WRITE_SIZE"] * 1024.0 / slices
        print(f"| {kern} | {c['FETCH_SIZE']:,.0f} | {c['WRITE_SIZE']:,.0f} | {fb / 1024:.1f} KiB | "
              f"{wb / 1024:.1f} KiB |")
        if kern not in ("k_forward", "k_backward"):
            continue
        rec = {"kernel": kern, "sources": TRAFFIC_SOURCES, "source_sha256": h.hexdigest(),
               "fetch_kib_raw": c["FETCH_SIZE"], "write_kib_raw": c["WRITE_SIZE"],
               "fetch_scale": scales["FETCH_SIZE"], "write_scale": scales["WRITE_SIZE"],
               "slices_per_dispatch_measured": slices, "bytes_per_slice": fb + wb,
               "fetch_bytes_per_slice": fb, "write_bytes_per_slice": wb}
        with open(os.path.join(ROOT, "profiles", f"traffic_{kern}.json"), "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
    print(f"\ncalibration: FETCH_SIZE x {scales['FETCH_SIZE']:.4f}, WRITE_SIZE x {scales['WRITE_SIZE']:.4f}")


def robust_sweep(args):
    """Candidates x quasi-static noise samples with uneven slice counts in one
    call per sweep: per-candidate mean fidelity and mean gradient."""
    import torch
    import synth
    from paper_2511_13330_amd import spin_chain_system
    n_cand = int(os.environ.get("LMAG_ROBUST_CANDIDATES", "256"))
    cfg = synth.config2(2, n_cand=n_cand)
    sysm = spin_chain_system(3, cfg["T1"], cfg["T2"], precision="f32", magnus_order=2,
                             hold="foh", chunk_slices=args.chunk, basis=args.basis)
    real = args.basis == "hermitian"
    amps = np.concatenate(cfg["amps_per_cand"])
    ns_c = np.asarray(cfg["n_slices_per_cand"])
    off_c = np.concatenate([[0], np.cumsum(ns_c)[:-1]])
    S = cfg["dB"].shape[0]
    ns = np.repeat(ns_c, S)
    off = np.repeat(off_c, S)
    groups = np.repeat(np.arange(n_cand), S)
    # per-item fields resident on the device, like the amplitudes
    static = torch.as_tensor(np.tile(np.asarray(cfg["B"])[None, :] + cfg["dB"], (n_cand, 1)),
                             dtype=torch.float64, device="cuda")
    scale = torch.as_tensor(np.tile(cfg["eps"], (n_cand, 1)), dtype=torch.float64, device="cuda")
    a = torch.tensor(amps, dtype=torch.float32, device="cuda")
    kw = dict(slice_offset=off, static_coef=static, ctrl_scale=scale, groups=groups)
    tuned = None
    if args.autotune and args.chunk == 0:
        tuned = sysm.autotune(a, ns, cfg["dt"], cfg["U_target"], reps=1, **kw)
    elif args.tuning and os.path.exists(args.tuning) and args.chunk == 0:
        sysm.load_tuning(args.tuning)
        key = f"p32{'h' if real else ''}_o2_d8_s{int(np.floor(np.log2(int(ns.sum()))))}"
        with open(args.tuning) as f:
            for line in f:
                rec = json.loads(line)
                if rec.get("key") == key:
                    tuned = (rec["chunk"], rec.get("variant", rec.get("inverse")), rec["ms"])
    F, g = sysm.fidelity_and_grad(a, ns, cfg["dt"], cfg["U_target"], **kw)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = max(1, min(args.steps, 3))
    for _ in range(steps):
        F, g = sysm.fidelity_and_grad(a, ns, cfg["dt"], cfg["U_target"], **kw)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    plan = sysm.last_plan()
    slices = int(ns.sum())
    hist = sysm.selection_histogram()   # of the call's last wave: its (m, s) mix stands for all
    flops = (flops_from_hist(hist, forward_flops_per_slice)
             + flops_from_hist(hist, backward_flops_per_slice)) * slices / max(1, int(hist.sum()))
    if real:
        flops /= 4   # real products: 2 n^3 flops where a complex one counts 8 n^3
    return {"metric": "robust sweep: candidates x noise samples fwd+grad, seconds per sweep",
            "value": dt, "unit": "s/sweep", "n_gpus": 1, "higher_is_better": False,
            "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (config-2 distributions: N ~ U{512..4096}, dB ~ N(0, 2pi), "
                    "eps ~ N(1, 0.01))",
            "config": {"workload": f"{n_cand} candidates x {S} noise samples, uneven N, "
                                   "3-spin FOH 2nd order", "items": int(len(ns)),
                       "slice_evaluations": slices, "waves": plan["waves"],
                       "chunk_slices": plan["chunk_slices"],
                       "representation": ("real (basis of Hermitian operators)" if real
                                          else "complex (column stacking)"),
                       "autotune": {"chunk": tuned[0], "inverse_variant": tuned[1],
                                    "ms_per_call_when_tuned": tuned[2]} if tuned else None},
            "slice_evals_per_s": slices / dt, "tflops_algorithmic": flops / dt / 1e12,
            "F_mean_first_candidates": [float(x) for x in F[:4].cpu().numpy()]}


def large_system(args):
    """4 spins (superoperator 256 x 256, 8192 slices of 0.25 ns) or 6 spins
    (4096 x 4096, 128 slices of 1 ns): one fwd+grad evaluation per step through
    the block-tiled path."""
    import torch
    import synth
    from paper_2511_13330_amd import spin_chain_system
    cfg = synth.config3_four() if args.workload == "four_spin" else synth.config3_six()
    t0 = time.perf_counter()
    sysm = spin_chain_system(cfg["n_spins"], cfg["T1"], cfg["T2"], precision="f32",
                             magnus_order=2, hold="foh", chunk_slices=args.chunk,
                             workspace_bytes_max=int(args.workspace_gb * (1 << 30)),
                             basis=args.basis)
    t_setup = time.perf_counter() - t0
    N = cfg["n_slices"]
    a = torch.tensor(cfg["amps"], dtype=torch.float32, device="cuda")
    b = np.asarray(cfg["B"])[None, :]
    tuned = None
    if args.autotune and args.chunk == 0:
        tuned = sysm.autotune(a, [N], cfg["dt"], cfg["U_target"], static_coef=b, reps=1)
    elif args.tuning and os.path.exists(args.tuning) and args.chunk == 0:
        sysm.load_tuning(args.tuning)
        tag = "h" if args.basis == "hermitian" else ""
        key = f"p32{tag}_o2_d{cfg['d']}_s{int(np.floor(np.log2(N)))}"
        with open(args.tuning) as f:
            for line in f:
                rec = json.loads(line)
                if rec.get("key") == key:
                    tuned = (rec["chunk"], rec.get("variant", rec.get("inverse")), rec["ms"])
    F, g = sysm.fidelity_and_grad(a, [N], cfg["dt"], cfg["U_target"], static_coef=b)  # warm-up
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    sysm.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        F, g = sysm.fidelity_and_grad(a, [N], cfg["dt"], cfg["U_target"], static_coef=b)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    sysm.set_profiling(False)
    prof = sysm.read_profile()
    hist = sysm.selection_histogram()
    n = 4 ** cfg["n_spins"]
    # the products' count in complex flops (8 n^3 each); in the real basis of
    # Hermitian operators each is one real product (2 n^3)
    flops = (flops_from_hist(hist, forward_flops_per_slice)
             + flops_from_hist(hist, backward_flops_per_slice)) * (n / N_SUPER) ** 3
    if args.basis == "hermitian":
        flops /= 4.0
    return {"metric": f"fwd+grad evaluations/s ({cfg['n_spins']} spins, {N} slices)",
            "value": 1.0 / dt, "unit": "evals/s", "n_gpus": 1, "higher_is_better": True,
            "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded config-3 draws)",
            "config": {"workload": f"{cfg['n_spins']} spins, superoperator {n}x{n}, {N} slices of "
                                   f"{cfg['dt'] * 1e3:g} ns, FOH 2nd order, FP32 fwd+grad",
                       "workspace_budget_gib": args.workspace_gb or None,
                       "representation": ("real (basis of Hermitian operators)"
                                          if args.basis == "hermitian"
                                          else "complex (column stacking)"),
                       "autotune": {"chunk": tuned[0], "product_kernel": tuned[1], "ms": tuned[2]}
                       if tuned else None,
                       "plan": sysm.last_plan()},
            "seconds_per_eval": dt, "seconds_set_system": t_setup,
            "tflops_algorithmic": flops / dt / 1e12,
            "frac_fp32_mfma": flops / dt / 1e12 / PEAK_FP32_MFMA_TFLOPS,
            "stage_ms": {k: v[0] / steps for k, v in prof.items()},
            "F": float(F.item())}


def hubbard(args):
    """Hubbard model of three dots (Eq. 1; superoperator 4096 x 4096, the size
    of the paper's measured propagator), 128 slices of 0.5 ns with dissipation:
    the propagator alone (the paper's measured step) and fwd+grad, per call."""
    import torch
    import synth
    from paper_2511_13330_amd import hubbard_system
    cfg = synth.hubbard3()
    t0 = time.perf_counter()
    sysm = hubbard_system(3, cfg["T1"], cfg["T2"], precision="f32", magnus_order=2, hold="foh",
                          chunk_slices=args.chunk,
                          workspace_bytes_max=int(args.workspace_gb * (1 << 30)),
                          basis=args.basis)
    t_setup = time.perf_counter() - t0
    N = cfg["n_slices"]
    a = torch.tensor(cfg["amps"], dtype=torch.float32, device="cuda")
    b = torch.tensor(np.asarray(cfg["coef"])[None, :], dtype=torch.float64, device="cuda")
    UT = torch.as_tensor(cfg["U_target"], dtype=torch.complex128, device="cuda")
    tuned = None
    if args.tuning and os.path.exists(args.tuning) and args.chunk == 0:
        # the autotuner's stored choice for this size (same key as the library's)
        sysm.load_tuning(args.tuning)
        tag = "h" if args.basis == "hermitian" else ""
        key = f"p32{tag}_o2_d{cfg['d']}_s{int(np.floor(np.log2(N)))}"
        with open(args.tuning) as f:
            for line in f:
                rec = json.loads(line)
                if rec.get("key") == key:
                    tuned = {"chunk": rec["chunk"], "product_kernel": rec.get("variant"), "ms": rec["ms"]}
    U = sysm.propagate(a, [N], cfg["dt"], static_coef=b)            # warm-up
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    t0 = time.perf_counter()
    for _ in range(steps):
        U = sysm.propagate(a, [N], cfg["dt"], static_coef=b)
    torch.cuda.synchronize()
    t_prop = (time.perf_counter() - t0) / steps
    plan_prop = sysm.last_plan()
    del U
    F, g = sysm.fidelity_and_grad(a, [N], cfg["dt"], UT, static_coef=b)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        F, g = sysm.fidelity_and_grad(a, [N], cfg["dt"], UT, static_coef=b)
    torch.cuda.synchronize()
    t_fg = (time.perf_counter() - t0) / steps
    return {"metric": "Hubbard 3-dot propagator (superoperator 4096 x 4096), seconds per call",
            "value": t_prop, "unit": "s/propagator", "n_gpus": 1, "higher_is_better": False,
            "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded Hubbard parameters and hopping pulses; the paper gives none)",
            "config": {"workload": f"3 dots x 4 states, {N} slices of {cfg['dt'] * 1e3:g} ns, FOH "
                                   "2nd order, T1/T2 per dot", "plan_propagate": plan_prop,
                       "plan_fwd_grad": sysm.last_plan(), "autotune": tuned,
                       "representation": ("real (basis of Hermitian operators)"
                                          if args.basis == "hermitian"
                                          else "complex (column stacking)")},
            "seconds_fwd_grad": t_fg, "seconds_set_system": t_setup, "F": float(F.item()),
            "context": "paper (Sec. IV): 1 min 15 s per propagator on an AMD EPYC 9634 CPU for this "
                       "superoperator size, slice count not stated"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=64, help="pulses per step")
    ap.add_argument("--chunk", type=int, default=0, help="slices per work unit (0 = auto)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--workspace-gb", type=float, default=0.0,
                    help="workspace budget of the large-system workloads in GiB (0 = 85 %% of free "
                         "device memory); beyond it the adjoint recomputes the forward")
    ap.add_argument("--no-latency", action="store_true", help="skip the single-pulse latency")
    ap.add_argument("--basis", default="hermitian", choices=["hermitian", "column"],
                    help="representation of the superoperators (FP32): the real basis of "
                         "Hermitian operators (default) or column stacking (complex)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune chunk length and inverse variant before the timed steps")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2511_13330_amd", "tuning",
                                                     "gfx950.jsonl"),
                    help="tuning lines written by lmag_autotune (LMAG_TUNE_CACHE) to load first; "
                         "'' for none")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run one plain device-to-device copy of BYTES (counter calibration)")
    ap.add_argument("--workload", default="pulse",
                    choices=["pulse", "proposal", "robust", "four_spin", "six_spin", "hubbard"],
                    help="pulse: the headline metric (default); proposal: learned proposal + "
                         "refine vs cold start; robust: candidates x noise samples, uneven N")
    ap.add_argument("--record-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="host only: write profiles/traffic_<kernel>.json from two counter runs "
                         "(rocprofv3 counter_collection.csv of a --copy-calibration run with this "
                         "--batch)")
    args = ap.parse_args()
    if args.record_traffic:
        if args.copy_calibration <= 0:
            ap.error("--record-traffic needs the --copy-calibration size the counter runs used")
        record_traffic(*args.record_traffic, slices=args.batch * 4096, copy_bytes=args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path).", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2511_13330_amd import spin_chain_system

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    if args.workload == "proposal":
        from paper_2511_13330_amd.proposal import run_experiment
        r = run_experiment(log=lambda s: print(s, file=sys.stderr, flush=True))
        p = r["proposal_refine"]
        print(json.dumps({
            "metric": "fraction of held-out targets reaching F >= 0.999 within 50 refine steps",
            "value": p["fraction_F_ge_0999"], "unit": "fraction", "n_gpus": 1,
            "higher_is_better": True, "vs_baseline": None, "dtype": "bf16 MLP / f32 propagator",
            "data": "synthetic reachable targets (closed-system propagators of smooth seeded pulses)",
            "config": {"workload": "learned proposal: 133-512-512-512-512 MLP, 256 slices of "
                                   "0.25 ns, batch 4096 inference, <= 50 refine steps",
                       "n_train": r["n_train"], "n_test": r["n_test"]},
            "result": r}), flush=True)
        return
    if args.workload == "robust":
        print(json.dumps(robust_sweep(args)), flush=True)
        return
    if args.workload == "hubbard":
        print(json.dumps(hubbard(args)), flush=True)
        return
    if args.workload in ("four_spin", "six_spin"):
        print(json.dumps(large_system(args)), flush=True)
        return
    dev = torch.device("cuda", 0)
    if args.copy_calibration > 0:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    B = args.batch
    cfg = synth.config1_batch(B)
    sysm = spin_chain_system(3, cfg["T1"], cfg["T2"], precision="f32", magnus_order=2,
                             hold="foh", chunk_slices=args.chunk, basis=args.basis)
    real = args.basis == "hermitian"
    amps = torch.tensor(cfg["amps_batch"].reshape(B * 4096, 2), dtype=torch.float32,
                        device=dev).contiguous()
    n_slices = np.full(B, 4096, dtype=np.int32)
    # the target and the static fields are resident like the amplitudes: a copy
    # from pageable host memory inside the step would wait for the previous
    # step's kernels and leave the device idle while the next step is launched
    static = torch.as_tensor(np.tile(np.asarray(cfg["B"])[None, :], (B, 1)),
                             dtype=torch.float64, device=dev)
    UT = torch.as_tensor(cfg["U_target"], dtype=torch.complex128, device=dev)

    def step(a=amps, ns=n_slices, st=static):
        return sysm.fidelity_and_grad(a, ns, cfg["dt"], UT, static_coef=st)

    tuned = None
    if args.tuning and os.path.exists(args.tuning) and args.chunk == 0 and not args.autotune:
        # the autotuner's stored choice for this size (same key as the library's)
        sysm.load_tuning(args.tuning)
        key = f"p32{'h' if real else ''}_o2_d8_s{int(np.floor(np.log2(B * 4096)))}"
        with open(args.tuning) as f:
            for line in f:
                rec = json.loads(line)
                if rec.get("key") == key:
                    tuned = (rec["chunk"], rec.get("variant", rec.get("inverse")), rec["ms"],
                             os.path.relpath(args.tuning, ROOT))
    if args.autotune and args.chunk == 0:
        tuned = sysm.autotune(amps, n_slices, cfg["dt"], UT, static_coef=static, reps=1)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sysm.read_profile()                      # drop warm-up records
    sysm.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        F, g = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sysm.set_profiling(False)
    prof = sysm.read_profile()
    plan = sysm.last_plan()
    hist = sysm.selection_histogram()
    F0 = float(F[0].item())

    value = B * args.steps / elapsed
    fwd_flops = flops_from_hist(hist, forward_flops_per_slice)
    bwd_flops = flops_from_hist(hist, backward_flops_per_slice)
    if real:
        # the same products on real matrices: 2 n^3 flops where a complex one counts 8 n^3
        fwd_flops /= 4
        bwd_flops /= 4
    stage_ms = {k: v[0] / max(1, v[1]) for k, v in prof.items()}
    kernels = {
        "k_backward": (bwd_flops, stage_ms["backward"]),
        "k_forward": (fwd_flops, stage_ms["forward"]),
    }
    dom = max(kernels, key=lambda k: kernels[k][1])
    fl, ms = kernels[dom]
    achieved = fl / (ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved,
                "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_MFMA_TFLOPS,
                "traffic": read_traffic(dom, plan["total_slices"]),
                "flops_per_launch": fl, "ms_per_launch": ms}
    if real:
        # the products are real (one MFMA product each); in complex flops the
        # column-stacking form of the same work would count four times as many
        roofline["complex_equivalent_tflops"] = 4 * achieved
    else:
        # the matrix cores execute each complex product in the 3M form
        # (3 real products, 6 n^3 flops) against the 8 n^3 counted above
        roofline["frac_executed_3m"] = 0.75 * achieved / PEAK_FP32_MFMA_TFLOPS
    other = [k for k in kernels if k != dom][0]
    fl2, ms2 = kernels[other]
    total_flops = fwd_flops + bwd_flops
    out = {
        "metric": METRIC, "value": value, "unit": "pulse evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded PCG64: U[0, 2pi*20] rad/us amplitudes, U[-2pi*10, 2pi*10] "
                "fields, Haar target)",
        "config": {"workload": "3 spins (d=8, superoperator 64x64), 4096 slices of 0.25 ns, "
                               "FOH second-order Magnus, FP32 forward+adjoint gradient, "
                               f"batch of {B} pulses per step",
                   "batch_pulses": B, "n_slices": 4096, "superop_dim": 64,
                   "representation": ("real (basis of Hermitian operators)" if real
                                      else "complex (column stacking)"),
                   "chunk_slices": plan["chunk_slices"], "grid": plan["grid"],
                   "inverse": "auto (power series, MFMA Neumann or Gauss-Jordan per slice bound)"
                   if not tuned or tuned[1] == 0 else ("Gauss-Jordan" if tuned[1] == 1 else "Neumann"),
                   "autotune": ({"chunk": tuned[0], "inverse_variant": tuned[1],
                                 "ms_per_call_when_tuned": tuned[2],
                                 "source": tuned[3] if len(tuned) > 3 else "tuned in this run"}
                                if tuned else None)},
        "roofline": roofline,
        "whole_step_tflops": total_flops / (elapsed / args.steps) / 1e12,
        "other_kernel": {"kernel": other, "achieved_tflops": fl2 / (ms2 * 1e-3) / 1e12,
                         "ms_per_launch": ms2},
        "stage_ms_per_launch": stage_ms,
        "F_pulse0": F0,
    }
    if not args.no_latency:
        a1 = amps[:4096].contiguous()
        for _ in range(max(1, args.warmup)):
            step(a1, n_slices[:1], static[:1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(a1, n_slices[:1], static[:1])
        torch.cuda.synchronize()
        out["latency_ms_single_pulse"] = 1e3 * (time.perf_counter() - t0) / args.steps
    if not args.no_cpu:
        cb, F_or, g_or = cpu_baseline(cfg)
        out["cpu_baseline"] = cb
        g0 = g[:4096].double().cpu().numpy()
        # the parity gate on the timed pulse 0 against the oracle run above
        out["parity_pulse0"] = {
            "dF": abs(F0 - F_or), "F_oracle": F_or,
            "grad_rel_err": float(np.linalg.norm(g0 - g_or) / np.linalg.norm(g_or)),
            "gate": "|dF| <= 1e-6, gradient relative error <= 1e-3 (all 8192 coordinates)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
