#!/usr/bin/env python3
"""Throughput of Levenberg-Marquardt reconstructions on one MI355X.

One step = one full reconstruction (15 outer LM iterations x 30 CG steps,
FP32, no early exit) of every slice of a batch of independent 128 x 128
slices, 360 angles over a full turn x 192 detector bins, Gaussian collimator
sigma 1.5 bins, gradient penalty alpha = 1e-2.  Inputs are seeded synthetic
9 x 9 rod-lattice phantoms with Poisson counting noise (peak 1e4), resident
in HBM before the timed region starts.  Prints ONE JSON line.

The damped step is taken in variables divided by their typical magnitudes
with the active set (--solver plain: D = W = I, clamp only).

Measured alongside:
* each kernel class's device time from HIP events on the launch stream (the
  dominant class gives the roofline entry, with the counter-measured HBM
  traffic of the committed profiles);
* the same batch with BF16 storage of the Jacobian weights;
* the reconstruction error against the phantoms;
* a single slice's latency;
* the FP64 CPU oracle, timed on the host cores on a bounded sample of the
  same workload;
* the serving half of the metric: a 10 s Poisson trace (30 requests/s)
  over the mixed grid sizes {64..256}^2 through the continuous-batching
  server (whole batched solves on concurrent streams), with p50/p99
  latency, the plain per-slice solver on the same trace, and a bitwise
  check of served results against the same slices solved alone; the same
  trace through the iteration-level server (per-size slot pools admitting
  at every outer iteration) beside it.

Other workloads (--workload): mixed grid sizes, serving alone (rate and
server selectable), the scanner geometry, and the safeguarded Deep
Gauss-Newton comparison.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic VALU work of one operator pass per in-support sample of the
# rotated lattice (the method's arithmetic: bilinear taps, the attenuation
# exponential, the per-ray sums and the tent gather), in lane-operations.
LANE_OPS_PER_SAMPLE = {"vjp": 70.0, "gradient": 70.0, "jvp": 50.0, "march": 30.0}
# FP32 VALU peak without packed math (the build disables packed FP32):
# 256 CUs x 64 lanes x 2.4 GHz, one lane-operation (an FMA counts once) per lane and clock.
PEAK_VALU_TLANEOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0
# Plans solved in batches of at least this many slices turn band staging on
# (maps whose bordered pair does not fit in LDS: 256^2, the 165^2 scanner grid)
BAND_STAGING_MIN_BATCH = 32


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=64, help="slices reconstructed per step")
    ap.add_argument("--grid", type=int, default=128, choices=[64, 128, 256],
                    help="main workload: 64 (9x9 lattice, 120 x 96; C1 uses --cg 20), 128 (9x9 lattice, "
                         "360 x 192) or 256 (17x17 lattice, 360 x 256)")
    ap.add_argument("--outer", type=int, default=15)
    ap.add_argument("--prior", type=float, default=0.0,
                    help="geometry prior weight gamma (main and scanner workloads): gamma on "
                         "emission and gamma / mu_scale^2 on attenuation wherever no rod can lie; 0 = off")
    ap.add_argument("--solver", default="scaled", choices=["scaled", "plain"],
                    help="scaled: damping and CG in variables divided by their typical magnitudes "
                         "(1 for emission, 0.05 for attenuation) with the active set; plain: "
                         "D = W = I, clamp only")
    ap.add_argument("--cg", type=int, default=30)
    ap.add_argument("--no-single", action="store_true", help="skip the single-slice latency run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0, help="0: min(16, cpu count)")
    ap.add_argument("--workload", default="main", choices=["main", "mixed", "serve", "scanner", "deepgn"],
                    help="main: batch of 128^2 slices (the headline metric); mixed: 64 slices of "
                         "mixed sizes {64..256}^2 solved together vs one at a time; serve: "
                         "open-loop Poisson requests of mixed sizes through the continuous-batching "
                         "server vs the plain per-slice solver")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=5.0, help="serve: seconds of arrivals")
    ap.add_argument("--pool", type=int, default=256, help="serve: distinct request payloads")
    ap.add_argument("--streams", type=int, default=4, help="serve (--server batch): concurrent solves")
    ap.add_argument("--server", default="iter", choices=["iter", "batch"],
                    help="serve: iter = per-size slot pools admitting requests at every outer-iteration "
                         "boundary; batch = whole batched solves on --streams streams")
    ap.add_argument("--capacity", type=int, default=8, help="serve (--server iter): slots per size")
    ap.add_argument("--no-plain", action="store_true", help="serve: skip the plain per-slice solver")
    ap.add_argument("--serve-rate", type=float, default=30.0,
                    help="main workload: arrival rate of the serving leg (0 = skip it)")
    ap.add_argument("--serve-duration", type=float, default=10.0,
                    help="main workload: seconds of arrivals of the serving leg")
    ap.add_argument("--hbm-budget-gb", type=float, default=64.0, help="serve: in-flight workspace cap")
    ap.add_argument("--autotune", action="store_true", help="autotune launch shapes first")
    ap.add_argument("--storage", default="fp32", choices=["fp32", "bf16"],
                    help="storage of staged maps and per-sample weights")
    ap.add_argument("--dg-set", default="lattice", choices=["lattice", "scanner"], help="deepgn: slice family")
    ap.add_argument("--dg-k", type=int, default=3, help="deepgn: number of learned refinements")
    ap.add_argument("--dg-train", type=int, default=192, help="deepgn: training slices")
    ap.add_argument("--dg-test", type=int, default=16, help="deepgn: held-out slices")
    ap.add_argument("--dg-outer", type=int, default=5, help="deepgn: outer iterations")
    ap.add_argument("--dg-epochs", type=int, default=40, help="deepgn: epochs per network")
    ap.add_argument("--dg-decay", type=float, default=1.0,
                    help="deepgn: divide the alphas by this factor per iteration (the paper uses 5)")
    ap.add_argument("--dg-decay-until", type=int, default=3, help="deepgn: iterations the decay runs for")
    ap.add_argument("--full-model", action="store_true",
                    help="scanner: the full discrete model (depth-dependent collimator response and "
                         "vertical correction) for the data and the reconstruction; the plain model "
                         "is timed beside it")
    ap.add_argument("--no-bf16-variant", action="store_true",
                    help="main workload: skip timing the BF16-storage variant beside FP32")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 256 MiB device copy (scale for HBM counters)")
    return ap.parse_args()


# Damped-step options of the main workload.  "scaled": the LM step taken in
# variables divided by their typical magnitudes (emission 1, attenuation
# 0.05 per pixel), i.e. identity damping and plain CG there (D = diag(1,
# 1/0.05^2), W = D^-1), with the variables held at a bound left out of CG.
SOLVER_OPTIONS = {
    "scaled": {"w_mu": 0.05 ** 2, "d_mu": 1.0 / 0.05 ** 2, "active_set": 1},
    "plain": {},
}
# The same for the scanner geometry: attenuation bounded by 0.14 /mm.
SCANNER_SOLVER_OPTIONS = {
    "scaled": {"w_mu": 0.14 ** 2, "d_mu": 1.0 / 0.14 ** 2, "active_set": 1},
    "plain": {},
}


def prior_tensors(gamma, mu_scale, region, ref_f, ref_mu, torch, np):
    """Device weights and references of the geometry prior (None when gamma
    is 0): gamma on emission and gamma / mu_scale^2 on attenuation inside
    the region where no rod can lie."""
    if gamma <= 0.0:
        return {}
    w = np.stack([gamma * region, gamma / mu_scale ** 2 * region])
    T = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    return {"prior_w": T(w), "prior_ref": T(np.stack([ref_f, ref_mu]))}


def quality(fs, ms, cfg, inputs, np):
    """Mean relative L2 error of the reconstructions against the phantoms
    inside the disk of the field of view."""
    cc = np.arange(cfg.n) - 0.5 * (cfg.n - 1)
    X, Y = np.meshgrid(cc, cc)
    disk = X ** 2 + Y ** 2 <= (0.5 * cfg.n) ** 2
    ef, em = [], []
    for s in range(len(fs)):
        tf, tm = inputs.rod_lattice(cfg, s)
        ef.append(np.linalg.norm((fs[s].cpu().numpy() - tf)[disk]) / np.linalg.norm(tf[disk]))
        em.append(np.linalg.norm((ms[s].cpu().numpy() - tm)[disk]) / np.linalg.norm(tm[disk]))
    return {"f_rel_err_fov": round(float(np.mean(ef)), 4), "mu_rel_err_fov": round(float(np.mean(em)), 4)}


def make_inputs(plan, cfg, batch, torch, inputs, np):
    """Phantoms (inputs module), clean data from the library's forward map,
    Poisson noise, and the closed-form initial guess mu0 = 0, f0 = c0."""
    ys, f0s, m0s = [], [], []
    one = torch.ones((cfg.n, cfg.n), dtype=torch.float32, device="cuda")
    zero = torch.zeros_like(one)
    a1 = plan.forward(one, zero).double().cpu().numpy()
    for s in range(batch):
        f, mu = inputs.rod_lattice(cfg, s)
        T = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
        y_clean = plan.forward(T(f), T(mu)).double().cpu().numpy()
        y = inputs.poisson_counts(y_clean, cfg.peak_counts, s)
        c0 = float((a1 * y).sum() / (a1 * a1).sum())
        ys.append(T(y))
        f0s.append(torch.full((cfg.n, cfg.n), c0, dtype=torch.float32, device="cuda"))
        m0s.append(zero.clone())
    return ys, f0s, m0s


def cpu_baseline(cfg, workers: int):
    """The FP64 oracle on host cores, on a bounded sample: each worker times
    one forward, one Jacobian product and one adjoint at full size on its own
    slice; a reconstruction is 15 x (2 forward + 1 JVP + 31 adjoint + 30 JVP)
    + 1 JVP passes, so recon/s = workers / (that many seconds)."""
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_sample, [(cfg, s) for s in range(workers)])
        wall = time.perf_counter() - t0
    t_fwd = sum(r[0] for r in res) / len(res)
    t_jvp = sum(r[1] for r in res) / len(res)
    t_vjp = sum(r[2] for r in res) / len(res)
    K, M = cfg.max_outer, cfg.n_cg
    per_recon = K * (2 * t_fwd + (M + 1) * t_jvp + (M + 1) * t_vjp) + t_jvp
    return {
        "value": workers / per_recon, "unit": "reconstructions/s", "cores": workers,
        "kind": "oracle", "cpu_model": cpu_model(),
        "sample": ("FP64 C oracle, one forward + one J v + one J^T w per worker at %dx%d, %d angles, "
                   "%d bins (%.1f s wall on %d workers), scaled to %d x (%d CG) passes per "
                   "reconstruction: %.1f s per reconstruction per core"
                   % (cfg.n, cfg.n, cfg.n_angles, cfg.n_bins, wall, workers, K, M, per_recon)),
    }


def cpu_model():
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_sample(arg):
    cfg, seed = arg
    import numpy as np
    import oracle
    from paper_2604_26745_amd import inputs
    g = oracle.Geometry(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
    f, mu = inputs.rod_lattice(cfg, seed)
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    y = oracle.forward(g, f, mu)
    t1 = time.perf_counter()
    oracle.jvp(g, f, mu, f, mu)
    t2 = time.perf_counter()
    oracle.vjp(g, f, mu, y + rng.standard_normal(y.shape))
    t3 = time.perf_counter()
    return t1 - t0, t2 - t1, t3 - t2


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("pget_kernels.hip", "pget_internal.h"):
        with open(os.path.join(ROOT, "paper_2604_26745_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel: str, workload: str):
    """HBM bytes per launch from the committed PMC summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            data = json.load(fh)
        ent = data.get(workload, {}).get(kernel)
        if not ent or ent.get("kernel_source") != kernel_source_hash():
            return None
        return float(ent["bytes_per_launch"])
    except Exception:
        return None


def instrumented_roofline(pget, torch, run_step, max_outer, n_cg, units, workload):
    """One more step with HIP events bracketing every launch of the heavy
    kernel classes on the launch stream (direct launches: events are not
    recorded inside a replayed graph), and the roofline object of the
    dominant class: its algorithmic lane-operations per launch over its
    average launch time, with the committed counter bytes of the workload
    when they were taken from the current kernel sources."""
    classes = (1 << pget.KC_VJP) | (1 << pget.KC_JVP) | (1 << pget.KC_MARCH) | \
              (1 << pget.KC_VECTOR) | (1 << pget.KC_GRADIENT)
    # timed launches per outer iteration: n_cg J^T, n_cg + 2 J, 2 n_cg + 6
    # vector kernels, 2 marches and the gradient; room to spare
    per_step = max_outer * (5 * n_cg + 24) + 16
    pget.timing_enable(classes, per_step + 64)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    run_step()
    torch.cuda.synchronize()
    instrumented_s = time.perf_counter() - t2
    kt = {pget.KERNEL_CLASS_NAMES[c]: pget.timing_read(c) for c in
          (pget.KC_VJP, pget.KC_JVP, pget.KC_MARCH, pget.KC_VECTOR, pget.KC_GRADIENT)}
    pget.timing_enable(0, 0)
    print("bench: instrumented step %.3f s; kernel ms (total, launches): %s" % (
        instrumented_s, {k: (round(v[0], 2), v[1]) for k, v in kt.items()}), file=sys.stderr,
        flush=True)
    dom = max(kt, key=lambda k: kt[k][0])
    tot_ms, launches = kt[dom]
    avg_s = tot_ms / 1e3 / max(launches, 1)
    achieved = LANE_OPS_PER_SAMPLE[dom] * units / avg_s / 1e12
    kernel_name = {"vjp": "k_vjp_lin", "gradient": "k_vjp_lin", "jvp": "k_jvp_lin",
                   "march": "k_march"}.get(dom, dom)
    roofline = {
        "bound": "alu", "kernel": kernel_name, "achieved": round(achieved, 3),
        "peak": round(PEAK_VALU_TLANEOPS, 3), "unit": "Tlane-op/s", "frac": round(achieved / PEAK_VALU_TLANEOPS, 4),
        "traffic": traffic_from_profile(kernel_name, workload),
        "avg_launch_us": round(avg_s * 1e6, 2), "launches": launches,
        "lane_ops_per_unit": LANE_OPS_PER_SAMPLE[dom], "units_per_launch": units,
    }
    if roofline["traffic"]:
        # counter-measured HBM rate of the same launches (the weight stream)
        roofline["hbm_gbs"] = round(roofline["traffic"] / avg_s / 1e9, 1)
        roofline["hbm_frac"] = round(roofline["traffic"] / avg_s / 1e9 / PEAK_HBM_GBS, 4)
    return roofline, kt, instrumented_s


def run_mixed(args, torch, np, inputs, pget):
    """64 slices with grid sizes drawn from {64, 96, 128, 192, 256}^2, 360
    angles, 1.5x grid bins, 9x9 or 17x17 lattices, Poisson peak 10^U(3,5);
    solved together (one plan per size, groups concurrent) and, as the
    comparison, one slice at a time with the same kernels."""
    n = args.batch
    cfgs = [inputs.mixed_config(s)[0] for s in range(n)]
    cfgs = [inputs.scaled(c, max_outer=args.outer, n_cg=args.cg) for c in cfgs]
    plans = {}
    for c in cfgs:
        if c.n not in plans:
            plans[c.n] = pget.Plan(c.n, c.n_angles, c.n_bins, psf_sigma=c.psf_sigma, storage=args.storage)
    ys, f0s, m0s, pl = [], [], [], []
    ones = {}
    for s, c in enumerate(cfgs):
        plan = plans[c.n]
        if c.n not in ones:
            o = torch.ones((c.n, c.n), dtype=torch.float32, device="cuda")
            ones[c.n] = plan.forward(o, torch.zeros_like(o)).double().cpu().numpy()
        a1 = ones[c.n]
        f, mu = inputs.rod_lattice(c, s)
        T = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
        y = inputs.poisson_counts(plan.forward(T(f), T(mu)).double().cpu().numpy(), c.peak_counts, s)
        c0 = float((a1 * y).sum() / (a1 * a1).sum())
        ys.append(T(y)); pl.append(plan)
        f0s.append(torch.full((c.n, c.n), c0, dtype=torch.float32, device="cuda"))
        m0s.append(torch.zeros((c.n, c.n), dtype=torch.float32, device="cuda"))
    prm = [pget.SolverParams(max_outer=c.max_outer, n_cg=c.n_cg, alpha_f=c.alpha, alpha_mu=c.alpha,
                             **SOLVER_OPTIONS[args.solver])
           for c in cfgs]
    counts = {}
    for c in cfgs:
        counts[c.n] = counts.get(c.n, 0) + 1
    if args.autotune:
        for nn, plan in plans.items():
            plan.autotune(counts[nn])
            plan.autotune(1)
    print("bench: mixed batch sizes %s" % sorted(counts.items()), file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        pget.lm_solve_multi(pl, ys, f0s, m0s, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fs, ms, rbs = pget.lm_solve_multi(pl, ys, f0s, m0s, prm, sync=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    value = n * args.steps / el
    # plain per-slice solver: same kernels, one slice at a time
    for s in range(min(n, len(plans))):
        pl[s].lm_solve(ys[s], f0s[s], m0s[s], prm[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(n):
        pl[s].lm_solve(ys[s], f0s[s], m0s[s], prm[s], sync=False)
    torch.cuda.synchronize()
    el1 = time.perf_counter() - t1
    plain = n / el1
    reps = [r.to_report() for r in rbs]
    assert all(r.status == 0 for r in reps)
    # each size group alone, as a same-size batch: what the concurrent groups
    # of the mixed call would take one after another
    alone = {}
    for nn, plan in plans.items():
        idx = [s for s in range(n) if cfgs[s].n == nn]
        sub = lambda v: [v[s] for s in idx]
        plan.lm_solve_batched(sub(ys), sub(f0s), sub(m0s), sub(prm))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(args.steps):
            plan.lm_solve_batched(sub(ys), sub(f0s), sub(m0s), sub(prm))
        torch.cuda.synchronize()
        alone[nn] = (time.perf_counter() - t2) / args.steps
    seq_ms = 1e3 * sum(alone.values())
    # work: in-support lattice samples x outer iterations x CG steps (each CG
    # step streams every sample through one product and one adjoint)
    work = sum(plans[c.n].support_samples * c.max_outer * c.n_cg for c in cfgs)
    groups = {str(nn): {"slices": counts[nn], "alone_ms": round(1e3 * t, 2),
                        "gsamples_per_s": round(counts[nn] * plans[nn].support_samples * args.outer * args.cg
                                                / t / 1e9, 2)}
              for nn, t in sorted(alone.items())}
    print("bench: mixed step %.1f ms; groups alone %s ms, sequential sum %.1f ms" % (
        1e3 * el / args.steps, {k: v["alone_ms"] for k, v in groups.items()}, seq_ms), file=sys.stderr, flush=True)
    out = {
        "metric": "LM reconstructions/s, mixed grid sizes {64..256}^2 x 360 angles (FP32)",
        "value": round(value, 4), "unit": "reconstructions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * el / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mixed_sizes_%d_slices" % n, "sizes": sorted(counts.items()),
                   "solver": dict({"name": args.solver}, **SOLVER_OPTIONS[args.solver]),
                   "outer": args.outer, "cg": args.cg, "autotuned": bool(args.autotune),
                   "tuned_shapes": {str(k): p.tuned_shape(counts[k]) for k, p in plans.items()}},
        "plain_per_slice": {"value": round(plain, 4), "unit": "reconstructions/s",
                            "speedup": round(value / plain, 3)},
        "size_groups": {"alone": groups, "sequential_sum_ms": round(seq_ms, 2),
                        "concurrent_over_sequential": round(seq_ms / (1e3 * el / args.steps), 3),
                        "work_gsamples_per_s": round(work * args.steps / el / 1e9, 2),
                        "work_unit": "in-support samples x outer iterations x CG steps"},
    }
    print(json.dumps(out), flush=True)


def run_scanner(args, torch, np, inputs, pget):
    """Scanner geometry: 9x9 assemblies (full / missing / replaced / medium
    rods in turn) drawn on a 330^2 grid of 1 mm pixels, projected there by
    the library, 2 % Gaussian noise, reconstructed batched on the 165^2 grid
    of 2 mm pixels (182 bins of 2 mm, 360 angles); the data are expressed in
    the reconstruction grid's units (ray sums per 2 mm step).  --solver scaled: the step
    in variables divided by their upper bounds (emission 1, attenuation
    0.14 /mm) with the active set, started from water inside the field of
    view; plain: D = W = I from mu0 = 0.  Reports throughput and the mean
    relative error of the maps inside the field of view."""
    import dataclasses
    cfg = dataclasses.replace(inputs.SCANNER_165, max_outer=args.outer, n_cg=args.cg)
    full = args.full_model
    if full and args.storage != "fp32":
        sys.exit("bench: the full discrete model runs with FP32 storage only")
    geo = {}
    for o in (1, cfg.oversample):
        d = inputs.scanner_geometry(cfg, o, full_model=full)
        ys_ = d.pop("y_scale")
        n = d.pop("n")
        pl = pget.Plan(n, d.pop("n_angles"), d.pop("n_bins"), storage=args.storage, **d)
        if o == 1:
            pl.set_band_staging(args.batch >= BAND_STAGING_MIN_BATCH)
        if full:
            dep, al, far = inputs.scanner_full_model(cfg, pl.n_samples)
            pl.set_depth_factor(dep)
            pl.set_depth_response(al, far)
        geo[o] = (pl, ys_)
    plan, cscale = geo[1]
    fine, fscale = geo[cfg.oversample]
    T = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    kinds = ("full", "missing", "replaced", "medium")
    B = args.batch
    one = torch.ones((cfg.n, cfg.n), dtype=torch.float32, device="cuda")
    a1 = plan.forward(one, torch.zeros_like(one)).double().cpu().numpy()
    ys, f0s, m0s, truth = [], [], [], []
    for s_ in range(B):
        ff, mf = inputs.scanner_phantom(cfg, s_, kinds[s_ % 4], cfg.oversample)
        y = inputs.gaussian_noise((fscale / cscale) * fine.forward(T(ff), T(mf)).double().cpu().numpy(), cfg.noise, s_)
        truth.append(inputs.scanner_phantom(cfg, s_, kinds[s_ % 4], 1))
        c0 = float((a1 * y).sum() / (a1 * a1).sum())
        ys.append(T(y))
        f0s.append(torch.full((cfg.n, cfg.n), c0, dtype=torch.float32, device="cuda"))
        if args.solver == "scaled":
            m0s.append(T(np.where(inputs.fov_mask(cfg), cfg.water_mu, 0.0)))
        else:
            m0s.append(torch.zeros((cfg.n, cfg.n), dtype=torch.float32, device="cuda"))
    opts = SCANNER_SOLVER_OPTIONS[args.solver]
    prior = prior_tensors(args.prior, cfg.rod_mu_range[1], *inputs.scanner_rod_prior(cfg), torch, np)
    prm = [pget.SolverParams(max_outer=cfg.max_outer, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha, **opts,
                             **prior) for _ in range(B)]
    print("bench: scanner geometry, %d slices, data on the %d^2 grid" % (B, cfg.n * cfg.oversample),
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        plan.lm_solve_batched(ys, f0s, m0s, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fs, ms, rbs = plan.lm_solve_batched(ys, f0s, m0s, prm, sync=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    reps = [r.to_report() for r in rbs]
    assert all(r.status == 0 for r in reps)
    wl = "%s_batch%d" % (cfg.name, B) + ("_full_model" if full else "")
    roofline, _, _ = instrumented_roofline(pget, torch, lambda: plan.lm_solve_batched(ys, f0s, m0s, prm, sync=False),
                                           cfg.max_outer, cfg.n_cg, plan.support_samples * B, wl)
    plain = None
    if full:
        # the same data and launch shapes reconstructed with the plain model
        d = inputs.scanner_geometry(cfg, 1, full_model=True)
        d.pop("y_scale")
        p0 = pget.Plan(d.pop("n"), d.pop("n_angles"), d.pop("n_bins"), **d)
        p0.set_band_staging(args.batch >= BAND_STAGING_MIN_BATCH)
        fs0, ms0, _ = p0.lm_solve_batched(ys, f0s, m0s, prm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            fs0, ms0, _ = p0.lm_solve_batched(ys, f0s, m0s, prm, sync=False)
        torch.cuda.synchronize()
        plain = (time.perf_counter() - t1, fs0, ms0)
        roofline0, _, _ = instrumented_roofline(pget, torch, lambda: p0.lm_solve_batched(ys, f0s, m0s, prm, sync=False),
                                                cfg.max_outer, cfg.n_cg, p0.support_samples * B,
                                                "%s_batch%d" % (cfg.name, B))
    mask = inputs.fov_mask(cfg)
    ef = [np.linalg.norm((f.cpu().numpy() - t[0])[mask]) / np.linalg.norm(t[0][mask]) for f, t in zip(fs, truth)]
    em = [np.linalg.norm((m.cpu().numpy() - t[1])[mask]) / np.linalg.norm(t[1][mask]) for m, t in zip(ms, truth)]
    model = ", full discrete model" if full else ""
    out = {
        "metric": "LM reconstructions/s, scanner geometry 165^2 x 360 angles x 182 bins (%s%s)"
                  % (args.storage.upper(), model),
        "value": round(B * args.steps / el, 4), "unit": "reconstructions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * el / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else "bf16-storage/f32-compute",
        "data": "synthetic: 9x9 assemblies on a 1 mm grid, 2% Gaussian noise",
        "config": {"workload": wl,
                   "map_bands": int(plan.lib.pget_plan_jvp_bands(plan.handle)),
                   "outer": cfg.max_outer, "cg": cfg.n_cg,
                   "pixel_mm": cfg.pixel_mm, "bin_mm": cfg.bin_mm, "oversample": cfg.oversample,
                   "solver": dict({"name": args.solver, "prior_gamma": args.prior}, **opts),
                   "mu0": "water in the field of view" if args.solver == "scaled" else "zero"},
        "quality": {"f_rel_err_fov": round(float(np.mean(ef)), 4), "mu_rel_err_fov": round(float(np.mean(em)), 4),
                    "initial_f_rel_err_fov": round(float(np.mean(
                        [np.linalg.norm((f0.cpu().numpy() - t[0])[mask]) / np.linalg.norm(t[0][mask])
                         for f0, t in zip(f0s, truth)])), 4)},
    }
    out["roofline"] = roofline
    if full:
        out["config"]["full_model"] = {"psf_sigma_far_bins": cfg.psf_sigma_far_bins,
                                       "depth_factor_far": cfg.depth_factor_far}
        el0, fs0, ms0 = plain
        ef0 = [np.linalg.norm((f.cpu().numpy() - t[0])[mask]) / np.linalg.norm(t[0][mask]) for f, t in zip(fs0, truth)]
        em0 = [np.linalg.norm((m.cpu().numpy() - t[1])[mask]) / np.linalg.norm(t[1][mask]) for m, t in zip(ms0, truth)]
        out["plain_model"] = {"value": round(B * args.steps / el0, 4), "ms_per_step": round(1e3 * el0 / args.steps, 3),
                              "f_rel_err_fov": round(float(np.mean(ef0)), 4),
                              "mu_rel_err_fov": round(float(np.mean(em0)), 4), "roofline": roofline0}
    print(json.dumps(out), flush=True)


def run_deepgn(args, torch, np, inputs, pget):
    """Safeguarded Deep Gauss-Newton: K learned refinements trained per
    Alg. 1 on synthetic slices (seeds 1000+), then Alg. 2 on held-out slices
    (seeds 0..n_test-1) against plain LM at the same and at 15 outer
    iterations.  --dg-set lattice: the 128^2 9x9 lattice of the main workload
    (Poisson counts, f0 = c0, mu0 = 0, the solver defaults); scanner: the
    165^2 scanner geometry (data from the 330^2 grid, 2 % Gaussian noise)
    with a water-level start.  Both use the scaled damped step with the
    active set, for LM and Deep-GN alike.  Convolutions run without
    MIOpen (PyTorch's GEMM path), so no kernel search runs on a fresh box."""
    from paper_2604_26745_amd import refine
    torch.backends.cudnn.enabled = False
    T = lambda a: torch.tensor(a, dtype=torch.float32, device="cuda")
    log = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
    K, n_train, n_test, outer = args.dg_k, args.dg_train, args.dg_test, args.dg_outer
    if args.dg_set == "scanner":
        cfg = inputs.SCANNER_165
        geo = {}
        for o in (1, cfg.oversample):
            d = inputs.scanner_geometry(cfg, o)
            ys_ = d.pop("y_scale")
            n = d.pop("n")
            geo[o] = (pget.Plan(n, d.pop("n_angles"), d.pop("n_bins"), **d), ys_)
        plan, cscale = geo[1]
        fine, fscale = geo[cfg.oversample]
        kinds = ("full", "missing", "replaced", "medium")
        mask = inputs.fov_mask(cfg)
        water = np.where(mask, cfg.water_mu, 0.0)
        f_max, mu_max = 1.0, 0.14
        opts = SCANNER_SOLVER_OPTIONS["scaled"]
        prm = pget.SolverParams(max_outer=outer, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha, **opts,
                                alpha_decay=args.dg_decay, alpha_decay_until=args.dg_decay_until)
        wl = "deepgn_scanner9x9_n165_K%d" % K
        extra = {"solver": opts, "mu0": "water in the field of view"}
        data = "synthetic: scanner-geometry 9x9 assemblies, 2% Gaussian noise"
    else:
        cfg = inputs.MAIN_128
        plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma)
        cc = np.arange(cfg.n) - 0.5 * (cfg.n - 1)
        X, Y = np.meshgrid(cc, cc)
        mask = X ** 2 + Y ** 2 <= (0.5 * cfg.n) ** 2
        f_max, mu_max = 3.0, 0.05
        opts = SOLVER_OPTIONS["scaled"]
        prm = pget.SolverParams(max_outer=outer, n_cg=cfg.n_cg, alpha_f=cfg.alpha, alpha_mu=cfg.alpha, **opts,
                                alpha_decay=args.dg_decay, alpha_decay_until=args.dg_decay_until)
        wl = "deepgn_%s_K%d" % (cfg.name, K)
        extra = {"solver": opts, "mu0": "zero", "peak_counts": cfg.peak_counts}
        data = "synthetic: 9x9 rod lattices, Poisson counts"
    one = torch.ones((cfg.n, cfg.n), dtype=torch.float32, device="cuda")
    a1 = plan.forward(one, torch.zeros_like(one)).double().cpu().numpy()

    def sample(s_):
        if args.dg_set == "scanner":
            ff, mf = inputs.scanner_phantom(cfg, s_, kinds[s_ % 4], cfg.oversample)
            y = inputs.gaussian_noise((fscale / cscale) * fine.forward(T(ff), T(mf)).double().cpu().numpy(), cfg.noise, s_)
            tf, tm = inputs.scanner_phantom(cfg, s_, kinds[s_ % 4], 1)
            m0 = T(water)
        else:
            tf, tm = inputs.rod_lattice(cfg, s_)
            y = inputs.poisson_counts(plan.forward(T(tf), T(tm)).double().cpu().numpy(), cfg.peak_counts, s_)
            m0 = torch.zeros_like(one)
        c0 = float((a1 * y).sum() / (a1 * a1).sum())
        return T(y), (torch.full_like(one, c0), m0), (T(tf), T(tm))

    train = [sample(1000 + i) for i in range(n_train)]
    log("deepgn: %d training slices drawn" % n_train)
    t0 = time.perf_counter()
    models, rep = refine.train_networks(plan, [t[0] for t in train], [t[1] for t in train],
                                        [t[2] for t in train], prm, K=K, epochs=args.dg_epochs, mask=mask,
                                        log=log, f_max=f_max, mu_max=mu_max)
    t_train = time.perf_counter() - t0
    test = [sample(i) for i in range(n_test)]

    def err(f, mu, tr):
        tf, tm = tr[0].cpu().numpy(), tr[1].cpu().numpy()
        return (float(np.linalg.norm((f.cpu().numpy() - tf)[mask]) / np.linalg.norm(tf[mask])),
                float(np.linalg.norm((mu.cpu().numpy() - tm)[mask]) / np.linalg.norm(tm[mask])))

    res = {"lm_%d" % outer: [], "lm_15": [], "deepgn_%d" % outer: []}
    kept, calls, t_lm, t_dg, sg = 0, 0, 0.0, 0.0, []
    for y, (f0, m0), tr in test:
        torch.cuda.synchronize(); ta = time.perf_counter()
        f, mu, _ = plan.lm_solve(y, f0, m0, prm)
        torch.cuda.synchronize(); t_lm += time.perf_counter() - ta
        res["lm_%d" % outer].append(err(f, mu, tr))
        f, mu, _ = plan.lm_solve(y, f0, m0, pget.SolverParams(**{**prm.__dict__, "max_outer": 15}))
        res["lm_15"].append(err(f, mu, tr))
        st = {}
        torch.cuda.synchronize(); ta = time.perf_counter()
        f, mu, rb = refine.deep_gn_solve(plan, y, f0, m0, prm, models, st)
        torch.cuda.synchronize(); t_dg += time.perf_counter() - ta
        res["deepgn_%d" % outer].append(err(f, mu, tr))
        r = rb.to_report()
        kept += sum(r.hook_accepted)
        calls += st["hook_calls"]
        for k in range(r.iters_run):
            if not math.isnan(r.hook_pred[k]):
                sg.append((r.hook_rho[k], r.hook_pred[k] / r.pred[k]))
    summ = {k: {"f_rel_err_fov": round(float(np.mean([e[0] for e in v])), 4),
                "mu_rel_err_fov": round(float(np.mean([e[1] for e in v])), 4)} for k, v in res.items()}
    out = {
        "metric": "safeguarded Deep Gauss-Newton: reconstruction error after %d iterations vs plain LM" % outer,
        "value": summ["deepgn_%d" % outer]["f_rel_err_fov"], "unit": "relative L2 error of f in the FOV",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * t_dg / n_test, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "%s, %d training / %d test slices" % (data, n_train, n_test),
        "config": dict({"workload": wl, "outer": outer, "cg": cfg.n_cg, "cnn_params": rep.n_params,
                        "epochs": args.dg_epochs, "train_s": round(t_train, 1),
                        "alpha_decay": [args.dg_decay, args.dg_decay_until]}, **extra),
        "errors": summ, "hook_proposals_kept": kept, "hook_calls": calls,
        "safeguard": {"evaluated": len(sg), "rho_gt_eta": sum(1 for a, _ in sg if a > prm.eta),
                      "model_not_worse": sum(1 for _, b in sg if b >= 1.0),
                      "median_rho": round(max(float(np.median([a for a, _ in sg])), -1e30), 4) if sg else None,
                      "median_pred_ratio": round(float(np.median([b for _, b in sg])), 4) if sg else None},
        "train_mse": {"lm_point": [round(v, 6) for v in rep.loss_before], "network": [round(v, 6) for v in rep.loss_after]},
        "ms_per_solve": {"lm_%d" % outer: round(1e3 * t_lm / n_test, 2), "deepgn_%d" % outer: round(1e3 * t_dg / n_test, 2)},
    }
    print(json.dumps(out), flush=True)


def serving_measure(torch, pget, rate, duration, pool_n, outer, cg, solver, server="iter", capacity=8,
                    streams=4, hbm_budget_gb=64.0, check=16, plain=True):
    """Mixed-size requests (Poisson arrivals over the {64..256}^2 mix,
    early exit at tolerance 1e-4) through the continuous-batching server --
    "iter": per-size slot pools with admission at every outer-iteration
    boundary; "batch": whole batched solves on `streams` streams -- and the
    same trace through the plain per-slice solver.  `check` seeded requests
    are compared with their slice solved alone (bitwise)."""
    import numpy as np
    from paper_2604_26745_amd import serve
    plans, pool = serve.make_pool(pool_n, outer, cg)
    prm = pget.SolverParams(max_outer=outer, n_cg=cg, tol=1e-4, **SOLVER_OPTIONS[solver])
    outputs = {}
    if server == "iter":
        pools = serve.make_pools(plans, pool, prm, {n: capacity for n in plans})
        for gp in pools.values():
            gp.keep_outputs = True
        srv = serve.IterServer(pools, hbm_budget=hbm_budget_gb * 1e9)
    else:
        ex = serve.GpuExecutor(plans, pool, prm, n_slots=streams)
        srv = serve.Server(ex, hbm_budget=hbm_budget_gb * 1e9, n_slots=streams)
        print("bench: serve warm-up (graph capture per size and batch)", file=sys.stderr, flush=True)
        srv.warm()
        launch = ex.launch

        def keep(size, rs, slot):
            h = launch(size, rs, slot)
            for i, r in enumerate(rs):
                outputs[r.rid] = (h[1][0][i], h[1][1][i])
            return h
        ex.launch = keep
    reqs = serve.make_trace(rate, duration, pool, seed=0)
    print("bench: serving %d requests at %.0f/s (%s server)" % (len(reqs), rate, server), file=sys.stderr,
          flush=True)
    st = serve.run_trace(srv, reqs)
    print("bench: served %s" % st, file=sys.stderr, flush=True)
    step_stats = None
    if server == "iter":
        for gp in pools.values():
            outputs.update(gp.outputs)
        # per size: outer-iteration steps taken, and their mean device and
        # host (launch to retirement) times
        step_stats = {str(n): {"steps": gp.step_stats["steps"],
                               "gpu_ms": round(gp.step_stats["gpu_ms"] / max(gp.step_stats["steps"], 1), 2),
                               "wall_ms": round(gp.step_stats["wall_ms"] / max(gp.step_stats["steps"], 1), 2)}
                      for n, gp in sorted(pools.items())}
        print("bench: pool steps %s" % step_stats, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    picks = np.random.default_rng([0, 7]).choice(len(reqs), size=min(check, len(reqs)), replace=False)
    worst, bitwise = [0.0, 0.0], 0
    for k in picks:
        r = reqs[int(k)]
        sl = pool[r.slot]
        fa, ma, _ = plans[r.size].lm_solve(sl.y, sl.f0, sl.mu0, prm)
        f, m = outputs[r.rid]
        worst = [max(worst[0], float(torch.linalg.norm(f - fa) / torch.linalg.norm(fa))),
                 max(worst[1], float(torch.linalg.norm(m - ma) / torch.linalg.norm(ma)))]
        bitwise += int(torch.equal(f, fa) and torch.equal(m, ma))
    print("bench: served vs alone, %d requests: %d bitwise equal, max rel f %.2e mu %.2e"
          % (len(picks), bitwise, worst[0], worst[1]), file=sys.stderr, flush=True)
    if server == "iter":
        del pools, srv
    pl = {"recon_per_s": math.nan, "p50_ms": math.nan, "p99_ms": math.nan}
    if plain:
        reqs2 = serve.make_trace(rate, duration, pool, seed=0)
        pl = serve.run_plain(plans, pool, prm, reqs2)
        print("bench: plain %s" % pl, file=sys.stderr, flush=True)
    return {
        "server": server, "rate_per_s": rate, "arrival_window_s": duration, "requests": len(reqs),
        "recon_per_s": round(st["recon_per_s"], 3),
        "latency_ms": {"p50": round(st["p50_ms"], 1), "p99": round(st["p99_ms"], 1),
                       "mean": round(st["mean_ms"], 1)},
        "makespan_s": round(st["makespan_s"], 3),
        "mean_occupancy" if server == "iter" else "mean_batch": round(st["mean_batch"], 3),
        "workspace_gb": round(st["peak_in_flight_gb"], 3),
        "plain_per_slice": {"recon_per_s": round(pl["recon_per_s"], 3), "p50_ms": round(pl["p50_ms"], 1),
                            "p99_ms": round(pl["p99_ms"], 1)},
        **({"pool_steps": step_stats} if step_stats else {}),
        "check_vs_alone": {"requests": int(len(picks)), "bitwise_equal": bitwise,
                           "max_rel_l2_f": float("%.3g" % worst[0]), "max_rel_l2_mu": float("%.3g" % worst[1])},
        "config": {"solver": dict({"name": solver}, **SOLVER_OPTIONS[solver]), "pool": pool_n, "tol": 1e-4,
                   "outer": outer, "cg": cg, "capacity_per_size" if server == "iter" else "streams":
                   capacity if server == "iter" else streams},
    }


def run_serve(args, torch, pget):
    """The serving workload alone, as its own JSON line."""
    sv = serving_measure(torch, pget, args.rate, args.duration, args.pool, args.outer, args.cg, args.solver,
                         server=args.server, capacity=args.capacity, streams=args.streams,
                         hbm_budget_gb=args.hbm_budget_gb, plain=not args.no_plain)
    out = {
        "metric": "serving: LM reconstructions/s with p50/p99 latency, mixed sizes {64..256}^2",
        "value": sv["recon_per_s"], "unit": "reconstructions/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(1e3 * sv["makespan_s"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": dict({"workload": "serve_poisson_%g_per_s_%gs" % (args.rate, args.duration)}, **sv["config"]),
        "serving": sv,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported "
              "(independent slices would shard across GPUs with no communication)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2604_26745_amd import inputs, pget

    if not os.path.exists(pget.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "mixed":
        run_mixed(args, torch, np, inputs, pget)
        return
    if args.workload == "deepgn":
        run_deepgn(args, torch, np, inputs, pget)
        return
    if args.workload == "scanner":
        run_scanner(args, torch, np, inputs, pget)
        return
    if args.workload == "serve":
        run_serve(args, torch, pget)
        return
    base = {64: inputs.SMALL_64, 128: inputs.MAIN_128, 256: inputs.LARGE_256}[args.grid]
    cfg = inputs.scaled(base, max_outer=args.outer, n_cg=args.cg)
    plan = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma, storage=args.storage)
    B = args.batch
    # maps too large for LDS (256^2): band staging pays for large batches
    bands = plan.set_band_staging(B >= BAND_STAGING_MIN_BATCH)
    if args.autotune:
        print("bench: autotune %s" % plan.autotune(B), file=sys.stderr, flush=True)
    ys, f0s, m0s = make_inputs(plan, cfg, B, torch, inputs, np)
    prior = prior_tensors(args.prior, 0.05, *inputs.lattice_rod_prior(cfg), torch, np)
    prm = [pget.SolverParams(max_outer=cfg.max_outer, n_cg=cfg.n_cg, alpha_f=cfg.alpha,
                             alpha_mu=cfg.alpha, **SOLVER_OPTIONS[args.solver], **prior) for _ in range(B)]
    print("bench: %d slices of %s, %d outer x %d CG, warmup %d, steps %d"
          % (B, cfg.name, cfg.max_outer, cfg.n_cg, args.warmup, args.steps), file=sys.stderr,
          flush=True)
    for w in range(args.warmup):
        plan.lm_solve_batched(ys, f0s, m0s, prm)
        print("bench: warmup %d done" % (w + 1), file=sys.stderr, flush=True)

    # timed region: K steps of the production path (the solver's kernel
    # sequence replayed as a HIP graph)
    torch.cuda.synchronize()
    # events on the solver's stream between steps (no extra synchronisation)
    # give the per-step times behind the median and the minimum
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    step_ev[0].record()
    reports = None
    for s in range(args.steps):
        fs, ms, reports = plan.lm_solve_batched(ys, f0s, m0s, prm, sync=False)
        step_ev[s + 1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    step_ms = sorted(step_ev[s].elapsed_time(step_ev[s + 1]) for s in range(args.steps))
    ms_step = 1e3 * elapsed / args.steps
    value = B * args.steps / elapsed
    reps = [r.to_report() for r in reports]
    assert all(r.status == 0 for r in reps), "solver reported a failure"
    print("bench: timed %.3f s (%d steps)" % (elapsed, args.steps), file=sys.stderr, flush=True)

    workload = "%s_batch%d" % (cfg.name, B) + ("_bf16" if args.storage == "bf16" else "")
    roofline, kt, instrumented_s = instrumented_roofline(
        pget, torch, lambda: plan.lm_solve_batched(ys, f0s, m0s, prm, sync=False), cfg.max_outer, cfg.n_cg,
        plan.support_samples * B, workload)
    # HBM GB/s of the projector (A, the ray march) and both Jacobian products:
    # committed counter bytes per launch over this run's average launch time
    kernel_gbs = {}
    for cls, kname in (("march", "k_march"), ("jvp", "k_jvp_lin"), ("vjp", "k_vjp_lin")):
        b = traffic_from_profile(kname, workload)
        cls_ms, n = kt[cls]
        if b and n:
            kernel_gbs[kname] = round(b / (cls_ms / 1e3 / n) / 1e9, 1)
    kernel_share = {k: round(v[0] / (1e3 * instrumented_s), 4) for k, v in kt.items()}
    if kernel_gbs:
        roofline["kernel_hbm_gbs"] = kernel_gbs

    single = None
    if not args.no_single:
        ps = prm[:1]
        plan.lm_solve(ys[0], f0s[0], m0s[0], ps[0])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        plan.lm_solve(ys[0], f0s[0], m0s[0], ps[0])
        torch.cuda.synchronize()
        single = {"latency_ms": round(1e3 * (time.perf_counter() - t2), 2)}
        single["recon_per_s"] = round(1e3 / single["latency_ms"], 3)

    # the BF16-storage variant on the same inputs and options (weights and
    # staged search direction in bfloat16, arithmetic in FP32)
    bf16 = None
    if args.storage == "fp32" and not args.no_bf16_variant:
        plan_b = pget.Plan(cfg.n, cfg.n_angles, cfg.n_bins, psf_sigma=cfg.psf_sigma, storage="bf16")
        plan_b.set_band_staging(B >= BAND_STAGING_MIN_BATCH)
        for _ in range(max(1, args.warmup)):
            plan_b.lm_solve_batched(ys, f0s, m0s, prm)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(args.steps):
            fb, mb, rb_ = plan_b.lm_solve_batched(ys, f0s, m0s, prm, sync=False)
        torch.cuda.synchronize()
        el_b = time.perf_counter() - tb
        assert all(r.to_report().status == 0 for r in rb_), "BF16 solver reported a failure"
        bf16 = {"value": round(B * args.steps / el_b, 4), "unit": "reconstructions/s",
                "ms_per_step": round(1e3 * el_b / args.steps, 3), "speedup_vs_fp32": round((B * args.steps / el_b) / value, 3),
                "dtype": "bf16-storage/f32-compute", "quality": quality(fb, mb, cfg, inputs, np)}
        print("bench: BF16 storage %.2f recon/s" % bf16["value"], file=sys.stderr, flush=True)
        del plan_b

    # the serving half of the metric: a Poisson trace over the mixed sizes
    serving = None
    if args.serve_rate > 0 and args.grid == 128 and args.storage == "fp32":
        # both servers on the same trace: whole batched solves on concurrent
        # streams (the headline, with the plain per-slice solver beside it)
        # and per-size slot pools admitting at every outer iteration
        serving = serving_measure(torch, pget, args.serve_rate, args.serve_duration, args.pool, args.outer,
                                  args.cg, args.solver, server="batch", streams=args.streams,
                                  hbm_budget_gb=args.hbm_budget_gb)
        serving["iteration_level"] = serving_measure(
            torch, pget, args.serve_rate, args.serve_duration, args.pool, args.outer, args.cg, args.solver,
            server="iter", capacity=args.capacity, hbm_budget_gb=args.hbm_budget_gb, plain=False, check=4)

    cpu = None
    if not args.no_cpu_baseline:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        print("bench: CPU oracle sample on %d workers" % workers, file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, workers)

    out = {
        "metric": "LM reconstructions/s at %d^2 x %d angles (%s)" % (cfg.n, cfg.n_angles, args.storage.upper()),
        "value": round(value, 4),
        "unit": "reconstructions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "step_ms": {"median": round(step_ms[len(step_ms) // 2], 3), "min": round(step_ms[0], 3)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "fp32" else "bf16-storage/f32-compute",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "storage": args.storage,
            "map_bands": bands,
            "slices_per_step": B,
            "grid": cfg.n, "angles": cfg.n_angles, "bins": cfg.n_bins, "psf_sigma": cfg.psf_sigma,
            "outer": cfg.max_outer, "cg": cfg.n_cg, "alpha": cfg.alpha,
            "solver": dict({"name": args.solver, "prior_gamma": args.prior}, **SOLVER_OPTIONS[args.solver]),
            "phantom": "%dx%d rod lattice, r=%g px, pitch %g px, %d empty rods, Poisson peak %g" % (
                cfg.n_rods, cfg.n_rods, cfg.rod_radius, cfg.pitch, cfg.n_empty, cfg.peak_counts),
        },
        "quality": dict(quality(fs, ms, cfg, inputs, np),
                        start=quality(f0s, m0s, cfg, inputs, np)),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "bf16_storage": bf16,
        "kernel_time_share": kernel_share,
        "instrumented_step_ms": round(1e3 * instrumented_s, 3),
        "single_slice": single,
        "serving": serving,
        "final_phi_mean": float(np.mean([r.phi[-1] for r in reps])),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
