"""Benchmark of the many-variable VMC hot path on one MI355X.

A step is one SR iteration of the 10x10 periodic Hubbard model (U = 8,
N_e = 100, unconstrained pair amplitudes f_ij: N_p = 10002): 4096 walkers x
10 sweeps (100 proposals each), the local energy and O_k of every walker
after the last sweep, then the SR statistics, the S build, the Cholesky
solve, the parameter update and the full double refresh of every walker.
The headline runs every step in double precision (no periodic refresh
inside the sampling, S on the FP64 matrix cores); the same steps in mixed precision
(single-precision sweeps and O, double refresh after every 32 applied
updates (accepted hops, the steps that change X^-1),
split-bf16 S with FP32 accumulation, double solve) are reported beside it
with the error of every mixed result against the double path.  Inputs are
seeded and synthetic and resident in HBM before timing starts.

Printed: one JSON line with the walker hop-update rate (proposals/s) over
whole steps, the S-build rates, the roofline of the dominant kernel, the
mixed-precision run, per-result precision errors, the 8x8, 16x16-RBM and
32-cluster workloads, and the CPU oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--skip-legs]
    python bench.py --rbm-gain [--sr-steps K]   # 16x16 PJ vs PJ x RBM training
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0
METRIC = "walker hop-updates/s + SR S-build TFLOP/s, batched/mixed vs plain FP64"
HEADLINE = "sq10_u8"
# no periodic refresh on the double path: over a step's 1000 proposals its inverse
# drifts at the 1e-13 level (the double replays hold 1e-10 over 2000 proposals
# without one), and every step ends with the full double refresh after the update
FP64_REFRESH = 0
MIXED_REFRESH = 32      # applied updates between double refreshes on the mixed path
MIXED_UNIT = "updates"  # what MIXED_REFRESH counts (accepted hops: the steps that change X^-1)
KINDS = ["sweep", "refresh", "measure", "sr_stats", "s_build", "sr_solve"]
# the dominant kernel of the headline step and the committed counter summary
# of its HBM traffic (bench reports traffic = null once its sources change)
TRAFFIC_SUMMARY = "sweep_ap_fp64_sq10_traffic.txt"
TRAFFIC_SOURCES = ("k_sweep_ap.hip", "ap_walk.h", "common.h", "launch.h")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_sr_workload(wl, precision, steps, warmup, refresh_every, solver="chol", sweep_threads=0,
                    use_graph=True, autotune=False, build_s=True, cg_tol=1e-10, cg_maxit=1000,
                    schedule="buckets", refresh_unit="proposals"):
    """Time whole SR steps of every instance of the workload.  With use_graph
    the sampling part of a step (the sweeps and the measurements) is captured
    once into a HIP graph and replayed; the SR build and update run eagerly.
    With autotune the sweep variant of every instance is chosen by timing
    after the warm-up."""
    import numpy as np
    import torch

    from paper_1711_11418_amd import MVMC

    insts = wl["instances"]
    params = np.concatenate([i.params0 for i in insts])
    sweeps = wl["sweeps"]
    every = wl.get("sample_every", 1)   # sweeps between samples
    slots = sweeps // every
    side = torch.cuda.Stream()
    tuned = None
    with torch.cuda.stream(side):
        ctx = MVMC(insts, params, precision=precision, refresh_every=refresh_every,
                   seed=wl["sampler_seed"], n_slots=slots, solver=solver, build_s=build_s,
                   sweep_threads=sweep_threads, stream=side, schedule=schedule,
                   refresh_unit=refresh_unit)
        for _ in range(wl["warmup"]):   # one launch per sweep, as in the timed steps
            ctx.sample_async(1)
        torch.cuda.synchronize()
        if autotune:
            ms = ctx.autotune(3)
            tuned = {"variants": ctx.sweep_variants(),
                     "ms_by_variant": np.where(np.isnan(ms), None, ms).tolist()}

        def sampling(profile=False):
            acc = 0
            for s in range(slots):
                if profile:
                    acc += int(np.sum(ctx.sample(every)))
                else:
                    ctx.sample_async(every)
                ctx.measure(s)
            return acc

        escalations, cg_iters, errs = [], [], []

        def sr():
            E, Er, V = ctx.build_sr(slots, with_S=build_s)
            it = ctx.sr_update(dtau=wl["dtau"], eps_rel=wl["eps_rel"], eps_abs=wl["eps_abs"],
                               solver=solver, cg_tol=cg_tol, cg_maxit=cg_maxit)
            if solver == "chol":
                escalations.append(int(np.max(it)))
            else:
                cg_iters.append(int(np.max(it)))
            errs.append([float(e) for e in Er])
            return [float(e) for e in E]

        for _ in range(warmup):
            sampling()
            sr()
        graph = None
        if use_graph:
            torch.cuda.synchronize()
            graph = ctx.capture_sampling(every, range(slots))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        energies = []
        for _ in range(steps):
            if graph is not None:
                graph.replay()
            else:
                sampling()
            energies.append(sr())
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # one more step, eager, with HIP events around every kernel group
        ctx.sample(0)          # read and clear the accepted counters
        ctx.timing(True)
        accepted = sampling(profile=True)
        sr()
        ms, calls = ctx.timing(False)
        variants = ctx.sweep_variants()
        torch.cuda.synchronize()
        ctx.close()
    per_sweep = sum(i.n_walkers * i.n_elec for i in insts)
    proposals = steps * sweeps * per_sweep
    i0 = insts[0]
    return {
        "seconds": dt, "proposals": proposals, "rate": proposals / dt,
        "ms_per_step": 1e3 * dt / steps,
        "energies": [e[0] for e in energies] if len(insts) == 1 else energies,
        "energy_errors": [e[0] for e in errs[warmup:]] if len(insts) == 1 else errs[warmup:],
        "accept_ratio": accepted / (sweeps * per_sweep), "kernel_ms": ms.tolist(),
        "kernel_calls": calls.tolist(), "W": i0.n_walkers, "ne": i0.n_elec, "np": i0.n_params,
        "ns": i0.n_sites, "sweeps": sweeps, "N": slots * i0.n_walkers, "graph": graph is not None,
        "autotune": tuned, "variants": variants, "cholesky_shift_raises": escalations,
        "n_hidden": i0.n_hidden,
        "cg_iterations": cg_iters, "steps": steps,
    }


def km(r):
    return dict(zip(KINDS, r["kernel_ms"]))


def sweep_bytes(r, wsize, model):
    """Bytes of the sweeps of one SR step.  "method": every proposal reads one
    row of X^-1 (N_e w) and every accepted one reads and writes all of it
    (2 N_e^2 w).  "ap": the anti-parallel-block kernel reads one column or row
    of M^-1 (n w, n = N_e/2) per proposal and 3 n^2 w per accepted one (v or
    t, then the rank-1 update).  "full": the full-X^-1 LDS/HBM kernel reads
    half a row per proposal and one n x n block plus two blocks read and
    written per accepted one (1.25 N_e^2 w)."""
    ne = r["ne"]
    n = ne // 2
    props = r["proposals"] / max(r["steps"], 1)
    acc = props * r["accept_ratio"]
    if model == "method":
        return props * ne * wsize + acc * 2 * ne * ne * wsize
    if model == "ap":
        return props * n * wsize + acc * 3 * n * n * wsize
    return props * n * wsize + acc * 1.25 * ne * ne * wsize


def sweep_model_of(variant):
    if variant.startswith("ap"):
        return "ap"
    if variant.startswith("reg"):
        return "method"
    return "full"


def sweep_hbm(r, wsize):
    """Modelled HBM rate of the sweeps of one SR step on the kernel's own
    byte model, with the method's model beside it."""
    ms = km(r)["sweep"]
    own = sweep_model_of(r["variants"][0])
    b_own = sweep_bytes(r, wsize, own)
    b_met = sweep_bytes(r, wsize, "method")
    return {"kernel": r["variants"][0], "byte_model": own, "sweep_ms_per_step": ms,
            "bytes_per_step": b_own, "gbs": b_own / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": b_own / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "method_model_bytes_per_step": b_met,
            "method_model_frac_of_hbm_peak": b_met / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def measure_hbm(r, wsize):
    """E_loc and O_k: every sample reads the opposite-spin half of X^-1
    (N_e^2/2 w, the part the kernel reads) and writes its O row (N_p w)."""
    ne, npar = r["ne"], r["np"]
    bytes_ = r["N"] * (ne * ne // 2 + npar) * wsize
    ms = km(r)["measure"]
    return {"bytes_per_step": bytes_, "ms_per_step": ms, "gbs": bytes_ / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def s_build_rates(r, mixed):
    """S = O~^T O~ / N over the upper triangle: N N_p (N_p + 1) flops; the
    split-bf16 build issues three bf16 products."""
    N, npar = r["N"], r["np"]
    if r["kernel_calls"][4] == 0:
        return None
    ms = km(r)["s_build"] / r["kernel_calls"][4]
    fl = N * npar * (npar + 1)
    out = {"shape": [N, npar], "ms": ms, "tflops": fl / (ms * 1e-3) / 1e12}
    if mixed:
        out.update({"kernel": "split-bf16 MFMA (hi.hi + hi.lo + lo.hi), FP32 accumulate",
                    "issued_bf16_tflops": 3 * fl / (ms * 1e-3) / 1e12,
                    "issued_frac_of_bf16_peak": 3 * fl / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS})
    else:
        out.update({"kernel": "FP64 MFMA 16x16x4",
                    "frac_of_fp64_peak": fl / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS})
    return out


def refresh_rate(r):
    """Block-route refresh: Gauss-Jordan inversion of the n x n block,
    2 n^3 flops per walker."""
    n = r["ne"] // 2
    calls = max(r["kernel_calls"][1], 1)
    ms = km(r)["refresh"]
    fl = r["kernel_calls"][1] * r["W"] * 2.0 * n ** 3
    return {"launch_groups_per_step": calls, "ms_per_step": ms,
            "fp64_tflops": fl / (ms * 1e-3) / 1e12 if ms > 0 else None,
            "flops_model": "2 (N_e/2)^3 per walker per refresh"}


def step_summary(r, wsize, mixed):
    k = km(r)
    return {"value": r["rate"], "unit": "hop-updates/s", "ms_per_step": r["ms_per_step"],
            "accept_ratio": r["accept_ratio"], "sweep_variant": r["variants"],
            "kernel_ms_per_step": k, "sweep_hbm": sweep_hbm(r, wsize),
            "measure_hbm": measure_hbm(r, wsize), "s_build": s_build_rates(r, mixed),
            "refresh": refresh_rate(r),
            "cholesky_fp64_tflops": (r["np"] ** 3 / 3 / (k["sr_solve"] * 1e-3) / 1e12
                                     if r["cholesky_shift_raises"] else None),
            "cholesky_shift_raises": r["cholesky_shift_raises"],
            "energy_per_site": [e / r["ns"] for e in r["energies"]],
            "energy_error_per_site": [e / r["ns"] for e in r["energy_errors"]]}


def precision_errors():
    """Mixed against double on the 10x10 workload, result by result.

    The mixed context is warmed up; its configurations, counters and empty
    lists are loaded into a double context and both are recomputed in double,
    so every comparison below starts from the same walkers:
      ratios   one sweep traced on both (compared until a decision differs)
      E_loc, O measured on both at the loaded configurations
      S, g     built on both from those samples (split-bf16 vs FP64)
      dalpha   the SR step of both (double Cholesky of each S_reg)
    and energies at equal sample counts from two independent chains
    (different Philox keys), with sigma = std(walker means)/sqrt(W)."""
    import numpy as np
    import torch

    from mvmc_inputs import workload
    from paper_1711_11418_amd import MVMC

    wl = workload(HEADLINE)
    inst = wl["instances"][0]
    kw = dict(seed=wl["sampler_seed"], n_slots=1, solver="chol", build_s=True)
    m = MVMC([inst], inst.params0, precision="mixed", refresh_every=MIXED_REFRESH,
             refresh_unit=MIXED_UNIT, **kw)
    d = MVMC([inst], inst.params0, precision="fp64", refresh_every=FP64_REFRESH, **kw)
    m.sample(40)
    pos, cnt, emp = m.get_state(with_empty=True)
    d.set_state(pos.cpu().numpy(), cnt.cpu().numpy(), emp.cpu().numpy())
    m.refresh()
    out = {}
    # E_loc and O at the same configurations
    m.measure(0)
    d.measure(0)
    em, ed = m.eloc_of(0, 1).double(), d.eloc_of(0, 1)
    Om, Od = m.O_of(0, 1).double(), d.O_of(0, 1)
    rel_e = (em - ed).abs() / ed.abs().clamp_min(1e-300)
    dO = (Om - Od).abs()
    out["eloc"] = {"max_rel": float(rel_e.max()), "median_rel": float(rel_e.median())}
    out["O"] = {"max_abs_over_max_O": float(dO.max() / Od.abs().max()),
                "median_abs": float(dO.median())}
    # S, g, energy and the SR step from these samples
    Em, Erm, _ = m.build_sr(1)
    Ed, Erd, _ = d.build_sr(1)
    S_err = float((m.S_of(0).double() - d.S_of(0)).abs().max() / d.S_of(0).abs().max())
    g_err = float((m.g - d.g).abs().max() / d.g.abs().max())
    out["S"] = {"max_abs_over_max_S": S_err}
    out["g"] = {"max_abs_over_max_g": g_err}
    out["mean_energy_same_samples"] = {"mixed": float(Em[0]), "fp64": float(Ed[0]),
                                       "diff_over_sigma": float((Em[0] - Ed[0]) / Erd[0])}
    a = dict(dtau=wl["dtau"], eps_rel=wl["eps_rel"], eps_abs=wl["eps_abs"], solver="chol")
    m.sr_update(**a)
    d.sr_update(**a)
    da = float(torch.linalg.norm(m.dparams - d.dparams) / torch.linalg.norm(d.dparams))
    out["dalpha"] = {"rel_l2": da}
    m.close()
    d.close()
    # ratios over one sweep from identical states
    m = MVMC([inst], inst.params0, precision="mixed", refresh_every=MIXED_REFRESH,
             refresh_unit=MIXED_UNIT, **kw)
    d = MVMC([inst], inst.params0, precision="fp64", refresh_every=FP64_REFRESH, **kw)
    m.sample(40)
    pos, cnt, emp = m.get_state(with_empty=True)
    d.set_state(pos.cpu().numpy(), cnt.cpu().numpy(), emp.cpu().numpy())
    m.refresh()
    m.enable_trace(inst.n_elec)
    d.enable_trace(inst.n_elec)
    m.sample(1)
    d.sample(1)
    tm, td = m.trace_records(), d.trace_records()
    m.close()
    d.close()
    diff = tm["accepted"] != td["accepted"]
    first = np.where(diff.any(axis=1), diff.argmax(axis=1), tm.shape[1])
    mask = np.arange(tm.shape[1])[None, :] <= np.minimum(first, tm.shape[1] - 1)[:, None]
    mask &= td["i_new"] >= 0
    rr = np.abs(tm["ratio"] - td["ratio"])[mask] / np.maximum(np.abs(td["ratio"][mask]), 1e-300)
    out["ratio"] = {"compared": int(mask.sum()), "median_rel": float(np.median(rr)),
                    "p99_rel": float(np.percentile(rr, 99)), "max_rel": float(rr.max()),
                    "walkers_with_a_differing_decision": int(diff.any(axis=1).sum()),
                    "walkers": int(tm.shape[0])}
    # energies at equal sample counts from independent chains
    res = {}
    for prec, R, seed in (("mixed", MIXED_REFRESH, 91), ("fp64", FP64_REFRESH, 92)):
        slots = 8
        c = MVMC([inst], inst.params0, precision=prec, refresh_every=R, seed=seed,
                 n_slots=slots, solver="cg", build_s=False,
                 refresh_unit=MIXED_UNIT if prec == "mixed" else "proposals")
        c.sample(40)
        for s in range(slots):
            c.sample_async(5)
            c.measure(s)
        E, Er, _ = c.build_sr(slots, with_S=False)
        res[prec] = (float(E[0]), float(Er[0]))
        c.close()
    z = (res["mixed"][0] - res["fp64"][0]) / np.hypot(res["mixed"][1], res["fp64"][1])
    out["energy_equal_samples"] = {
        "samples": 8 * inst.n_walkers, "mixed": res["mixed"], "fp64": res["fp64"],
        "z": float(z), "within_2_sigma": bool(abs(z) < 2.0),
        "note": "(E, sigma) per precision; 8 samples per walker, 5 sweeps apart, after 40 "
                "sweeps, initial parameters"}
    return out


def s_build_leg():
    """Split-bf16 S build at the 4096-sample x 10^4-parameter shape, at the
    tile side the library's tuner picks on this data."""
    import torch

    from mvmc_inputs import workload
    from paper_1711_11418_amd import MVMC

    wl = workload(HEADLINE)
    inst = wl["instances"][0]
    ctx = MVMC([inst], inst.params0, precision="mixed", refresh_every=MIXED_REFRESH,
               seed=wl["sampler_seed"], n_slots=1, solver="cg", build_s=True,
               refresh_unit=MIXED_UNIT)
    ctx.autotune(1)          # sweep variants, and arms the S tile tuner
    ctx.sample(2)
    ctx.measure(0)
    ctx.build_sr(1)          # tunes the tile side on this O (untimed)
    sides, tune_ms = ctx.s_tiles()
    torch.cuda.synchronize()
    ctx.timing(True)
    reps = 3
    for _ in range(reps):
        ctx.build_sr(1)
    ms, calls = ctx.timing(False)
    ctx.close()
    N, npar = inst.n_walkers, inst.n_params
    flops = N * npar * (npar + 1)
    avg = ms[4] / max(calls[4], 1)
    # context: the vendor GEMM (torch.mm, hipBLASLt) forming the same
    # three-pass bf16 product as a full square [N_p x 3N] x [3N x N_p]
    g = torch.Generator(device="cuda").manual_seed(1)
    a = torch.randn(npar, 3 * N, device="cuda", dtype=torch.bfloat16, generator=g)
    b = torch.randn(3 * N, npar, device="cuda", dtype=torch.bfloat16, generator=g)
    for _ in range(2):
        c = a @ b
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        c = a @ b
    e1.record()
    torch.cuda.synchronize()
    gemm_ms = e0.elapsed_time(e1) / 3
    del a, b, c
    tile = sides[0] or 64
    nt = -(-npar // tile)
    rows = -(-N // 32) * 32 if sides[0] else -(-N // 16) * 16
    issued = 3 * 2 * rows * tile * tile * nt * (nt + 1) // 2
    return {"shape": [N, npar], "ms": avg, "tflops": flops / (avg * 1e-3) / 1e12,
            "algorithmic_flops": flops, "issued_mfma_tflops": issued / (avg * 1e-3) / 1e12,
            "issued_frac_of_bf16_peak": issued / (avg * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
            "tile": tile,
            "tuning_ms_by_tile": {"128": float(tune_ms[0][0]), "192": float(tune_ms[0][1]),
                                  "256": float(tune_ms[0][2])},
            "vendor_gemm_same_product_ms": gemm_ms,
            "note": "time of the S kernels only (centring and split excluded)"}


def reg_sweep_roofline(r):
    """The register-resident sweep keeps the walker's X^-1 in VGPRs for the
    whole launch, so neither HBM nor the method's byte model bounds it; its
    algorithmic flops (2 N_e per proposal, 6 N_e^2 per accepted one) against
    the FP64 vector peak, with the launch's latency chain the real limit."""
    ne = r["ne"]
    launches = max(r["kernel_calls"][0], 1)
    avg_ms = km(r)["sweep"] / launches
    props = r["proposals"] / max(r["steps"], 1) / launches
    acc = r["accept_ratio"] * props
    flops = props * 2 * ne + acc * 6 * ne * ne
    return {"avg_launch_ms": avg_ms, "alg_flops_per_launch": flops,
            "fp64_tflops": flops / (avg_ms * 1e-3) / 1e12,
            "frac_of_fp64_peak": flops / (avg_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "bound": "latency (one wavefront per walker, dependent proposal chain)"}


def sq8_leg(steps):
    """8x8 Hubbard, U = 4, N_e = 64, 2x2-sublattice f + distance Jastrow +
    Gutzwiller (N_p = 271), 1024 walkers x 200 sweeps with a measurement
    after every sweep, FP64 S and Cholesky; double and mixed."""
    from mvmc_inputs import workload
    wl = workload("sq8_u4")
    r = run_sr_workload(wl, "fp64", steps, 1, wl["refresh_every"])
    m = run_sr_workload(wl, "mixed", steps, 1, MIXED_REFRESH, refresh_unit=MIXED_UNIT)
    out = {"fp64": step_summary(r, 8, False), "mixed": step_summary(m, 4, True)}
    out["fp64"]["sweep_reg_alu"] = reg_sweep_roofline(r)
    out["mixed_speedup_vs_fp64"] = m["rate"] / r["rate"]
    return out


def lanczos_leg(sr_steps=30, slots=20):
    """First-step power-Lanczos (section 3.4) on the 8x8, U = 4 workload: the
    state is trained by sr_steps FP64 SR steps, then F(x, H) and F(x, H^2)
    are measured on 1024 walkers x `slots` samples one sweep apart, and the
    moments give alpha_1 and E_1(alpha_1) against E = h1.  Timed: the
    F(x, H^2) kernel (HIP events around its launches)."""
    import numpy as np

    from mvmc_inputs import workload
    from paper_1711_11418_amd import MVMC
    wl = workload("sq8_u4")
    inst = wl["instances"][0]
    ctx = MVMC([inst], inst.params0, seed=wl["sampler_seed"], n_slots=10, solver="chol",
               build_s=True, refresh_every=wl["refresh_every"])
    ctx.sample(wl["warmup"])
    for _ in range(sr_steps):
        for s in range(10):
            ctx.sample_async(1)
            ctx.measure(s)
        ctx.build_sr(10)
        ctx.sr_update(dtau=wl["dtau"], eps_rel=wl["eps_rel"], eps_abs=wl["eps_abs"])
    p = ctx.params.cpu().numpy().copy()
    ctx.close()
    ev = MVMC([inst], p, seed=wl["sampler_seed"] + 3, n_slots=slots, build_s=False, solver="cg",
              refresh_every=wl["refresh_every"])
    ev.sample(wl["warmup"])
    ms = 0.0
    for s in range(slots):
        ev.sample(1)
        ev.timing(True)
        ev.measure_h2(s)
        ms += ev.timing(False)[0][2]
    out = ev.lanczos_first_step(slots)[0]
    f1 = ev.f1.cpu().numpy()[:slots * inst.n_walkers].reshape(slots, inst.n_walkers)
    wmean = f1.mean(axis=0)
    sigma = wmean.std(ddof=1) / np.sqrt(inst.n_walkers)
    ev.close()
    ns, n = inst.n_sites, inst.n_up
    gemm_flops = 2.0 * n * ns * (2 * n + ns)
    per_call = ms / slots
    return {"workload": "sq8_u4 after %d FP64 SR steps" % sr_steps, "walkers": inst.n_walkers,
            "samples": slots * inst.n_walkers,
            "E_per_site": out[0] / ns, "sigma_E_per_site": sigma / ns,
            "alpha_1": out[4], "E1_per_site": out[5] / ns,
            "gain_per_site": (out[0] - out[5]) / ns, "moments": out[:4].tolist(),
            "real_roots": int(out[6]),
            "h2_kernel_ms_per_1024_walkers": per_call,
            "h2_walkers_per_s": inst.n_walkers / (per_call * 1e-3),
            "products_tflops": gemm_flops * inst.n_walkers / (per_call * 1e-3) / 1e12}


def uhf_start(inst, m0=0.3, mix=0.5, iters=2000, noise=0.02, seed=17):
    """Initial parameters from the unrestricted Hartree-Fock solution, as the
    paper starts its Hubbard optimisations (section 4.1.1): per spin
    H_s = T + U <n_{i,-s}> n_{i,s} iterated to self-consistency from a Neel
    seed on the bipartite lattice, the lowest N_s orbitals Phi_s of each
    spin, and f_ij = sum_n Phi_{i n up} Phi_{j n dn} (Eq. fijSL), averaged
    over the members of each f slot and scaled to max |f| = 1, plus
    Gaussian noise of `noise` (seeded): the exact mean-field amplitude is so
    symmetric that translated copies of it vanish identically on some
    configurations, and the projected sweep needs every term invertible.
    Gutzwiller and Jastrow parameters start at zero."""
    import numpy as np
    ns = inst.n_sites
    T = np.zeros((ns, ns))
    nb = [[] for _ in range(ns)]
    for (i, j), t in zip(np.asarray(inst.bonds), inst.bond_t):
        T[i, j] = T[j, i] = -t
        nb[i].append(j)
        nb[j].append(i)
    color = -np.ones(ns, dtype=int)
    color[0] = 0
    todo = [0]
    while todo:
        i = todo.pop()
        for j in nb[i]:
            if color[j] < 0:
                color[j] = 1 - color[i]
                todo.append(j)
    U = np.asarray(inst.U, dtype=float)
    stag = 1.0 - 2.0 * color
    nu = inst.n_up / ns + m0 * stag
    nd = inst.n_dn / ns - m0 * stag
    for _ in range(iters):
        _, vu = np.linalg.eigh(T + np.diag(U * nd))
        _, vd = np.linalg.eigh(T + np.diag(U * nu))
        pu, pd = vu[:, :inst.n_up], vd[:, :inst.n_dn]
        nu1, nd1 = (pu ** 2).sum(1), (pd ** 2).sum(1)
        done = max(np.abs(nu1 - nu).max(), np.abs(nd1 - nd).max()) < 1e-12
        nu, nd = mix * nu1 + (1 - mix) * nu, mix * nd1 + (1 - mix) * nd
        if done:
            break
    f = pu @ pd.T
    fidx = np.asarray(inst.f_idx)
    fv = np.zeros(inst.n_f)
    cnt = np.zeros(inst.n_f)
    for i in range(ns):
        for j in range(ns):
            if fidx[i, j] >= 0:
                fv[fidx[i, j]] += f[i, j]
                cnt[fidx[i, j]] += 1
    fv /= np.maximum(cnt, 1)
    fv /= np.abs(fv).max()
    fv += noise * np.random.default_rng(seed).standard_normal(inst.n_f)
    p = np.zeros(inst.n_params)
    p[:inst.n_f] = fv
    return p


def projection_leg(sr_steps=1500, slots=4):
    """4x4 Hubbard, U = 4, t = 1, half filling (section 4.1.1, Table 3): a
    2x2-sublattice pair amplitude (64 slots), one Gutzwiller and 5 Jastrow
    distance classes (N_p = 70), 1024 walkers, FP64.  From the UHF start
    (uhf_start) the plain state is trained by sr_steps SR steps (`slots`
    samples per walker one sweep apart, Cholesky); from those parameters two
    runs of sr_steps more steps follow with the same sampler seed: with the
    momentum projection over the four translations of the 2x2 cell at K = 0
    (with the sublattice structure, the full K = 0 projection of section
    3.2.2) and without it.  Energies from 32 samples per walker, 2 sweeps
    apart; also the UHF start with and without the projection.  The paper's
    row for this state also carries the total-spin projection, which is not
    built here: its numbers are context, not a target.  Timed: the sweep
    kernels (HIP events) over the last 20 steps of each run."""
    import copy

    import numpy as np

    from mvmc_inputs import workload
    from paper_1711_11418_amd import MVMC
    wl = workload("sq4_u4_proj4")
    proj = wl["instances"][0]
    plain = copy.deepcopy(proj)
    plain.proj_q, plain.proj_w = None, None
    ns = proj.n_sites

    def train(inst, p0, tag, seed_off):
        ctx = MVMC([inst], p0, seed=wl["sampler_seed"] + seed_off, n_slots=slots,
                   solver="chol", build_s=True, refresh_every=wl["refresh_every"])
        ctx.sample(wl["warmup"])
        hist = []
        timed = min(20, sr_steps)
        t0 = time.perf_counter()
        for it in range(sr_steps):
            if it == sr_steps - timed:
                ctx.timing(True)
            for s in range(slots):
                ctx.sample_async(1)
                ctx.measure(s)
            E, Ee, _ = ctx.build_sr(slots)
            ctx.sr_update(dtau=wl["dtau"], eps_rel=wl["eps_rel"], eps_abs=wl["eps_abs"])
            hist.append(float(E[0]) / ns)
            if it % 250 == 0 or it == sr_steps - 1:
                log(f"[projection] {tag} step {it}: E/N = {hist[-1]:.5f} "
                    f"+- {float(Ee[0]) / ns:.5f}")
        train_s = time.perf_counter() - t0
        ms, _ = ctx.timing(False)
        p = ctx.params.cpu().numpy().copy()
        ctx.close()
        props = timed * slots * inst.n_elec * inst.n_walkers
        return p, {"sr_steps": sr_steps, "train_seconds": train_s,
                   "history_per_site_every_50": hist[::50],
                   "sweep_hop_updates_per_s": props / (ms[0] * 1e-3),
                   "ms_per_sr_step": train_s * 1e3 / sr_steps}

    def evaluate(inst, params):
        ev_slots = 32
        ev = MVMC([inst], params, seed=wl["sampler_seed"] + 99, n_slots=ev_slots, solver="cg",
                  build_s=False, refresh_every=wl["refresh_every"])
        ev.sample(wl["warmup"])
        for s in range(ev_slots):
            ev.sample_async(2)
            ev.measure(s)
        E, Ee, _ = ev.build_sr(ev_slots, with_S=False)
        ev.close()
        return {"energy_per_site": float(E[0]) / ns, "sigma_per_site": float(Ee[0]) / ns,
                "samples": ev_slots * inst.n_walkers}

    out = {"workload": "sq4_u4_proj4: 4x4 Hubbard U=4 half filling, 2x2-sublattice f, "
                       "N_p=%d, %d walkers, FP64" % (proj.n_params, proj.n_walkers),
           "n_proj": len(proj.proj_w)}
    p0 = uhf_start(plain)
    out["uhf_start"] = {"plain": evaluate(plain, p0), "projected": evaluate(proj, p0)}
    p1, out["pretrain_plain"] = train(plain, p0, "plain (first)", 0)
    p_pl, out["plain"] = train(plain, p1, "plain", 1)
    out["plain"].update(evaluate(plain, p_pl))
    p_pr, out["projected"] = train(proj, p1, "projected", 1)
    out["projected"].update(evaluate(proj, p_pr))
    d = out["plain"]["energy_per_site"] - out["projected"]["energy_per_site"]
    out["gain_per_site"] = d
    out["gain_over_sigma"] = d / float(np.hypot(out["plain"]["sigma_per_site"],
                                                out["projected"]["sigma_per_site"]))
    out["context_table3"] = {"ED": -0.85136, "mVMC_2x2_momentum_and_spin_projection": -0.84985,
                             "mVMC_2x2_sigma": 0.00003}
    out["relative_error_vs_ED"] = abs(out["projected"]["energy_per_site"] + 0.85136) / 0.85136
    return out


def rbm_leg(steps):
    """16x16 Hubbard, U = 8, N_e = 224 (1/8 hole doping), 2x2-sublattice f
    times an RBM factor of 512 hidden units over the 512 spin-resolved
    occupations (N_p = 264194), 8192 walkers, single-precision sweeps with a
    double refresh once per sweep (224 proposals), 10 sweeps and one sample
    per walker per SR step, SR by CG over the centred O (8192 x 264320 single
    precision, no explicit S) run to the Algorithm 1 stopping rule."""
    from mvmc_inputs import workload
    wl = workload("sq16_u8_rbm", warmup=10)
    r = run_sr_workload(wl, "mixed", steps, 1, wl["refresh_every"], solver="cg",
                        build_s=False, cg_tol=wl["cg_tol"], cg_maxit=wl["cg_maxit"])
    out = step_summary(r, 4, True)
    out.pop("s_build")
    o_bytes = r["N"] * (-(-r["np"] // 128) * 128) * 4
    it = r["cg_iterations"][-1] if r["cg_iterations"] else 0
    out.update({"walkers": r["W"], "n_elec": r["ne"], "n_params": r["np"],
                "refresh_every": wl["refresh_every"], "cg_tol": wl["cg_tol"],
                "cg_iterations": r["cg_iterations"], "cg_maxit": wl["cg_maxit"],
                "cg_ms_per_iteration": km(r)["sr_solve"] / max(it, 1),
                "cg_gbs_per_iteration":
                    2 * o_bytes / (km(r)["sr_solve"] / max(it, 1) * 1e-3) / 1e9})
    return out


def batch_leg(steps):
    """32 ragged clusters (square L = 4..12, U in [2, 10], filling 0.8-1.0,
    256 walkers each), mixed precision, each instance its own SR step.  Both
    schedules: the persistent queue launch (one sweep launch per call,
    walkers longest first, refreshes inside the launch) and the per-bucket
    launches with autotuned variants; the faster one is the leg's value."""
    from mvmc_inputs import workload
    wl = workload("batch32_ragged")
    insts = wl["instances"]
    out = {"instances": len(insts), "walkers": sum(i.n_walkers for i in insts),
           "n_elec_range": [min(i.n_elec for i in insts), max(i.n_elec for i in insts)]}
    for sched in ("queue", "buckets"):
        log(f"[bench] batch32_ragged {sched}")
        r = run_sr_workload(wl, "mixed", steps, 1, wl["refresh_every"], use_graph=True,
                            autotune=sched == "buckets", schedule=sched, refresh_unit=MIXED_UNIT)
        leg = {"value": r["rate"], "unit": "hop-updates/s", "ms_per_step": r["ms_per_step"],
               "sweeps_per_step": r["sweeps"], "accept_ratio": r["accept_ratio"],
               "kernel_ms_per_step": km(r),
               "energy_per_site_last_step": [e / i.n_sites
                                             for e, i in zip(r["energies"][-1], insts)]}
        if sched == "buckets":
            leg["autotune"] = r["autotune"]
        out[sched] = leg
    best = min(("queue", "buckets"), key=lambda k: out[k]["ms_per_step"])
    out.update({k: v for k, v in out[best].items() if k != "autotune"})
    out["schedule"] = best
    return out


def rbm_gain(sr_steps):
    """16x16, U = 8, N_e = 224, 8192 walkers, 10 sweeps and one sample per
    walker per SR step.  The plain Pfaffian-Jastrow(-Gutzwiller) state is
    first trained by SR for sr_steps steps; from that state two runs of
    sr_steps more steps follow on the same GPU with the same sampler seed:
    the plain state alone, and the same state times an RBM factor whose
    parameters start small (a tenth of the workload's RBM draw, so the
    product starts at the trained state's energy).  Each final state's
    energy is then estimated with the same number of samples (16 per walker,
    5 sweeps apart)."""
    import numpy as np

    from mvmc_inputs import workload
    from paper_1711_11418_amd import MVMC

    def train(inst, params, wl, tag, steps):
        ctx = MVMC([inst], params, precision="mixed", refresh_every=wl["refresh_every"],
                   seed=wl["sampler_seed"], n_slots=1, solver="cg", build_s=False)
        ctx.sample(wl["warmup"])
        hist, iters = [], []
        t0 = time.perf_counter()
        for it in range(steps):
            ctx.sample_async(wl["sweeps"])
            ctx.measure(0)
            E, Er, _ = ctx.build_sr(1, with_S=False)
            hist.append((float(E[0]) / inst.n_sites, float(Er[0]) / inst.n_sites))
            iters.append(int(ctx.sr_update(dtau=wl["dtau"], eps_rel=wl["eps_rel"],
                                           eps_abs=wl["eps_abs"], solver="cg",
                                           cg_tol=wl["cg_tol"], cg_maxit=wl["cg_maxit"])[0]))
            if it % 10 == 0:
                log(f"[rbm-gain] {tag} step {it}: E/N = {hist[-1][0]:.5f} +- {hist[-1][1]:.5f}, "
                    f"CG {iters[-1]}")
        train_s = time.perf_counter() - t0
        p = ctx.params.cpu().numpy().copy()
        ctx.close()
        return p, {"n_params": inst.n_params, "sr_steps": steps, "train_seconds": train_s,
                   "history_per_site": hist, "cg_iterations": iters}

    def evaluate(inst, params, wl):
        slots = 16
        ev = MVMC([inst], params, precision="mixed", refresh_every=wl["refresh_every"],
                  seed=wl["sampler_seed"] + 7, n_slots=slots, solver="cg", build_s=False)
        ev.sample(wl["warmup"])
        for s in range(slots):
            ev.sample_async(5)
            ev.measure(s)
        E, Er, _ = ev.build_sr(slots, with_S=False)
        ev.close()
        return {"energy_per_site": float(E[0]) / inst.n_sites,
                "sigma_per_site": float(Er[0]) / inst.n_sites, "samples": slots * inst.n_walkers}

    wl_pj, wl_rbm = workload("sq16_u8_pj"), workload("sq16_u8_rbm")
    pj, rbm = wl_pj["instances"][0], wl_rbm["instances"][0]
    p1, pre = train(pj, pj.params0, wl_pj, "pj (first)", sr_steps)
    out = {"pretrain": pre, "pretrained": evaluate(pj, p1, wl_pj)}
    p_pj, out["pj"] = train(pj, p1, wl_pj, "pj", sr_steps)
    out["pj"].update(evaluate(pj, p_pj, wl_pj))
    p0_rbm = np.concatenate([p1, 0.1 * rbm.params0[pj.n_params:]])
    p_rbm, out["pj_rbm"] = train(rbm, p0_rbm, wl_rbm, "pj_rbm", sr_steps)
    out["pj_rbm"].update(evaluate(rbm, p_rbm, wl_rbm))
    d = out["pj_rbm"]["energy_per_site"] - out["pj"]["energy_per_site"]
    out["gain_per_site"] = -d
    out["gain_over_sigma"] = -d / float(np.hypot(out["pj_rbm"]["sigma_per_site"],
                                                 out["pj"]["sigma_per_site"]))
    return out


def hbm_copy_probe(gib=1.0, reps=10):
    """Attainable HBM bandwidth: torch's elementwise negation over a buffer of
    `gib` GiB (read once, written once).  Under rocprofv3 --pmc its
    FETCH_SIZE and WRITE_SIZE calibrate the counters against known bytes."""
    import torch
    n = int(gib * (1 << 30)) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"kernel": "torch.neg (elementwise)", "bytes_per_launch": 2 * n * 8, "ms": ms,
            "gbs": 2 * n * 8 / (ms * 1e-3) / 1e9}


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_11418_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, scaled by the calibration copy; None when the summary is missing
    or the kernel's sources changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None, "no counter summary"
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("sources_sha256_16") != sources_digest():
        return None, "kernel sources changed since the counters were taken"
    copy_bytes = float(kv["copy_bytes_per_launch"])
    f_scale = copy_bytes / 2 / (float(kv["copy_fetch_kib"]) * 1024)
    w_scale = copy_bytes / 2 / (float(kv["copy_write_kib"]) * 1024)
    t = (float(kv["kernel_fetch_kib"]) * 1024 * f_scale
         + float(kv["kernel_write_kib"]) * 1024 * w_scale)
    return t, (f"FETCH_SIZE+WRITE_SIZE per launch (mean over one step's launches), scaled by the copy "
               f"({f_scale:.3f}, {w_scale:.3f})")


def headline_roofline(r, wsize):
    """Roofline of the dominant kernel of the headline step, the
    anti-parallel-block sweep: its algorithmic bytes per launch (n w per
    proposal, 3 n^2 w per accepted one) over its average launch time (HIP
    events on the library's stream), against the HBM peak."""
    launches = max(r["kernel_calls"][0], 1)
    avg_ms = km(r)["sweep"] / launches
    b = sweep_bytes(r, wsize, sweep_model_of(r["variants"][0])) / launches
    bm = sweep_bytes(r, wsize, "method") / launches
    gbs = b / (avg_ms * 1e-3) / 1e9
    traffic, note = measured_traffic()
    # the timed steps run without a trace or exchange updates, so walkers
    # without an RBM factor take the variant with that code left out
    full = "false" if r.get("n_hidden", 0) == 0 else "true"
    return {"kernel": f"k_sweep_ap<double, {r['variants'][0][2:]}, {full}>", "bound": "hbm",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": traffic, "traffic_note": note,
            "avg_launch_ms": avg_ms, "launches_per_step": launches,
            "alg_bytes_per_launch": b, "byte_model": "n w per proposal + 3 n^2 w per accepted "
                                                     "proposal (n = N_e/2, w = 8)",
            "method_model_bytes_per_launch": bm,
            "method_model_frac": bm / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def _oracle_worker(args):
    os.environ["OMP_NUM_THREADS"] = "1"
    from mvmc_inputs import random_configs, workload
    from oracle import sampler
    from oracle import wavefunction as wf
    wid, name, n_prop, budget = args
    inst = workload(name, n_walkers=4)["instances"][0]
    m = wf.expand(inst, inst.params0)
    A = wf.skew_table(m)
    done = 0
    t0 = time.perf_counter()
    for pos in random_configs(inst, 64, 100 + wid):
        if wf.log_psi(m, pos, A)[0] == 0.0:
            continue
        wk = sampler.make_walker(m, pos, gid=wid)
        for _ in range(n_prop):
            sampler.step(m, wk, 1711, A)
            done += 1
            if time.perf_counter() - t0 > budget:
                return done, time.perf_counter() - t0
    return done, time.perf_counter() - t0


def cpu_baseline(budget_s=15.0):
    """The oracle (full-recompute Metropolis, two Parlett-Reid Pfaffians per
    proposal) on the host cores, one process per core, on a time-bounded
    sample of the headline 10x10 workload; numpy O^T O at 4096 x 2000 and
    numpy's Cholesky at 10^4 in double as context."""
    import multiprocessing as mp

    import numpy as np
    cores = min(os.cpu_count() or 1, 16)
    pool = mp.get_context("spawn").Pool(cores)
    try:
        res = pool.map(_oracle_worker, [(w, HEADLINE, 10 ** 9, budget_s) for w in range(cores)])
    finally:
        pool.close()
        pool.join()
    props, wall = sum(x[0] for x in res), max(x[1] for x in res)
    rng = np.random.default_rng(0)
    O = rng.standard_normal((4096, 2000))
    t0 = time.perf_counter()
    O.T @ O / 4096
    ts = time.perf_counter() - t0
    B = rng.standard_normal((10000, 10000))
    B = (B + B.T) * 0.5 + 10000.0 * np.eye(10000)   # symmetric, diagonally dominant: SPD
    t0 = time.perf_counter()
    np.linalg.cholesky(B)
    tc = time.perf_counter() - t0
    try:
        blas = np.show_config(mode="dicts")["Build Dependencies"]["blas"]["name"]
    except Exception:   # the configuration report differs between numpy versions
        blas = "unknown"
    return {"value": props / wall, "unit": "hop-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{props} full-recompute proposals on the 10x10 U=8 workload "
                      f"(N_e = 100), {cores} processes x {budget_s:.0f} s",
            "s_build_gflops_numpy_fp64": 4096 * 2000 * 2001 / ts / 1e9,
            "cholesky_1e4_numpy_fp64_s": tc, "nproc": os.cpu_count(), "blas": blas}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--skip-legs", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch the sampling eagerly")
    ap.add_argument("--s-build-only", action="store_true",
                    help="print only the split-bf16 S build leg (for kernel profiling)")
    ap.add_argument("--lanczos-only", action="store_true",
                    help="print only the first-step power-Lanczos leg")
    ap.add_argument("--batch-only", action="store_true",
                    help="print only the ragged-batch leg (queue and bucket schedules)")
    ap.add_argument("--projection-only", action="store_true",
                    help="train the 4x4 U=4 state with and without the momentum projection")
    ap.add_argument("--rbm-gain", action="store_true",
                    help="train 16x16 PJ and PJ x RBM by SR and print their energies")
    ap.add_argument("--sr-steps", type=int, default=40)
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the walkers of this workload fit one MI355X; "
              "multi-GPU sharding is described in DESIGN.md and not run.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    from mvmc_inputs import workload

    if a.s_build_only:
        print(json.dumps({"s_build_bf16x3_sq10": s_build_leg()}), flush=True)
        return
    if a.rbm_gain:
        print(json.dumps({"rbm_gain_sq16": rbm_gain(a.sr_steps)}), flush=True)
        return
    if a.lanczos_only:
        print(json.dumps({"lanczos_sq8": lanczos_leg()}), flush=True)
        return
    if a.projection_only:
        print(json.dumps({"projection_sq4": projection_leg()}), flush=True)
        return
    if a.batch_only:
        print(json.dumps({"batch32_ragged": batch_leg(max(1, a.steps - 1))}), flush=True)
        return

    copy = hbm_copy_probe()
    log(f"[bench] HBM copy probe: {copy['gbs']:.0f} GB/s")
    from paper_1711_11418_amd.binding import peak_probe
    probes = {k: peak_probe(k) for k in ("bf16_mfma", "fp64_mfma", "fp64_fma")}
    log(f"[bench] instruction peaks (TFLOP/s): {probes}")
    wl = workload(HEADLINE)
    log(f"[bench] {HEADLINE} fp64: W=4096 sweeps/step={wl['sweeps']} steps={a.steps} "
        f"warmup={a.warmup}")
    r = run_sr_workload(wl, "fp64", a.steps, a.warmup, FP64_REFRESH, use_graph=not a.no_graph)
    head = step_summary(r, 8, False)
    log(f"[bench]   fp64: {r['rate']:.3e} hop-updates/s, {r['ms_per_step']:.1f} ms/step, "
        f"kernel ms {', '.join(f'{k} {v:.2f}' for k, v in km(r).items())}")
    out = {
        "metric": METRIC, "value": r["rate"], "unit": "hop-updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sq10_u8: 10x10 Hubbard U=8, N_e=100, unconstrained f "
                               "(N_p=10002), 4096 walkers x 10 sweeps + E_loc/O_k + S (FP64 "
                               "MFMA) + Cholesky + update + double refresh per SR step",
                   "walkers": r["W"], "n_elec": r["ne"], "n_params": r["np"],
                   "sweeps_per_step": r["sweeps"], "samples_per_step": r["N"],
                   "refresh_every": FP64_REFRESH, "sampling_in_hip_graph": r["graph"]},
        "accepted_per_s": r["rate"] * r["accept_ratio"],
        "s_build_tflops": head["s_build"]["tflops"],
        "roofline": headline_roofline(r, 8),
        "fp64": head,
        "measured_peaks": {"hbm_copy_gbs": copy["gbs"], "hbm_copy": copy,
                           "bf16_mfma_tflops": probes["bf16_mfma"],
                           "fp64_mfma_tflops": probes["fp64_mfma"],
                           "fp64_fma_tflops": probes["fp64_fma"],
                           "note": "register-only loops on non-zero data, two wavefronts per "
                                   "SIMD (mvmc_peak_probe); datasheet peaks in roofline.peak"},
    }
    log(f"[bench] {HEADLINE} mixed (refresh every {MIXED_REFRESH} {MIXED_UNIT})")
    mx = run_sr_workload(wl, "mixed", a.steps, a.warmup, MIXED_REFRESH,
                         use_graph=not a.no_graph, refresh_unit=MIXED_UNIT)
    out["mixed"] = step_summary(mx, 4, True)
    out["mixed"]["refresh_every"] = {"n": MIXED_REFRESH, "unit": MIXED_UNIT}
    out["mixed"]["speedup_vs_fp64"] = mx["rate"] / r["rate"]
    out["mixed"]["s_build_speedup_vs_fp64"] = (head["s_build"]["ms"] /
                                               out["mixed"]["s_build"]["ms"])
    out["s_build_bf16x3_tflops"] = out["mixed"]["s_build"]["tflops"]
    log(f"[bench]   mixed: {mx['rate']:.3e} hop-updates/s, {mx['ms_per_step']:.1f} ms/step, "
        f"kernel ms {', '.join(f'{k} {v:.2f}' for k, v in km(mx).items())}")
    if not a.skip_legs:
        log("[bench] precision errors: mixed vs double result by result")
        out["precision_errors"] = precision_errors()
        log(f"[bench]   {json.dumps(out['precision_errors'])}")
        log("[bench] split-bf16 S build at 4096 x 10^4, tuned tile")
        out["s_build_bf16x3_sq10"] = s_build_leg()
        out["s_build_bf16x3_sq10"]["issued_frac_of_measured_bf16_mfma"] = (
            out["s_build_bf16x3_sq10"]["issued_mfma_tflops"] / probes["bf16_mfma"])
        log("[bench] 8x8 leg (double and mixed)")
        out["sq8_u4"] = sq8_leg(max(1, a.steps))
        log(f"[bench]   8x8 fp64 {out['sq8_u4']['fp64']['value']:.3e}, mixed "
            f"{out['sq8_u4']['mixed']['value']:.3e} hop-updates/s")
        log("[bench] first-step power-Lanczos on 8x8 (trained state)")
        out["lanczos_sq8"] = lanczos_leg()
        log(f"[bench]   E/N {out['lanczos_sq8']['E_per_site']:.5f}, E_1/N "
            f"{out['lanczos_sq8']['E1_per_site']:.5f}, alpha_1 {out['lanczos_sq8']['alpha_1']:.4f}")
        log("[bench] 4x4 U=4 with and without the momentum projection (trained by SR)")
        out["projection_sq4"] = projection_leg()
        log(f"[bench]   projected {out['projection_sq4']['projected']['energy_per_site']:.5f}, "
            f"plain {out['projection_sq4']['plain']['energy_per_site']:.5f} per site, gain "
            f"{out['projection_sq4']['gain_over_sigma']:.1f} sigma")
        log("[bench] 16x16 RBM leg (8192 walkers, CG)")
        out["sq16_u8_rbm"] = rbm_leg(1)
        log(f"[bench]   16x16 {out['sq16_u8_rbm']['value']:.3e} hop-updates/s, "
            f"{out['sq16_u8_rbm']['ms_per_step']:.0f} ms/step, CG "
            f"{out['sq16_u8_rbm']['cg_iterations']}")
        log("[bench] ragged batch of 32 clusters (mixed; queue, then autotuned buckets)")
        out["batch32_ragged"] = batch_leg(max(1, a.steps - 1))
    if not a.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
