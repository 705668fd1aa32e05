"""Benchmark of the many-variable VMC hot path on one MI355X.

A step is one SR iteration of the 8x8 periodic Hubbard model (U = 4,
N_e = 64, 2x2-sublattice pair amplitudes + distance Jastrow + Gutzwiller,
N_p = 271): 1024 walkers x 200 sweeps (64 proposals each) with the local
energy and O_k measured after every sweep, then the SR statistics, the S
build, the Cholesky solve, the parameter update and the full refresh of
every walker.  Inputs are seeded and synthetic and resident in HBM before
timing starts.

Printed: one JSON line with the walker hop-update rate (proposals/s) over
whole steps, the S-build rate, the roofline of the sweep kernel, the
mixed-precision run of the same workload, the split-bf16 S build at the
4096 x 10^4 shape, and the CPU oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--no-cpu] [--skip-legs]
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
TRAFFIC_SUMMARY = "sweep_reg_fp64_c2_sq8_traffic.txt"
TRAFFIC_SOURCES = ("k_sweep_reg.hip", "common.h", "ap_block.h", "wave.h")   # the sweep kernel and its headers
METRIC = "walker hop-updates/s + SR S-build TFLOP/s, batched/mixed vs plain FP64"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_sr_workload(wl, precision, steps, warmup, refresh_every, solver="chol", sweep_threads=0,
                    use_graph=True, autotune=False, build_s=True, cg_tol=1e-10, cg_maxit=1000):
    """Time whole SR steps of every instance of the workload.  With use_graph
    the sampling part of a step (the sweeps and the measurement after each
    of them) is captured once into a HIP graph and replayed; the SR build and
    update run eagerly.  With autotune the sweep variant of every instance is
    chosen by timing after the warm-up."""
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
                   sweep_threads=sweep_threads, stream=side)
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

        escalations = []

        cg_iters = []

        def sr():
            E, Er, V = ctx.build_sr(slots, with_S=build_s)
            it = ctx.sr_update(dtau=wl["dtau"], eps_rel=wl["eps_rel"], eps_abs=wl["eps_abs"],
                               solver=solver, cg_tol=cg_tol, cg_maxit=cg_maxit)
            if solver == "chol":
                escalations.append(int(np.max(it)))
            else:
                cg_iters.append(int(np.max(it)))
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
        torch.cuda.synchronize()
        ctx.close()
    per_sweep = sum(i.n_walkers * i.n_elec for i in insts)
    proposals = steps * sweeps * per_sweep
    i0 = insts[0]
    return {
        "seconds": dt, "proposals": proposals, "rate": proposals / dt,
        "ms_per_step": 1e3 * dt / steps,
        "energies": [e[0] for e in energies] if len(insts) == 1 else energies,
        "accept_ratio": accepted / (sweeps * per_sweep), "kernel_ms": ms.tolist(),
        "kernel_calls": calls.tolist(), "W": i0.n_walkers, "ne": i0.n_elec, "np": i0.n_params,
        "sweeps": sweeps, "N": slots * i0.n_walkers, "graph": graph is not None,
        "autotune": tuned, "cholesky_shift_raises": escalations, "cg_iterations": cg_iters,
        "steps": steps,
    }


def measure_hbm_model(r, wsize):
    """E_loc and O_k: every sample reads Y once (N_e^2 w) and writes its O row
    (N_p w); modelled rate over the measurement time of one SR step."""
    ne, npar = r["ne"], r["np"]
    bytes_ = r["N"] * (ne * ne + npar) * wsize
    ms = r["kernel_ms"][2]
    gbs = bytes_ / (ms * 1e-3) / 1e9
    return {"alg_bytes_per_step": bytes_, "ms_per_step": ms, "achieved_gbs": gbs,
            "peak_gbs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS}


def sweep_hbm_model(r, wsize, sweep_ms, kernel_model=True):
    """Modelled HBM rate of the sweeps of one SR step.  The method's byte
    model: every proposal reads one row of Y (N_e w bytes), every accept
    reads and writes all of Y (2 N_e^2 w bytes).  The LDS/HBM kernel moves
    less: with the anti-parallel pair amplitude the same-spin blocks of Y
    are zero, so a proposal reads half a row and an accept reads one
    N_e/2 x N_e/2 block for q and reads and writes the two opposite-spin
    blocks (1.25 N_e^2 w bytes); that count is reported beside it."""
    ne = r["ne"]
    props = r["proposals"] / max(r["steps"], 1)
    acc = props * r["accept_ratio"]
    bytes_ = props * ne * wsize + acc * 2 * ne * ne * wsize
    gbs = bytes_ / (sweep_ms * 1e-3) / 1e9
    out = {"alg_bytes_per_step": bytes_, "sweep_ms_per_step": sweep_ms, "achieved_gbs": gbs,
           "peak_gbs": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS}
    if kernel_model:
        kb = props * ne // 2 * wsize + acc * 1.25 * ne * ne * wsize
        kg = kb / (sweep_ms * 1e-3) / 1e9
        out.update({"kernel_bytes_per_step": kb, "kernel_gbs": kg,
                    "kernel_frac": kg / HBM_PEAK_GBS})
    return out


def precision_leg(steps):
    """10x10 Hubbard, U = 8, N_e = 100, unconstrained f (N_p = 10002), 4096
    walkers, 10 sweeps and one sample per walker per SR step, S and a
    Cholesky solve: the mixed path (single-precision sweeps, double
    refresh every 32 proposals, split-bf16 S) against the plain double path
    (refresh every 4 sweeps, double S), same kernels otherwise."""
    from mvmc_inputs import workload
    out = {}
    for prec, R in (("mixed", 32), ("fp64", 400)):
        wl = workload("c3_sq10_mixed", warmup=20)
        log(f"[bench]   10x10 {prec} (refresh every {R})")
        r = run_sr_workload(wl, prec, steps, 1, R, solver="chol")
        i0 = wl["instances"][0]
        km = dict(zip(["sweep", "refresh", "measure", "sr_stats", "s_build", "sr_solve"],
                      r["kernel_ms"]))
        N, npar = r["N"], r["np"]
        nh = r["ne"] // 2
        ref_calls = max(r["kernel_calls"][1], 1)
        # block-route refresh: Gauss-Jordan inversion of the N_e/2 x N_e/2 block, 2 n^3 flops
        ref_flops = ref_calls * r["W"] * 2.0 * nh ** 3
        out[prec] = {"value": r["rate"], "unit": "hop-updates/s", "ms_per_step": r["ms_per_step"],
                     "accept_ratio": r["accept_ratio"], "kernel_ms_per_step": km,
                     "s_build_tflops": N * npar * (npar + 1) / (km["s_build"] * 1e-3) / 1e12,
                     "sweep_modelled_hbm": sweep_hbm_model(r, 4 if prec == "mixed" else 8,
                                                           km["sweep"]),
                     "refresh": {"launches_per_step": r["kernel_calls"][1],
                                 "fp64_tflops": ref_flops / (km["refresh"] * 1e-3) / 1e12,
                                 "peak_tflops": FP64_PEAK_TFLOPS,
                                 "flops_model": "2 (N_e/2)^3 per walker (block route)"},
                     "cholesky": {"fp64_tflops": npar ** 3 / 3 / (km["sr_solve"] * 1e-3) / 1e12,
                                  "peak_tflops": FP64_PEAK_TFLOPS,
                                  "note": "N_p^3/3 flops over the whole solve (factor, "
                                          "substitutions, update)"},
                     "cholesky_shift_raises": r["cholesky_shift_raises"],
                     "energy_per_site": [e / i0.n_sites for e in r["energies"]]}
    out["speedup_mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
    out["s_build_speedup_mixed_vs_fp64"] = (out["fp64"]["kernel_ms_per_step"]["s_build"] /
                                            out["mixed"]["kernel_ms_per_step"]["s_build"])
    return out


def rbm_leg(steps):
    """16x16 Hubbard, U = 8, N_e = 224 (1/8 hole doping), 2x2-sublattice f
    times an RBM factor of 512 hidden units over the 512 spin-resolved
    occupations (N_p = 264194), 8192 walkers, single-precision sweeps, 10
    sweeps and one sample per walker per SR step, SR by CG over the centred
    O (8192 x 264320 single precision, no explicit S); CG is capped at 50
    iterations per step here."""
    from mvmc_inputs import workload
    wl = workload("c5_sq16_rbm_mixed", warmup=10)
    r = run_sr_workload(wl, "mixed", steps, 1, 0, solver="cg", build_s=False, cg_tol=1e-6,
                        cg_maxit=50)
    i0 = wl["instances"][0]
    km = dict(zip(["sweep", "refresh", "measure", "sr_stats", "s_build", "sr_solve"],
                  r["kernel_ms"]))
    o_bytes = r["N"] * (-(-r["np"] // 128) * 128) * 4
    it = r["cg_iterations"][-1] if r["cg_iterations"] else 0
    return {"value": r["rate"], "unit": "hop-updates/s", "ms_per_step": r["ms_per_step"],
            "walkers": r["W"], "n_elec": r["ne"], "n_params": r["np"], "n_hidden": i0.n_hidden,
            "accept_ratio": r["accept_ratio"], "kernel_ms_per_step": km,
            "cg_iterations": r["cg_iterations"], "cg_cap": 50,
            "cg_ms_per_iteration": km["sr_solve"] / max(it, 1),
            "cg_gbs_per_iteration": 2 * o_bytes / (km["sr_solve"] / max(it, 1) * 1e-3) / 1e9,
            "sweep_modelled_hbm": sweep_hbm_model(r, 4, km["sweep"]),
            "energy_per_site": [e / i0.n_sites for e in r["energies"]]}


def batch_leg(steps):
    """32 ragged clusters (square L = 4..12, U in [2, 10], filling 0.8-1.0,
    256 walkers each), mixed precision, each instance its own SR step; all
    instances of a register tier sweep in one launch, variants autotuned."""
    from mvmc_inputs import workload
    wl = workload("c4_batch32_mixed")
    r = run_sr_workload(wl, "mixed", steps, 1, wl["refresh_every"], use_graph=True,
                        autotune=True)
    insts = wl["instances"]
    return {"value": r["rate"], "unit": "hop-updates/s", "ms_per_step": r["ms_per_step"],
            "instances": len(insts), "walkers": sum(i.n_walkers for i in insts),
            "n_elec_range": [min(i.n_elec for i in insts), max(i.n_elec for i in insts)],
            "sweeps_per_step": r["sweeps"], "accept_ratio": r["accept_ratio"],
            "kernel_ms_per_step": dict(zip(["sweep", "refresh", "measure", "sr_stats",
                                            "s_build", "sr_solve"], r["kernel_ms"])),
            "autotune": r["autotune"], "energy_per_site_last_step":
                [e / i.n_sites for e, i in zip(r["energies"][-1], insts)]}


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


def sweep_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_11418_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per sweep launch from the committed counter summary, scaled by
    the calibration copy; None when the summary is missing or the sweep
    kernel's sources changed after the counters were taken."""
    path = os.path.join(ROOT, "profiles", TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None, "no counter summary"
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("sources_sha256_16") != sweep_sources_digest():
        return None, "sweep sources changed since the counters were taken"
    copy_bytes = float(kv["copy_bytes_per_launch"])
    f_scale = copy_bytes / 2 / (float(kv["copy_fetch_kib"]) * 1024)
    w_scale = copy_bytes / 2 / (float(kv["copy_write_kib"]) * 1024)
    t = (float(kv["sweep_fetch_kib"]) * 1024 * f_scale
         + float(kv["sweep_write_kib"]) * 1024 * w_scale)
    return t, f"FETCH_SIZE+WRITE_SIZE per launch (median), scaled by the copy ({f_scale:.3f}, {w_scale:.3f})"


def sweep_roofline(r, wsize):
    """Algorithmic bytes of the sweep per launch over its measured duration."""
    W, ne = r["W"], r["ne"]
    avg_ms = r["kernel_ms"][0] / max(r["kernel_calls"][0], 1)
    props = W * ne                          # one sweep per launch in this workload
    acc = r["accept_ratio"] * props
    bytes_ = props * ne * wsize + acc * 2 * ne * ne * wsize
    flops = props * 2 * ne + acc * 6 * ne * ne
    return avg_ms, bytes_, flops


def sweep_roofline_entry(sweep_threads, avg_ms, bytes_, flops, traffic, traffic_note,
                         probes=None, copy_gbs=None):
    """Roofline of the sweep kernel.  The byte model charges every proposal
    one row of Y and every accept a read and a write of all of Y.  The
    register-resident kernel keeps Y on chip for the whole launch (the
    counters see it read and written once), so its modelled-byte rate is not
    bounded by HBM and the kernel is reported against the double-precision
    vector peak with its algorithmic flops; the LDS kernel streams Y through
    LDS and is reported against HBM."""
    gbs = bytes_ / (avg_ms * 1e-3) / 1e9
    tflops = flops / (avg_ms * 1e-3) / 1e12
    common = {"avg_launch_ms": avg_ms, "alg_bytes_per_launch": bytes_,
              "alg_flops_per_launch": flops, "traffic": traffic, "traffic_note": traffic_note,
              "traffic_frac_of_alg": None if traffic is None else traffic / bytes_}
    if sweep_threads == 0:
        return {"kernel": "k_sweep_reg<double, 64, 4, false, false>", "bound": "alu",
                "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / FP64_PEAK_TFLOPS,
                "frac_of_measured_fp64_fma": (tflops / probes["fp64_fma"]) if probes else None,
                "modelled_hbm": {"achieved_gbs": gbs, "peak_gbs": HBM_PEAK_GBS,
                                 "frac": gbs / HBM_PEAK_GBS},
                "residency": "Y in registers for the whole launch", **common}
    return {"kernel": f"k_sweep<double, true, {sweep_threads}>", "bound": "hbm",
            "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "fp64_tflops": tflops, **common}


def s_build_leg():
    """Split-bf16 S build at the 4096-sample x 10^4-parameter shape, at the
    tile side the library's tuner picks on this data."""
    import numpy as np
    import torch

    from mvmc_inputs import workload
    from paper_1711_11418_amd import MVMC

    wl = workload("c3_sq10_mixed")
    inst = wl["instances"][0]
    ctx = MVMC([inst], inst.params0, precision="mixed", refresh_every=32,
               seed=wl["sampler_seed"], n_slots=1, solver="cg", build_s=True)
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
    # upper-triangle tiles of the chosen side (64 for narrow parameter
    # sets), three bf16 MFMA passes each over the samples rounded up to 32
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


def _oracle_worker(args):
    import numpy as np
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


def cpu_baseline(budget_s=12.0):
    """The oracle (full-recompute Metropolis, Parlett-Reid per proposal) on
    the host cores, one process per core, on time-bounded samples of the 8x8
    workload (the headline), the 8-site ring and the 10x10 workload; plus
    numpy O^T O at 4096 x 2000 and numpy's Cholesky at 10^4, in double."""
    import multiprocessing as mp

    import numpy as np
    cores = min(os.cpu_count() or 1, 16)

    def rate(name, budget):
        with mp.get_context("spawn").Pool(cores) as pool:
            res = pool.map(_oracle_worker, [(w, name, 10 ** 9, budget) for w in range(cores)])
        return sum(r[0] for r in res), max(r[1] for r in res)

    props, wall = rate("c2_sq8_fp64", budget_s)
    p1, w1 = rate("c1_ring8_fp64", 3.0)
    p3, w3 = rate("c3_sq10_mixed", 5.0)
    rng = np.random.default_rng(0)
    O = rng.standard_normal((4096, 2000))
    t0 = time.perf_counter()
    S = O.T @ O / 4096
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
            "sample": f"{props} full-recompute proposals on the 8x8 U=4 workload, "
                      f"{cores} processes x {budget_s:.0f} s",
            "ring8_hop_updates_per_s": p1 / w1, "sq10_hop_updates_per_s": p3 / w3,
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
    ap.add_argument("--sweep-threads", type=int, default=0,
                    help="0: register-resident sweep where it fits; 64/128/256: LDS sweep")
    ap.add_argument("--s-build-only", action="store_true",
                    help="print only the split-bf16 S build leg (for kernel profiling)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the walkers of this workload fit one MI355X; "
              "multi-GPU sharding is described in DESIGN.md and not run.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    from mvmc_inputs import workload

    if a.s_build_only:
        print(json.dumps({"s_build_bf16x3_c3": s_build_leg()}), flush=True)
        return

    copy = hbm_copy_probe()
    log(f"[bench] HBM copy probe: {copy['gbs']:.0f} GB/s")
    from paper_1711_11418_amd.binding import peak_probe
    probes = {k: peak_probe(k) for k in ("bf16_mfma", "fp64_mfma", "fp64_fma")}
    log(f"[bench] instruction peaks (TFLOP/s): {probes}")
    wl = workload("c2_sq8_fp64")
    log(f"[bench] c2_sq8_fp64 fp64: W=1024 sweeps/step={wl['sweeps']} steps={a.steps} "
        f"warmup={a.warmup}")
    r = run_sr_workload(wl, "fp64", a.steps, a.warmup, wl["refresh_every"],
                        sweep_threads=a.sweep_threads, use_graph=not a.no_graph)
    avg_ms, bytes_, flops = sweep_roofline(r, 8)
    s_ms = r["kernel_ms"][4] / max(r["kernel_calls"][4], 1)
    s_flops = r["N"] * r["np"] * (r["np"] + 1)
    traffic, traffic_note = measured_traffic() if a.sweep_threads == 0 else (None, "LDS sweep")
    out = {
        "metric": METRIC, "value": r["rate"], "unit": "hop-updates/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c2_sq8_fp64: 8x8 Hubbard U=4, Ne=64, Np=271, 1024 walkers x "
                               "200 sweeps + SR (Cholesky) per step",
                   "walkers": r["W"], "n_elec": r["ne"], "n_params": r["np"],
                   "sweeps_per_step": r["sweeps"], "samples_per_step": r["N"],
                   "sampling_in_hip_graph": r["graph"]},
        "accepted_per_s": r["rate"] * r["accept_ratio"],
        "accept_ratio": r["accept_ratio"],
        "s_build": {"tflops": s_flops / (s_ms * 1e-3) / 1e12, "ms": s_ms, "dtype": "f64",
                    "shape": [r["N"], r["np"]], "kernel": "FP64 MFMA 16x16x4",
                    "frac_of_fp64_peak": s_flops / (s_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                    "frac_of_measured_fp64_mfma": s_flops / (s_ms * 1e-3) / 1e12 /
                                                  probes["fp64_mfma"]},
        "roofline": sweep_roofline_entry(a.sweep_threads, avg_ms, bytes_, flops, traffic,
                                         traffic_note, probes, copy["gbs"]),
        "measured_peaks": {"hbm_copy_gbs": copy["gbs"], "hbm_copy": copy,
                           "bf16_mfma_tflops": probes["bf16_mfma"],
                           "fp64_mfma_tflops": probes["fp64_mfma"],
                           "fp64_fma_tflops": probes["fp64_fma"],
                           "note": "register-only loops on non-zero data, two wavefronts per "
                                   "SIMD (mvmc_peak_probe); datasheet peaks in roofline.peak"},
        "kernel_ms_per_step": dict(zip(["sweep", "refresh", "measure", "sr_stats", "s_build",
                                        "sr_solve"], r["kernel_ms"])),
        "measure_modelled_hbm": measure_hbm_model(r, 8),
        "energy_per_site": [e / 64 for e in r["energies"]],
    }
    if not a.skip_legs:
        log("[bench] mixed-precision leg (same workload, fp32 sweeps, refresh every 32)")
        m = run_sr_workload(wl, "mixed", max(1, a.steps - 1), 1, 32,
                            sweep_threads=a.sweep_threads, use_graph=not a.no_graph)
        out["mixed"] = {"value": m["rate"], "ms_per_step": m["ms_per_step"],
                        "speedup_vs_fp64": m["rate"] / r["rate"],
                        "energy_per_site": [e / 64 for e in m["energies"]],
                        "kernel_ms_per_step": m["kernel_ms"]}
        log("[bench] split-bf16 S build at 4096 x 10^4")
        out["s_build_bf16x3_c3"] = s_build_leg()
        out["s_build_bf16x3_c3"]["issued_frac_of_measured_bf16_mfma"] = (
            out["s_build_bf16x3_c3"]["issued_mfma_tflops"] / probes["bf16_mfma"])
        log("[bench] 10x10 precision leg: mixed vs plain FP64")
        out["sq10_mixed_vs_fp64"] = precision_leg(2)
        log("[bench] 16x16 RBM leg (8192 walkers, CG)")
        out["sq16_rbm_mixed"] = rbm_leg(1)
        log("[bench] ragged batch of 32 clusters (mixed, autotuned)")
        out["batch32_mixed"] = batch_leg(max(1, a.steps - 1))
    if not a.no_cpu:
        log("[bench] CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
