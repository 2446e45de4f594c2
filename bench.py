"""Benchmark of the MPDATA step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default: the 2-D periodic 2048x2048 FP64 step, n_iters=3 with the limiter
(stream-function advector of Courant sum 0.5, 64 non-negative blobs), and,
as sub-objects of the same JSON line, the batched solve (1024 ragged FP32
grids, one launch per step replayed from a HIP graph, against per-grid
launches) and the adjoint (gradient through K steps of the 1024^2 FP64
recipe, checkpoint every 20).  Inputs are resident in HBM before each timed
region; K steps are timed with HIP events on the stream the kernels run on,
bracketed by device syncs.  The line carries Mcell-steps/s, the roofline of
the dominant kernel (arithmetic and HBM, the binding one named) and the
FP64 CPU oracle timed on a bounded sample of the same workload, on one core
and on all host cores.

Other workloads (--workload): 2d-f32, 3d, 1d, batched, adjoint, osc (the
translating oscillator with source terms), sw (the 2-D shallow-water drop with
prognosed velocity), copy (counter calibration).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Arithmetic roofline, one counted operation (add, subtract, multiply,
# divide, min, max, compare) per lane per clock: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz = 39.32 T op/s, for FP64 and for the unpacked FP32 the
# kernels are built with.  (The published 78.6 / 157.3 TFLOP/s count a fused
# multiply-add as two and, for FP32, two packed lanes.)
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# the same chip's VALU issue: one wave64 instruction per SIMD every 4 clocks
SIMDS, XCDS, CLOCK_HZ = 1024, 8, 2.4e9
# algorithmic operations per cell-step of the dominant kernel (each add,
# subtract, multiply, divide, min, max and compare counts one): donor pass
# 15; per corrective pass 52 for the two pseudo-velocities, 66 for the
# limiter, 15 for the corrective donor pass (2-D, G = 1)
ALG_OPS = {"2d_periodic_2048x2048_fct_iters3": 15 + 2 * (52 + 66 + 15),
           "batched_1024x2d_periodic_64to768_fct_iters2": 15 + (52 + 66 + 15)}


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="2d",
                    choices=["2d", "2d-f32", "3d", "1d", "batched", "adjoint", "osc", "sw",
                             "copy"])
    ap.add_argument("--kernel", default="auto", choices=["auto", "staged", "fused"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle timing leg")
    ap.add_argument("--no-sub", action="store_true",
                    help="default workload only: leave out the batched and adjoint legs")
    ap.add_argument("--kahan", action="store_true",
                    help="Kahan-compensated donor-cell updates (the library-default summation)")
    ap.add_argument("--abs", action="store_true", help="|psi| in the psi-fractions")
    ap.add_argument("--dfl", action="store_true", help="divergent-flow pseudo-velocity term")
    ap.add_argument("--fct", action="store_true",
                    help="add the limiter (3-D and 1-D workloads; the 2-D ones have it)")
    ap.add_argument("--xcd-order", type=int, default=1,
                    help="batched tile order with --tile-rows: 1 grouped per XCD, 0 grid by grid")
    ap.add_argument("--tile-rows", type=int, default=None,
                    help="fused kernel rows per wavefront chunk (default: autotune)")
    return ap.parse_args()


def _profile_entry(fname, kernel_name, workload):
    """A per-launch record of a committed rocprofv3 counter summary
    (profiles/traffic.json: HBM bytes; profiles/valu.json: issue counters),
    used only while the kernel source still has the hash recorded with it."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        ent = data.get(f"{kernel_name}:{workload}")
        if not ent:
            return None
        from paper_1407_1309_amd.build import source_hash
        if ent.get("source_hash") != source_hash(kernel_name):
            return None
        return ent
    except Exception:
        return None


def _traffic_entry(kernel_name, workload):
    ent = _profile_entry("traffic.json", kernel_name, workload)
    return ent.get("bytes_per_launch") if ent else None


def _valu_entry(kernel_name, workload, cells, alg_ops):
    """VALU issue of the kernel from its committed counters: lane-instructions
    issued per cell-step (SQ_INSTS_VALU x 64 / cells) against the algorithmic
    operations, and the fraction of the SIMDs' issue capacity they fill over
    the kernel's mean duration in the same counter pass (4 clocks per wave64
    VALU instruction at the nominal clock; the GRBM clock count is not used,
    since the clock runs below nominal under some kernels)."""
    ent = _profile_entry("valu.json", kernel_name, workload)
    if not ent or "avg_us" not in ent:
        return None
    insts = float(ent["SQ_INSTS_VALU"])
    us = float(ent["avg_us"])
    return {"lane_instr_per_cell_step": round(insts * 64 / cells, 1),
            "alg_ops_per_cell_step": alg_ops,
            "issue_busy": round(insts * 4 / SIMDS / (us * 1e-6 * CLOCK_HZ), 4),
            "counters": {"SQ_INSTS_VALU": insts, "kernel_us_in_counter_pass": us}}


def _roofline(kernel, kernel_ms, launches, alg_bytes, alg_ops=None, traffic=None, valu=None):
    """Roofline of one kernel from its mean launch time: the HBM roofline
    (algorithmic bytes per launch) and, where the algorithmic operation
    count is known, the arithmetic one; `bound` names the one the kernel is
    closer to (the larger fraction), whose figures fill the top level."""
    sec = kernel_ms / 1e3
    gbs = alg_bytes / sec / 1e9
    hbm = {"achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": alg_bytes}
    out = {"bound": "hbm", "achieved": hbm["achieved"], "peak": hbm["peak"], "unit": "GB/s",
           "frac": hbm["frac"], "traffic": traffic, "kernel": kernel,
           "kernel_ms": round(kernel_ms, 6), "launches": launches, "hbm": hbm}
    if alg_ops is not None:
        tops = alg_ops / sec / 1e12
        alu = {"achieved": round(tops, 3), "peak": round(ALU_PEAK_TOPS, 2), "unit": "TFLOP/s",
               "frac": round(tops / ALU_PEAK_TOPS, 4), "alg_ops_per_launch": alg_ops,
               "convention": "add, subtract, multiply, divide, min, max, compare = 1 op; "
                             "peak = 1 op per lane per clock"}
        out["alu"] = alu
        if alu["frac"] > hbm["frac"]:
            out.update(bound="alu", achieved=alu["achieved"], peak=alu["peak"],
                       unit="TFLOP/s", frac=alu["frac"])
    out["valu"] = valu
    return out


def _oracle_rate(run, cells_steps):
    """Cell-steps per second of `run()` (one call), timed on the host."""
    t0 = time.perf_counter()
    res = run()
    return cells_steps / (time.perf_counter() - t0), res


def _host():
    """CPU model and logical CPU count of the host the oracle is timed on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu": model, "logical_cpus": os.cpu_count()}


def _time_steps(run, steps, torch):
    """Time `run(steps)` with HIP events on the current stream."""
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3      # seconds


def bench_single(args, torch, mpdata, synth, oracle):
    f32 = args.workload in ("2d-f32",)
    if args.workload in ("2d", "2d-f32"):
        case = synth.case_2d()
        name = "2d_periodic_2048x2048_fct_iters3"
    elif args.workload == "3d":
        case = synth.case_3d()
        name = "3d_open_384x384x256_tot_iga_iters2_gz"
    else:
        case = synth.case_1d()
        name = "1d_periodic_500_iters2"
    for flag, bit in (("kahan", mpdata.OPT_KAHAN), ("abs", mpdata.OPT_ABS), ("dfl", mpdata.OPT_DFL),
                      ("fct", mpdata.OPT_FCT)):
        if getattr(args, flag) and not case.opts & bit:
            case.opts |= bit
            name += "_" + flag
    dtype = torch.float32 if f32 else torch.float64
    es = 4 if f32 else 8
    K = args.steps if args.steps is not None else case.n_steps
    W = args.warmup
    kernel = {"auto": mpdata.KERNEL_AUTO, "staged": mpdata.KERNEL_STAGED,
              "fused": mpdata.KERNEL_FUSED}[args.kernel]
    dev = torch.device("cuda:0")
    plan = mpdata.Plan(case.psi.shape, dtype=dtype, n_iters=case.n_iters, opts=case.opts,
                       bc=case.bc, has_g=case.g is not None, device=dev, kernel=kernel)
    psi0 = torch.from_numpy(case.psi).to(dev, dtype)
    c = [torch.from_numpy(x).to(dev, dtype).contiguous() for x in case.c]
    g = torch.from_numpy(case.g).to(dev, dtype) if case.g is not None else None
    N = int(np.prod(case.psi.shape))

    if args.tile_rows is None:
        tile_rows = plan.autotune(psi0, c, g=g)      # outside the timed region
    else:
        tile_rows = args.tile_rows
        plan.set_tile_rows(tile_rows)
    psi = psi0.clone()
    plan.step(psi, c, g=g, n_steps=W)
    secs = _time_steps(lambda k: plan.step(psi, c, g=g, n_steps=k), K, torch)
    ms = secs * 1e3 / max(K, 1)
    value = N * K / secs / 1e6

    # mean launch time of the dominant kernel: HIP events on the plan's
    # stream before the first and after the last of K back-to-back launches
    psi_t = psi0.clone()
    plan.timing(K)
    plan.step(psi_t, c, g=g, n_steps=K)
    kern_ms, n_launch, kname = plan.timing_read()
    plan.timing(0)
    if kname == "k_resident1d":         # one launch runs all K steps
        kern_ms /= max(K, 1)

    # algorithmic bytes per launch of that kernel: read psi, every advector
    # component, G; write psi
    walls = 0
    for d in range(len(case.psi.shape)):
        sh = list(case.psi.shape)
        if case.bc == 1:
            sh[d] += 1                   # open: both edge walls are data
        walls += int(np.prod(sh))
    alg_bytes = es * (2 * N + walls + (N if case.g is not None else 0))
    fused = plan_uses_fused(plan, mpdata, kernel)
    wl = name + ("_f32" if f32 else "_f64")
    ops = ALG_OPS.get(name)
    roof = _roofline(kname, kern_ms, n_launch, alg_bytes,
                     alg_ops=ops * N if ops else None, traffic=_traffic_entry(kname, wl),
                     valu=_valu_entry(kname, wl, N, ops) if ops else None)
    if kname == "k_step3d" and (case.opts & mpdata.OPT_FCT or case.n_iters > 2):
        # the window spans every launch of a step: the 3-D kernel per pass
        # and the limited corrective pass (or donor pass) after it
        roof["kernel"] = "k_step3d + " + ("k_limcorr" if case.opts & mpdata.OPT_FCT
                                          else "k_donor") + " (whole step)"

    out = {
        "metric": "Mcell-steps/s", "value": round(value, 3), "unit": "Mcell-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if f32 else "f64", "data": "synthetic (seeded)",
        "config": {"workload": name, "shape": list(case.psi.shape), "n_iters": case.n_iters,
                   "opts": case.opts, "bc": "open" if case.bc else "periodic",
                   "kernel": "fused" if fused else "staged", "tile_rows": tile_rows,
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if not args.no_cpu:
        psi_o = case.psi.astype(np.float32).astype(np.float64) if f32 else case.psi
        c_o = [x.astype(np.float32).astype(np.float64) for x in case.c] if f32 else case.c
        g_o = case.g
        # bounded sample: a few steps of the full grid (the whole run of a
        # tiny grid); the GPU runs the same steps for the parity figures
        sample_steps = case.n_steps if N * case.n_steps <= 2 * 10 ** 7 else \
            max(1, min(4, 2 * 10 ** 7 // N))
        chk = psi0.clone()
        plan.step(chk, c, g=g, n_steps=sample_steps)
        torch.cuda.synchronize()
        got = chk.double().cpu().numpy()

        def run(parallel):
            return oracle.step(psi_o, c_o, g=g_o, n_iters=case.n_iters, opts=case.opts,
                               bc=case.bc, n_steps=sample_steps, parallel=parallel)

        rate1, ref = _oracle_rate(lambda: run(False), N * sample_steps)
        rate_mc, ref_mc = _oracle_rate(lambda: run(True), N * sample_steps)
        assert np.array_equal(ref, ref_mc)
        rel = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out["cpu_baseline"] = {
            "value": round(rate1 / 1e6, 4), "unit": "Mcell-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{sample_steps} steps of the full {name} grid, FP64 (also for FP32 runs)",
            "multicore": {"value": round(rate_mc / 1e6, 4), "unit": "Mcell-steps/s",
                          "cores": oracle.threads(parallel=True),
                          "kind": "oracle, OpenMP over each stage's outermost loop"}}
        out["parity_vs_oracle"] = {"steps": sample_steps, "rel_l2": rel,
                                   "max_dev": float(np.max(np.abs(got - ref))
                                                    / np.max(np.abs(ref)))}
    return out


def bench_batched(args, torch, mpdata, synth, oracle):
    """1024 independent 2-D periodic grids (sides 64..768), FP32, n_iters=2
    with the limiter: one launch per step over every tile of every grid,
    replayed from a HIP graph, against one launch per grid per step."""
    K = args.steps if args.steps is not None else 100
    W = args.warmup
    shapes = synth.batch_shapes()
    cases = synth.case_batch()
    dev = torch.device("cuda:0")
    bopts = mpdata.OPT_FCT | (mpdata.OPT_KAHAN if args.kahan else 0)
    bp = mpdata.BatchedPlan(shapes, dtype=torch.float32, n_iters=2, opts=bopts,
                            device=dev)
    psi0 = bp.pack([c.psi for c in cases], "psi")
    c0 = bp.pack([c.c[0] for c in cases], "c0")
    c1 = bp.pack([c.c[1] for c in cases], "c1")
    N = bp.n_psi
    if args.tile_rows is None:
        tile_rows, xcd = bp.autotune(psi0, c0, c1)      # outside the timed region
    else:
        tile_rows, xcd = args.tile_rows, bool(args.xcd_order)
        bp.set_tiling(tile_rows, xcd)
    psi = psi0.clone()
    bp.step(psi, c0, c1, n_steps=K, use_graph=True)       # capture + warm-up replay
    pg = psi0.clone()
    bp.step_per_grid(pg, c0, c1, n_steps=K)               # the same K steps, per grid
    torch.cuda.synchronize()
    same_bits = bool(torch.equal(psi, pg))
    secs = _time_steps(lambda k: bp.step(psi, c0, c1, n_steps=k, use_graph=True), K, torch)
    secs_pg = _time_steps(lambda k: bp.step_per_grid(pg, c0, c1, n_steps=k), K, torch)
    ms = secs * 1e3 / K
    # one launch per step (replayed back to back from the graph): the step
    # time is the kernel's launch time; read psi, both advector components
    # (without the periodic duplicate walls), write psi
    alg = 4 * (2 * N + bp.n_c0 - sum(b for a, b in shapes) + bp.n_c1 - sum(a for a, b in shapes))
    wname = "batched_1024x2d_periodic_64to768_fct_iters2"
    wl = "batched_f32" + ("_kahan" if args.kahan else "")
    ops = ALG_OPS[wname]
    out = {
        "metric": "Mcell-steps/s", "value": round(N * K / secs / 1e6, 3), "unit": "Mcell-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded)",
        "config": {"workload": wname + ("_kahan" if args.kahan else ""), "grids": len(shapes),
                   "cells": N, "launch": "one launch per step, HIP graph", "tile_rows": tile_rows,
                   "xcd_order": xcd, "parallelism": "single GPU"},
        "per_grid_launches": {"value": round(N * K / secs_pg / 1e6, 3), "unit": "Mcell-steps/s",
                              "ms_per_step": round(secs_pg * 1e3 / K, 6)},
        "speedup_vs_per_grid": round(secs_pg / secs, 3),
        "same_bits_as_per_grid": same_bits,
        "roofline": _roofline("k_fused2d_batched", ms, K, alg, alg_ops=ops * N,
                              traffic=_traffic_entry("k_fused2d_batched", wl),
                              valu=_valu_entry("k_fused2d_batched", wl, N, ops)),
    }
    if not args.no_cpu:
        order = [int(i) for i in np.argsort([a * b for a, b in shapes])[:4]]
        cells = sum(cases[i].psi.size for i in order) * 20

        def run(parallel):
            return [oracle.step(cases[i].psi.astype(np.float32).astype(np.float64),
                                [x.astype(np.float32).astype(np.float64) for x in cases[i].c],
                                n_iters=2, opts=bopts, n_steps=20, parallel=parallel)
                    for i in order]

        rate1, _ = _oracle_rate(lambda: run(False), cells)
        rate_mc, _ = _oracle_rate(lambda: run(True), cells)
        out["cpu_baseline"] = {"value": round(rate1 / 1e6, 4), "unit": "Mcell-steps/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "20 steps of the 4 smallest grids, FP64",
                               "multicore": {"value": round(rate_mc / 1e6, 4),
                                             "unit": "Mcell-steps/s",
                                             "cores": oracle.threads(parallel=True)}}
    return out


def bench_adjoint(args, torch, mpdata, synth, oracle):
    """Gradient of J = 1/2 ||psi_T - psi_obs||^2 w.r.t. psi0 and the advector
    through 200 steps of 2-D periodic 1024^2 FP64, n_iters=2 with the limiter,
    checkpoint every 20 steps."""
    w = synth.case_adjoint()
    case = w["case"]
    K = args.steps if args.steps is not None else case.n_steps
    ck = min(20, K)
    dev = torch.device("cuda:0")
    plan = mpdata.Plan(case.psi.shape, n_iters=2, opts=mpdata.OPT_FCT,
                       adj_steps=K, ckpt_every=ck, device=dev)
    psi = torch.from_numpy(case.psi).to(dev)
    c = [torch.from_numpy(x).to(dev) for x in case.c]
    obs = torch.from_numpy(w["psi_perturbed"]).to(dev)
    plan.step(obs, [torch.from_numpy(x).to(dev) for x in w["c_perturbed"]], n_steps=K)
    out = psi.clone()
    plan.step(out, c, n_steps=K)
    lam = (out - obs).contiguous()
    plan.autotune(psi, c)                   # chunk length of the fused state sweeps
    plan.adv_adj(psi, c, lam, n_steps=min(K, 2 * ck), ckpt_every=ck)     # warm-up
    t = {}

    def run(k):
        t["g"] = plan.adv_adj(psi, c, lam, n_steps=k, ckpt_every=ck)

    secs = _time_steps(run, K, torch)
    N = psi.numel()
    ms = secs * 1e3 / K
    # bytes per cell-step of the gradient: 16 FP64 values per cell (state, pass
    # field, advector, raw and limited pseudo-velocities, limiter coefficients,
    # adjoint in and out, advector adjoint read and written); the whole
    # gradient step (forward sweep, recompute with records, reverse kernels)
    # is the unit, so this is a step-level figure, not one kernel's
    alg = 8 * 16 * N
    res = {
        "metric": "Mcell-steps/s", "value": round(N * K / secs / 1e6, 3), "unit": "Mcell-steps/s",
        "n_gpus": 1, "steps": K, "warmup": 1, "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": "adjoint_2d_periodic_1024x1024_fct_iters2_ckpt20",
                   "checkpoint_every": ck, "parallelism": "single GPU"},
        "roofline": _roofline("whole gradient step", ms, K, alg),
    }
    if not args.no_cpu:
        sub = synth.case_2d(n=128, seed=5, sigma=(2.0, 8.0), n_iters=2, n_steps=10)
        lam_s = np.random.default_rng(0).normal(size=sub.psi.shape)

        def run(parallel):
            return oracle.adjoint(sub.psi, sub.c, lam_s, n_iters=2, opts=1, n_steps=10,
                                  ckpt_every=5, parallel=parallel)

        rate1, _ = _oracle_rate(lambda: run(False), sub.psi.size * 10)
        rate_mc, _ = _oracle_rate(lambda: run(True), sub.psi.size * 10)
        res["cpu_baseline"] = {"value": round(rate1 / 1e6, 4), "unit": "Mcell-steps/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "gradient through 10 steps of a 128^2 grid, FP64",
                               "multicore": {"value": round(rate_mc / 1e6, 4),
                                             "unit": "Mcell-steps/s",
                                             "cores": oracle.threads(parallel=True),
                                             "kind": "oracle, OpenMP forward stages; "
                                                     "reverse stages serial"}}
    return res


def bench_osc(args, torch, mpdata, synth, oracle):
    """Translating oscillator: 1-D periodic 1001 cells, C = 0.5,
    omega = 2 pi / 400, dt = 1, trapezoidal coupling, iga + fct, 1400 steps;
    each step advects both fields."""
    case = synth.case_osc()
    K = args.steps if args.steps is not None else case.n_steps
    W = args.warmup
    a = case.extra["a"]
    dev = torch.device("cuda:0")
    plan = mpdata.Plan(case.psi.shape, n_iters=case.n_iters, opts=case.opts, device=dev)
    c = [torch.from_numpy(x).to(dev) for x in case.c]
    psi0 = torch.from_numpy(case.psi).to(dev)
    phi0 = torch.from_numpy(case.extra["phi"]).to(dev)
    p, q = psi0.clone(), phi0.clone()
    plan.osc_step(p, q, c, a, n_steps=W)
    p, q = psi0.clone(), phi0.clone()
    secs = _time_steps(lambda k: plan.osc_step(p, q, c, a, n_steps=k), K, torch)
    N = 2 * case.psi.size                 # both fields advance every step
    ms = secs * 1e3 / K
    alg = 8 * 2 * (2 * case.psi.size + case.psi.size)   # psi, phi: read, write, + advector
    out = {
        "metric": "Mcell-steps/s", "value": round(N * K / secs / 1e6, 3), "unit": "Mcell-steps/s",
        "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "osc_1d_periodic_1001_iga_fct_iters2_trapez", "cells": N,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(alg / (ms / 1e3) / 1e9, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 6), "traffic": None,
                     "alg_bytes_per_launch": alg, "kernel": "whole oscillator step (4 launches)"},
    }
    if not args.no_cpu:
        t0 = time.perf_counter()
        rx, ry = oracle.osc_step(case.psi, case.extra["phi"], case.c, a, n_iters=case.n_iters,
                                 opts=case.opts, n_steps=K)
        dt = time.perf_counter() - t0
        torch.cuda.synchronize()
        got = np.concatenate([p.cpu().numpy(), q.cpu().numpy()])
        ref = np.concatenate([rx, ry])
        out["cpu_baseline"] = {"value": round(N * K / dt / 1e6, 4), "unit": "Mcell-steps/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"the whole {K}-step oscillator run, FP64, one thread"}
        out["parity_rel_l2_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    return out


def bench_sw(args, torch, mpdata, synth, oracle):
    """Shallow-water drop with prognosed velocity: 2-D open 2048 x 2048 over
    [-6, 6]^2, dt = dx / 5, g = 1, eps = 1e-8, iga + fct + dfl, n_iters = 2,
    FP64, from the drop at rest.  Each step computes the advector from two
    time levels, applies the trapezoidal forcing and advects the depth and
    both momenta."""
    case = synth.case_sw(n=2048)
    e = case.extra
    K = args.steps if args.steps is not None else 40
    W = args.warmup
    dev = torch.device("cuda:0")
    shape = case.psi.shape
    plan = mpdata.Plan(shape, n_iters=case.n_iters, opts=case.opts, bc=case.bc, device=dev)
    h0 = torch.from_numpy(case.psi).to(dev)
    q0 = [torch.from_numpy(x).to(dev) for x in e["q"]]
    c = [torch.empty((shape[0] + 1, shape[1]), dtype=torch.float64, device=dev),
         torch.empty((shape[0], shape[1] + 1), dtype=torch.float64, device=dev)]

    def fresh():
        return h0.clone(), [x.clone() for x in q0], h0.clone(), [x.clone() for x in q0]

    h, q, hp, qp = fresh()
    plan.sw_step(h, q, hp, qp, c, e["dt"], e["dx"], grav=e["grav"], eps=e["eps"], n_steps=W)
    h, q, hp, qp = fresh()
    secs = _time_steps(lambda k: plan.sw_step(h, q, hp, qp, c, e["dt"], e["dx"], grav=e["grav"],
                                              eps=e["eps"], n_steps=k), K, torch)
    cells = case.psi.size
    ms = secs * 1e3 / K
    # dominant kernel: the MPDATA step of one field (one launch, the donor
    # pass folded into the corrective pass), timed by the library's window
    # over K consecutive steps of the depth field with the last advector
    # (the window spans from the first to the last timed launch, so the
    # launches must follow each other)
    hh = h.clone()
    plan.step(hh, c, n_steps=2)
    plan.timing(K)
    plan.step(hh, c, n_steps=K)
    kern_ms, n_launch, kname = plan.timing_read()
    plan.timing(0)
    # algorithmic bytes of one field's step: psi and both advector
    # components read, psi written
    alg_k = 8 * (2 * cells + (shape[0] + 1) * shape[1] + shape[0] * (shape[1] + 1))
    # algorithmic bytes of a whole shallow-water step: levels n and n-1 of
    # h, q_x, q_y read, level n+1 written (the old level n becomes the
    # previous level)
    alg = 8 * 9 * cells
    out = {
        "metric": "Mcell-steps/s", "value": round(cells * K / secs / 1e6, 3),
        "unit": "Mcell-steps/s", "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(ms, 6),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": case.name + "_iga_fct_dfl_iters2_vip_trapez", "cells": cells,
                   "advected_fields": 3, "parallelism": "single GPU"},
        "roofline": _roofline(kname, kern_ms, n_launch, alg_k,
                              traffic=_traffic_entry(kname, "sw_2d_open_2048x2048")),
        "whole_step": {"alg_bytes": alg, "achieved_GBs": round(alg / (ms / 1e3) / 1e9, 2),
                       "frac": round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
    }
    if not args.no_cpu:
        sub = synth.case_sw(n=512)
        se = sub.extra
        n_sub = 24
        t0 = time.perf_counter()
        oracle.sw_run(sub.psi, se["q"], n_sub, se["dt"], se["dx"], eps=se["eps"],
                      grav=se["grav"], n_iters=sub.n_iters, opts=sub.opts, bc=sub.bc)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(sub.psi.size * n_sub / dt / 1e6, 4),
                               "unit": "Mcell-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{n_sub} steps of the same drop on 512 x 512 cells, "
                                         "FP64, one thread"}
    return out


def bench_copy(args, torch):
    """Calibration for the HBM byte counters: kernels of known traffic on a
    256 MiB buffer -- an elementwise in-place scale (reads and writes 256 MiB)
    and a device-to-device copy (reads and writes 256 MiB)."""
    K = args.steps if args.steps is not None else 20
    n = 256 * 1024 * 1024 // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a).fill_(2.0)
    b.mul_(1.0)
    b.copy_(a)
    s_scale = _time_steps(lambda k: [b.mul_(1.0) for _ in range(k)], K, torch)
    s_copy = _time_steps(lambda k: [b.copy_(a) for _ in range(k)], K, torch)
    gb = 2 * a.numel() * 8 / 1e9
    return {"metric": "copy GB/s", "value": round(gb * K / s_copy, 2), "unit": "GB/s",
            "n_gpus": 1, "steps": K, "warmup": 1, "ms_per_step": round(s_copy * 1e3 / K, 6),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic", "config": {"workload": "copy_256MiB"},
            "elementwise_scale_GBs": round(gb * K / s_scale, 2)}


def plan_uses_fused(plan, mpdata, requested):
    """Which step kernel the plan runs for the requested selection."""
    if requested == mpdata.KERNEL_STAGED:
        return False
    ok = mpdata.lib().mpdata_set_kernel(plan._handle, mpdata.KERNEL_FUSED) == 0
    plan.set_kernel(requested)
    return ok


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the MPDATA step "
              "here is a single-GPU build and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import oracle
    from paper_1407_1309_amd import mpdata, synth
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    if args.workload == "copy":
        out = bench_copy(args, torch)
    elif args.workload == "batched":
        out = bench_batched(args, torch, mpdata, synth, oracle)
    elif args.workload == "adjoint":
        out = bench_adjoint(args, torch, mpdata, synth, oracle)
    elif args.workload == "osc":
        out = bench_osc(args, torch, mpdata, synth, oracle)
    elif args.workload == "sw":
        out = bench_sw(args, torch, mpdata, synth, oracle)
    else:
        out = bench_single(args, torch, mpdata, synth, oracle)
        if args.workload == "2d" and not args.no_sub:
            # the metric's other two legs, observed in the same run
            keep = ("metric", "value", "unit", "steps", "ms_per_step", "dtype", "config",
                    "per_grid_launches", "speedup_vs_per_grid", "same_bits_as_per_grid",
                    "roofline", "cpu_baseline")
            for leg, fn in (("batched", bench_batched), ("adjoint", bench_adjoint)):
                sub = fn(args, torch, mpdata, synth, oracle)
                out[leg] = {k: sub[k] for k in keep if k in sub}
    if "cpu_baseline" in out:
        out["cpu_baseline"]["host"] = _host()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
