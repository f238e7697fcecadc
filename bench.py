"""Benchmark: batched entropic-OT Sinkhorn solves on SE(2) at 64 x 64 x 16.

Workload: B seeded pairs of lifted line images (8 segments of 10-40 px, each
moved by a small rigid motion for the second measure), w = (1, 3, 1), eps = 0.1,
11 x 11 window, log-domain Sinkhorn to marginal L1 1e-6 or 1000 iterations.
One step = one batch of B solves submitted together to the serving queue and
run to completion (continuous batching: one launch per half-step covers every
resident solve).  Inputs are on the device before the timed region starts.

Printed JSON line: the whole-job Sinkhorn iteration rate, solves/s (completed
and converged), p50/p99 solve latency, the roofline of the dominant kernel (the
log-domain convolution, timed with HIP events on the queue's stream), the same
solves run one at a time beside it, the FP64 CPU oracle timed on a bounded
sample on this host, and the linear se2_conv (BF16 and FP32, both on the matrix
cores) at the workloads' grid shapes against the BF16 and FP32 peaks.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

NX, NT, R = 64, 16, 5
W_METRIC = (1.0, 3.0, 1.0)
EPS = 0.1
# Minimum vector-ALU issue slots per LSE term the convolution kernel evaluates:
# dense visit = max pass (add, max) + sum pass (two FP64 adds, one FP64->FP32
# convert, one exp2 at EXP_SLOTS, one add); certified sparse visit = the sum pass
# only (the reference maximum is the shift).
EXP_SLOTS = 2  # v_exp_f32 issues at half rate on gfx950 (measured)
SLOTS_DENSE = 2 + 2 + 1 + EXP_SLOTS + 1
SLOTS_SPARSE = 2 + 1 + EXP_SLOTS + 1
# One slot = one lane-instruction; 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T
# lane-instructions/s is the vector-ALU issue peak.
VALU_PEAK = 39.3216
# Algorithmic HBM bytes per element of one log-domain half-step: the input potential,
# the log-marginal, the previous output (for the marginal error) and the new output,
# 4 bytes each in FP32.  The engine keeps those four arrays in FP64 (32 bytes).
BYTES_PER_ELEMENT = 16
FP64_STATE_BYTES_PER_ELEMENT = 32
# HBM bytes of one batched convolution half-step (k_sparse + k_rebuild of every lane) on
# this workload, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE (each scaled by what the
# counter reads for a plain 256 MiB copy: x2.0 and x1.0), summed over the 3 x 2004
# launch pairs of one bench step and divided by its 2004 half-steps;
# profiles/conv_lse_traffic_lines64x64x16_batch32.md.  Reported only while the kernel's
# sources (the kernel file and its shared header) are the ones measured.
TRAFFIC = {"sources_sha256": "4b92b2b3fb43faf22a994d6fe6185f846894a62a44e94e36acb14ceb54736175", "bytes_per_launch": 151655799.6,
           "sources": ("paper_2402_15322_amd/csrc/conv_lse.hip", "paper_2402_15322_amd/csrc/conv_lse.h")}


def measured_traffic():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC["sources"]:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC["bytes_per_launch"] if h.hexdigest() == TRAFFIC["sources_sha256"] else None


def log_conv_roofline(seconds, launches, outputs, terms_dense, terms_sparse, kernel, traffic=None):
    """Roofline of the log-domain convolution: algorithmic HBM bytes (BYTES_PER_ELEMENT per
    output element) per launch over the average launch time, against the HBM peak; beside it
    the vector-ALU issue rate of the terms evaluated, against the issue peak."""
    launches = max(1.0, launches)
    avg = seconds / launches
    elems = outputs / launches
    alg = BYTES_PER_ELEMENT * elems
    gbs = alg / avg / 1e9 if avg > 0 else 0.0
    slots = (SLOTS_DENSE * terms_dense + SLOTS_SPARSE * terms_sparse) / launches
    valu = slots / avg / 1e12 if avg > 0 else 0.0
    return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "traffic": traffic, "kernel": kernel, "avg_launch_us": avg * 1e6, "elements_per_launch": elems,
            "bytes_per_element": BYTES_PER_ELEMENT, "algorithmic_bytes_per_launch": alg,
            "fp64_state_bytes_per_element": FP64_STATE_BYTES_PER_ELEMENT,
            "fp64_state_frac": FP64_STATE_BYTES_PER_ELEMENT * elems / avg / 1e9 / PEAK_HBM_GBS if avg > 0 else None,
            "traffic_over_algorithmic": traffic / alg if traffic and alg > 0 else None,
            "dense_terms_per_launch": terms_dense / launches, "sparse_terms_per_launch": terms_sparse / launches,
            "valu_issue": {"lane_instr_per_s": valu * 1e12, "peak_lane_instr_per_s": VALU_PEAK * 1e12,
                           "frac": valu / VALU_PEAK, "instr_per_term": {"dense": SLOTS_DENSE, "sparse": SLOTS_SPARSE}}}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--max-iter", type=int, default=1000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--plain", type=int, default=2, help="solves run one at a time beside the queue")
    ap.add_argument("--cpu-iters", type=int, default=0, help="oracle iterations for the CPU baseline (0: auto)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="CPU only: the FP64 oracle timed per convolution, iteration and solve for every workload "
                         "configuration, all threads and one thread (own JSON line)")
    ap.add_argument("--oracle-timing-one-core", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-prune", action="store_true", help="dense convolutions only (no certified pruning)")
    ap.add_argument("--no-conv", action="store_true", help="skip the linear se2_conv measurements")
    ap.add_argument("--conv-only", action="store_true", help="only the linear se2_conv measurements")
    ap.add_argument("--conv-reps", type=int, default=20)
    ap.add_argument("--copy-ref-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size reference for HBM counters)")
    ap.add_argument("--serving", action="store_true",
                    help="serving workload instead: Poisson arrivals of mixed-size OT requests (own JSON line)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving trace that the default line carries as its `serving` object")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0, help="arrivals per second")
    ap.add_argument("--conv-rate", type=float, default=100.0,
                    help="arrivals per second of the converging (theta-motion) serving trace")
    ap.add_argument("--converging", action="store_true",
                    help="with --serving: the converging theta-motion trace instead of the paired lines")
    ap.add_argument("--budget-gb", type=float, default=4.0, help="queue HBM budget")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--plain-sample", type=int, default=2, help="one-at-a-time solves timed per grid size")
    ap.add_argument("--bary-n", type=int, default=6000,
                    help="class-barycenter leg: measures of 28x28x16 (0 skips the leg)")
    ap.add_argument("--bary-iters", type=int, default=20)
    ap.add_argument("--flow-steps", type=int, default=5, help="gradient-flow leg: JKO steps (0 skips the leg)")
    ap.add_argument("--c4-iters", type=int, default=5,
                    help="barycenter legs: IBP iterations of the 256x256x32 field workload (0 skips both legs)")
    ap.add_argument("--eps-start", type=float, default=1.6,
                    help="eps-scaling leg: first eps of the schedule (<= 0.1 skips the leg)")
    ap.add_argument("--eps-factor", type=float, default=0.5)
    ap.add_argument("--stage-iters", type=int, default=100)
    ap.add_argument("--conv-batch", type=int, default=32,
                    help="converged leg: theta-motion solves submitted together (0 skips the leg)")
    ap.add_argument("--conv-max-iter", type=int, default=3000)
    ap.add_argument("--conv-engines", default="f32,bf16>f32,f32_mfma,bf16>f32_mfma",
                    help="converged leg: engines, comma separated (prec, or bulk>prec)")
    ap.add_argument("--converged-only", action="store_true", help="only the converged leg (for profiling)")
    ap.add_argument("--eps-only", action="store_true",
                    help="only the eps-scaling leg of the headline batch on every engine (no timed steps)")
    ap.add_argument("--fields-only", action="store_true",
                    help="only the 256x256x32 axial-field barycenter on every engine (for profiling)")
    ap.add_argument("--halo-spread", action="store_true",
                    help="only the spread of the log-potentials over a tile's halo and the matrix-core engines' "
                         "fallback shares, per workload and eps")
    return ap.parse_args()


# Linear group convolutions timed beside the solver: the three grid shapes of the
# workloads, each at the batch one half-step of that workload applies (one convolution
# per solve at 64x64x16 for the bench batch; 2 measures x 5 interpolation weights at
# 128x128x16; 4 measures at 256x256x32 axial).
CONV_SHAPES = (
    # n, ntheta, radius, axial, w, eps, batch (None: the bench batch)
    (64, 16, 5, False, (1.0, 3.0, 1.0), 0.1, None),
    (128, 16, 7, False, (1.0, 3.0, 1.0), 0.05, 10),
    (256, 32, 10, True, (1.0, 4.0, 1.0), 0.03, 4),
)
PEAK_BF16_TFLOPS = 2500.0  # dense MFMA, bf16
PEAK_F32_TFLOPS = 157.3


def conv_measurements(native, torch, batch: int, reps: int):
    """se2_conv (BF16 and FP32) timed with HIP events on the current stream."""
    out = []
    for n, nt, R, axial, w, eps, b in CONV_SHAPES:
        b = b or batch
        k = native.Kernel(n, n, nt, axial, w, eps, R)
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        x = torch.rand((b, n, n, nt), device="cuda", generator=g)
        y = torch.empty_like(x)
        flops = 2.0 * b * n * n * nt * nt * (2 * R + 1) ** 2
        rec = {"shape": f"{n}x{n}x{nt}{' axial' if axial else ''}, {2 * R + 1}x{2 * R + 1} window", "batch": b,
               "flops_per_launch": flops}
        for prec, tag, peak in ((native.SE2_BF16, "bf16", PEAK_BF16_TFLOPS), (native.SE2_F32, "f32", PEAK_F32_TFLOPS)):
            native.se2_conv(k, prec, x, y)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                native.se2_conv(k, prec, x, y)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3 / reps
            rec[f"{tag}_us"] = t * 1e6
            rec[f"{tag}_tflops"] = flops / t / 1e12
            rec[f"{tag}_frac"] = flops / t / 1e12 / peak
        out.append(rec)
        del k
    return out


PEAK_HBM_GBS = 8000.0


def field_measurements(native, torch, reps: int):
    """Lift and projection (HBM-bound) on the orientation-field workload's grid: 4 fields of
    256 x 256 pixels, 32 axial orientation bins.  Bytes are the algorithmic ones: the lift
    reads magnitude and angle and writes ntheta values per pixel; the projection reads
    ntheta values and writes mass, argmax and angle per pixel."""
    n, nt, b = 256, 32, 4
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    mag = torch.rand((b, n, n), device="cuda", dtype=torch.float64, generator=g)
    ang = torch.rand((b, n, n), device="cuda", dtype=torch.float64, generator=g) * math.pi
    u = torch.empty((b, n, n, nt), device="cuda", dtype=torch.float64)
    mass = torch.empty((b, n, n), device="cuda", dtype=torch.float64)
    angle = torch.empty_like(mass)
    arg = torch.empty((b, n, n), device="cuda", dtype=torch.int32)
    npix = b * n * n
    legs = {"lift": (lambda: native.se2_lift_field(nt, True, mag, ang, u), npix * (16 + 8 * nt)),
            "project": (lambda: native.se2_project(True, u, mass, argmax=arg, angle=angle), npix * (8 * nt + 20))}
    out = {"shape": f"{b} x {n}x{n}x{nt} axial", "bound": "hbm", "peak_gbs": PEAK_HBM_GBS}
    for name, (fn, nbytes) in legs.items():
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / reps
        out[name] = {"us": t * 1e6, "bytes": nbytes, "gbs": nbytes / t / 1e9, "frac": nbytes / t / 1e9 / PEAK_HBM_GBS}
    return out


def class_barycenter(native, torch, images, iters: int, engines=("f32_mfma", "bf16")):
    """Barycenter of a whole class of small images (the paper's MNIST/QuickDraw setting:
    28 x 28 images, 16 orientations, spatial anisotropy 1.5, ~6000 images per class), here
    seeded stroke images: w = (1, 1.5, 1), eps = 0.5, 9 x 9 window, equal weights, IBP on the
    dense engine, through the queue with convolution timing on.  Run at `iters` and at
    2 * `iters` iterations: the difference is the steady-state cost of `iters` iterations
    (admission, validation and finishing cancel).  The same on the matrix-core engines, with
    the share of (tile, orientation) groups they recomputed exactly."""
    n = images.shape[0]
    k = native.Kernel(28, 28, 16, False, (1.0, 1.5, 1.0), 0.5, 4)
    dev = torch.from_numpy(images).cuda()
    mus = [dev[i] for i in range(n)]
    out = torch.empty(images.shape[1:], dtype=torch.float64, device="cuda")

    def two_runs(o_of):
        runs = []
        for it in (iters, 2 * iters):
            o = o_of(it)
            q = native.SolveQueue(hbm_budget_bytes=int(n) * (1 << 20) + (1 << 30), max_slots=1)
            q.profile(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ticket = q.submit_barycenter(k, mus, [1.0 / n] * n, o, out)
            rep = q.wait(ticket)
            wall = time.perf_counter() - t0
            kt = q.kernel_time()
            q.close()
            runs.append((wall, kt, rep))
        return runs

    (w1, k1, r1), (w2, k2, r2) = two_runs(
        lambda it: native.opts(tol=-1.0, max_iter=it, check_every=it, final_check=False, prune=False))
    per_iter = (w2 - w1) / iters
    conv_s = k2["seconds"] - k1["seconds"]
    terms = k2["terms"] - k1["terms"]
    res = {"workload": f"{n} stroke images 28x28x16, w=(1,1.5,1), eps=0.5, 9x9 window, equal weights",
           "measures": n, "iters": [r1["iters"], r2["iters"]], "wall_s": [w1, w2],
           "steady_ms_per_iter": per_iter * 1e3, "steady_iters_per_s": 1.0 / per_iter if per_iter > 0 else None,
           "convs_per_s": 2.0 * n / per_iter if per_iter > 0 else None,
           "conv_ms_per_iter": conv_s / iters * 1e3,
           "avg_conv_launch_us": conv_s / max(1.0, k2["launches"] - k1["launches"]) * 1e6,
           "lse_terms_per_s": terms / conv_s if conv_s > 0 else None,
           "roofline": log_conv_roofline(conv_s, k2["launches"] - k1["launches"], k2["outputs"] - k1["outputs"],
                                         terms, 0.0, "dense log-domain convolution (k_conv_lse)"),
           "marg_l1": r2["marg_l1"], "mass": r2["mass"], "matrix_core_engines": {}}
    groups_per_iter = 2.0 * n * 16 * (28 // 8 + 1) ** 2
    for name in engines:
        (v1, q1, s1), (v2, q2, s2) = two_runs(
            lambda it: engine_opts(native, name, tol=-1.0, max_iter=it, check_every=it, final_check=False))
        pi = (v2 - v1) / iters
        res["matrix_core_engines"][name] = {
            "steady_ms_per_iter": pi * 1e3, "conv_ms_per_iter": (q2["seconds"] - q1["seconds"]) / iters * 1e3,
            "fallback_group_share": (s2["fallbacks"] - s1["fallbacks"]) / (iters * groups_per_iter),
            "marg_l1": s2["marg_l1"], "marg_l1_rel_diff_vs_exact": abs(s2["marg_l1"] - r2["marg_l1"]) / r2["marg_l1"]}
    return res


def gradient_flow(native, torch, synth, steps: int):
    """Porous-medium gradient flow of a line-completion image (Section 5.4: m = 5,
    w = (1, sqrt 10, sqrt 2)) on 64 x 64 x 16: a dashed dominant line amid short line
    elements; eps = 0.5, 11 x 11 window, tau = 1e-4, F on densities against the cell measure
    1/(64*64*16); `steps` JKO steps on the device, each to first-marginal L1 1e-6 (max 500
    inner iterations), warm-started from the previous step."""
    mu = synth.line_completion()
    E = mu.size
    k = native.Kernel(64, 64, 16, False, (1.0, math.sqrt(10.0), math.sqrt(2.0)), 0.5, 5)
    mud = torch.from_numpy(mu).cuda()
    out = torch.empty_like(mud)
    o = native.opts(tol=1e-6, max_iter=500, check_every=10, final_check=False, prune=True)
    native.se2_gradient_flow(k, mud, 1e-4, 5.0, 1.0 / E, 1, o, out)   # warm-up (kernel tables, lists)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = native.se2_gradient_flow(k, mud, 1e-4, 5.0, 1.0 / E, steps, o, out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    inner = sum(r["iters"] for r in reps)
    return {"workload": "line-completion image 64x64x16, m=5, w=(1,sqrt10,sqrt2), eps=0.5, 11x11 window, "
                        "tau=1e-4, ref=1/E, tol 1e-6", "steps": steps, "wall_s": wall,
            "jko_steps_per_s": steps / wall, "inner_iters": [r["iters"] for r in reps],
            "inner_iters_per_s": inner / wall, "converged": sum(1 for r in reps if r["status"] == 0),
            "energy": [r["dual"] for r in reps], "transport_cost": [r["cost"] for r in reps]}


def barycenter_workloads(native, torch, synth, c4_iters: int, only=None):
    """The two barycenter workloads through the queue, convolution timing on.
    128x128x16 interpolation: two Bezier-stroke measures, w = (1,3,1), eps = 0.05, 15x15
    window, the five weights t in {0, 1/4, 1/2, 3/4, 1} as five resident requests, tol 1e-6,
    max 1000 IBP iterations, pruned engine.  256x256x32 axial fields: four measures, equal
    weights, w = (1,4,1), eps = 0.03, 21x21 window (the dense engine: the FP64 halo does not
    fit the sparse kernel's LDS), `c4_iters` IBP iterations.  `only`: the names to run."""
    import numpy as np
    out = {}
    for name, insts, o in (
            ("curves128x128x16_t5", [synth.curves128(0, t=t) for t in (0.0, 0.25, 0.5, 0.75, 1.0)],
             native.opts(tol=1e-6, max_iter=1000, check_every=10, final_check=True, prune=True)),
            ("fields256x256x32_axial_n4", [synth.fields256(0)],
             native.opts(tol=-1.0, max_iter=c4_iters, check_every=c4_iters, final_check=False, prune=True))):
        if only is not None and name not in only:
            continue
        g = insts[0].grid
        k = native.Kernel(g.nx, g.ny, g.nt, g.axial, insts[0].w, insts[0].eps, insts[0].radius)
        dev = [[torch.from_numpy(m).cuda() for m in inst.mus] for inst in insts]
        outs = [torch.empty_like(d[0]) for d in dev]
        q = native.SolveQueue(hbm_budget_bytes=8 << 30, max_slots=len(insts))
        q.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ts = [q.submit_barycenter(k, d, inst.lambdas, o, b) for d, inst, b in zip(dev, insts, outs)]
        reps = [q.wait(t) for t in ts]
        wall = time.perf_counter() - t0
        kt = q.kernel_time()
        q.close()
        engines = {}
        if name.startswith("fields256"):
            # the same IBP iterations as blocking calls on the exact engine and the matrix-core
            # engines, each barycenter against the queue's exact one (no oracle at this size; the
            # 64x64x8 downsample is in cpu_baseline).  Runs of c4_iters and 2 c4_iters iterations
            # are differenced: the cost per iteration without validation and finishing (later
            # iterations recompute more groups on the matrix-core engines than the first ones).
            ref = outs[0].cpu().numpy()
            E = float(ref.size)
            groups_per_iter = 2.0 * len(insts[0].mus) * (E / (64.0 * g.nt)) * g.nt
            for ename in ("f32", "bf16", "f32_mfma"):
                runs = []
                for it in (c4_iters, 2 * c4_iters):
                    oe = engine_opts(native, ename, tol=-1.0, max_iter=it, check_every=it, final_check=False)
                    be = torch.empty_like(outs[0])
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    re_ = native.se2_barycenter(k, dev[0], insts[0].lambdas, oe, be)
                    torch.cuda.synchronize()
                    runs.append((time.perf_counter() - t1, re_, be))
                (w1, r1, b1), (w2, r2, _) = runs
                per = (w2 - w1) / c4_iters
                engines[ename] = {"wall_s": w1, "ibp_iters_per_s": r1["iters"] / w1,
                                  "steady_ms_per_iter": per * 1e3,
                                  "fallback_group_share": (r2["fallbacks"] - r1["fallbacks"]) / (c4_iters * groups_per_iter),
                                  "barycenter_l1_vs_exact": float(np.abs(b1.cpu().numpy() - ref).sum())}
        out[name] = {"requests": len(insts), "iters": [r["iters"] for r in reps],
                     "converged": sum(1 for r in reps if r["status"] == native.SE2_CONVERGED),
                     "wall_s": wall, "ibp_iters_per_s": sum(r["iters"] for r in reps) / wall,
                     "marg_l1": [r["marg_l1"] for r in reps], "mass": [r["mass"] for r in reps],
                     "conv_seconds": kt["seconds"], "half_steps": kt["launches"],
                     "dense_terms": sum(r["terms_dense"] for r in reps),
                     "sparse_terms": sum(r["terms_sparse"] for r in reps),
                     "roofline": log_conv_roofline(kt["seconds"], kt["launches"], kt["outputs"],
                                                   sum(r["terms_dense"] for r in reps),
                                                   sum(r["terms_sparse"] for r in reps), "log-domain convolution"),
                     "matrix_core_engines": engines or None}
        del dev, outs, k
    return out


ENGINES = {"f32": ("SE2_F32", None), "f64": ("SE2_F64", None), "bf16": ("SE2_BF16", None),
           "f32_mfma": ("SE2_F32_MFMA", None), "bf16>f32": ("SE2_F32", "SE2_BF16"),
           "bf16>f32_mfma": ("SE2_F32_MFMA", "SE2_BF16")}


def engine_opts(native, name, **kw):
    prec, bulk = ENGINES[name]
    return native.opts(prec=getattr(native, prec), bulk=None if bulk is None else getattr(native, bulk), **kw)


def converged_leg(native, torch, synth, a):
    """The converging 64x64x16 instance: nu is mu's strokes with each segment's orientation
    turned by a seeded angle in U[-pi/16, pi/16] (a motion along theta), strokes splatted with
    sigma_xy = 3 px, floor 1e-6, w = (1,3,1), eps = 0.1, 11x11 window.  `conv_batch` solves are
    submitted together to the serving queue and run to marginal L1 1e-6 (at most
    `conv_max_iter` iterations), once per engine (warm-up run first, then the timed one), with
    convolution timing on: exact FP32 with certified pruning, FP32 on the matrix cores, and a
    bfloat16 bulk phase on the matrix cores before either.  The matrix-core engines' rate is
    the dense-window flops (2 per in-grid window term) over the union of the launch intervals."""
    import numpy as np
    insts = [synth.lines64_theta(i) for i in range(a.conv_batch)]
    g = insts[0].grid
    k = native.Kernel(g.nx, g.ny, g.nt, False, insts[0].w, insts[0].eps, insts[0].radius)
    mus = [torch.from_numpy(x.mu).cuda() for x in insts]
    nus = [torch.from_numpy(x.nu).cuda() for x in insts]
    res, pots, pick = {}, {}, 0
    for name in [e for e in a.conv_engines.split(",") if e]:
        o = engine_opts(native, name, tol=1e-6, max_iter=a.conv_max_iter, check_every=a.check_every,
                        final_check=True, prune=True, switch_tol=1e-3)
        fs = [torch.empty_like(m) for m in mus]
        gs = [torch.empty_like(m) for m in mus]
        q = native.SolveQueue(hbm_budget_bytes=native.ot_request_bytes(k, o) * a.conv_batch + (64 << 20),
                              max_slots=a.conv_batch)
        # warm-up, then the timed run, then a run with the convolution timing events on (its
        # solves are the same: the results do not depend on timing); the events cost most on
        # the small launches of a batch's last solves, so the timed run goes without them
        for run in ("warm-up", "timed", "profiled"):
            if run == "profiled":
                q.profile(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ts = [q.submit_ot(k, mus[i], nus[i], o, fs[i], gs[i]) for i in range(a.conv_batch)]
            reps_run = [q.wait(t) for t in ts]
            torch.cuda.synchronize()
            wall_run = time.perf_counter() - t0
            lat_run = []
            for t in ts:
                t_s, _, t_d = q.times(t)
                lat_run.append(t_d - t_s)
                q.release(t)
            if run == "timed":
                reps, wall, lat = reps_run, wall_run, lat_run
            elif run == "profiled":
                wall_prof = wall_run
        kt = q.kernel_time()
        q.close()
        its = np.array([r["iters"] for r in reps])
        conv = sum(1 for r in reps if r["status"] == native.SE2_CONVERGED)
        lin = sum(r["terms_linear"] for r in reps)
        rec = {"wall_s": wall, "converged": conv, "solves": len(reps), "converged_solves_per_s": conv / wall,
               "iters_per_s": float(its.sum()) / wall, "iters_median": float(np.median(its)), "iters_max": int(its.max()),
               "p50_latency_ms": float(np.percentile(lat, 50) * 1e3), "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
               "marg_l1_max": max(r["marg_l1"] for r in reps), "marg_l1_f64_max": max(r["marg_l1_f64"] for r in reps),
               "phase_switch_iter_median": float(np.median([r["phase_switch_iter"] for r in reps])),
               "fallback_groups": int(sum(r["fallbacks"] for r in reps)),
               "conv_seconds": kt["seconds"], "half_steps": kt["launches"],
               "avg_half_step_us": kt["seconds"] / max(1.0, kt["launches"]) * 1e6,
               "wall_s_with_timing_events": wall_prof}
        groups = 2.0 * float(its.sum()) * (g.nx // 8) * (g.ny // 8) * g.nt
        if lin > 0:
            # share of the window terms the matrix cores evaluated, and the rate of the whole
            # convolution time in dense-window flops against the peak of the final engine
            peak = PEAK_F32_TFLOPS if ENGINES[name][0] == "SE2_F32_MFMA" else PEAK_BF16_TFLOPS
            tf = 2.0 * kt["terms"] / kt["seconds"] / 1e12 if kt["seconds"] > 0 else 0.0
            rec["matrix_core"] = {"terms_share": lin / max(1.0, kt["terms"]), "dense_window_tflops": tf,
                                  "peak_tflops": peak, "frac": tf / peak,
                                  "fallback_groups_per_group_of_all_half_steps": rec["fallback_groups"] / groups}
        res[name] = rec
        if not pots:
            # the instance the first engine solved in the fewest iterations: the one the oracle
            # then runs to convergence beside them (its time stays bounded)
            pick = int(np.argmin(its))
        pots[name] = [(fs[pick].cpu().numpy(), gs[pick].cpu().numpy())]
    out = {"workload": "lines64x64x16-theta OT: orientation turned by U[-pi/16, pi/16] per segment, sigma_xy = 3 px, "
                       "floor 1e-6, w=(1,3,1), eps=0.1, 11x11 window, tol 1e-6, serving queue",
           "batch": a.conv_batch, "max_iter": a.conv_max_iter, "engines": res}
    return out, pots, insts[pick]


def halo_spread(native, torch, synth):
    """Why the matrix-core engines fall back: the spread of log2 b (the input of an a-update)
    and of log2 a over the halo of each 16 x 16 output tile (radius 5), for the 64x64x16 paired
    lines at eps 0.05, 0.1 and 0.5 after 50 and 1000 iterations (exact engine) and for the
    theta-motion instance; raw (max - min: one shift per tile), after removing a per-orientation
    offset, and after removing a least-squares plane in (x, y) plus a per-orientation offset.
    A tile's shifted values must stay within 87 (the certificate) for its outputs to pass.
    Beside it, the share of (tile, orientation) groups that the FP32 matrix-core engine
    recomputes exactly over 300 iterations, and the same for the class barycenter."""
    import numpy as np

    def spreads(x2, R=5, T=16):
        ny, nx, nt = x2.shape
        out = []
        for ty in range(0, ny, T):
            for tx in range(0, nx, T):
                h = x2[max(ty - R, 0):min(ty + T + R, ny), max(tx - R, 0):min(tx + T + R, nx), :]
                fin = np.isfinite(h)
                v = h[fin]
                yy, xx, kk = np.nonzero(fin)
                a2 = np.zeros((len(v), nt))
                a2[np.arange(len(v)), kk] = 1.0
                r2 = v - a2 @ np.linalg.lstsq(a2, v, rcond=None)[0]
                a3 = np.concatenate([np.stack([xx, yy], 1).astype(float), a2], 1)
                r3 = v - a3 @ np.linalg.lstsq(a3, v, rcond=None)[0]
                out.append((v.max() - v.min(), r2.max() - r2.min(), r3.max() - r3.min()))
        s_ = np.array(out)
        return {name: {"median": float(np.median(s_[:, i])), "p90": float(np.percentile(s_[:, i], 90)),
                       "share_within_87": float(np.mean(s_[:, i] <= 87.0))}
                for i, name in enumerate(("one_shift", "per_orientation", "plane_and_per_orientation"))}

    rec = {"tile": "16x16 outputs, halo radius 5, log2 units", "cases": []}
    for label, make, epss in (("lines64x64x16-paired/0", lambda: synth.lines64(0), (0.05, 0.1, 0.5)),
                              ("lines64x64x16-theta/0", lambda: synth.lines64_theta(0), (0.1,))):
        inst = make()
        g = inst.grid
        mu, nu = torch.from_numpy(inst.mu).cuda(), torch.from_numpy(inst.nu).cuda()
        for eps in epss:
            k = native.Kernel(g.nx, g.ny, g.nt, False, inst.w, eps, inst.radius)
            f, gg = torch.empty_like(mu), torch.empty_like(mu)
            for iters in (50, 1000):
                native.se2_sinkhorn(k, mu, nu, native.opts(tol=-1.0, max_iter=iters, check_every=50), f, gg)
                rec["cases"].append({"instance": label, "eps": eps, "iters": iters,
                                     "log2_b": spreads(gg.cpu().numpy() / eps / math.log(2.0)),
                                     "log2_a": spreads(f.cpu().numpy() / eps / math.log(2.0))})
            rep = native.se2_sinkhorn(k, mu, nu, native.opts(tol=-1.0, max_iter=300, prec=native.SE2_F32_MFMA), f, gg)
            rec["cases"][-1]["f32_mfma_fallback_share_300_iters"] = rep["fallbacks"] / (300.0 * 2 * (g.nx // 8) ** 2 * g.nt)
    imgs = synth.stroke_images(600, seed=6000)
    kb = native.Kernel(28, 28, 16, False, (1.0, 1.5, 1.0), 0.5, 4)
    dev = [torch.from_numpy(m).cuda() for m in imgs]
    out = torch.empty_like(dev[0])
    shares = {}
    for name in ("bf16", "f32_mfma"):
        rep = native.se2_barycenter(kb, dev, [1.0 / len(dev)] * len(dev),
                                    engine_opts(native, name, tol=-1.0, max_iter=20, check_every=20, final_check=False), out)
        shares[name] = rep["fallbacks"] / (20.0 * 2 * len(dev) * 16 * 16)
    rec["class_barycenter_600_images_fallback_share_20_iters"] = shares
    return rec


def eps_scaling_leg(native, torch, k, mus, nus, fs, gs, a, plain_curve=False):
    """The headline batch with eps-scaling: stage_iters iterations at each eps of
    eps_start * factor^s above the workload's eps, the rest of the same iteration budget at it;
    on the exact engine, and with a matrix-core bulk engine over the coarse stages
    (switch_tol 1: the exact engine takes over at the first check of the final eps, or earlier
    when over a quarter of the bulk engine's groups fall back).  Each variant runs a warm-up
    batch, then the timed one.  plain_curve: also the batch without eps-scaling at 2000, 3000
    and 4000 iterations (time to a given error)."""
    import numpy as np

    def eps_run(bulk=None, scaled=True, max_iter=None):
        o_s = native.opts(tol=a.tol, max_iter=max_iter or a.max_iter, check_every=a.check_every, final_check=True,
                          prune=not a.no_prune, eps_start=a.eps_start if scaled else 0.0, eps_factor=a.eps_factor,
                          stage_iters=a.stage_iters if scaled else 0, bulk=bulk, switch_tol=1.0)
        qs = native.SolveQueue(hbm_budget_bytes=native.ot_request_bytes(k, o_s) * a.batch + (64 << 20),
                               max_slots=a.batch)
        for _ in range(2):  # a warm-up batch (stage kernels, tables), then the timed one
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            ts_ = [qs.submit_ot(k, mus[i], nus[i], o_s, fs[i], gs[i]) for i in range(a.batch)]
            rs_ = [qs.wait(t) for t in ts_]
            torch.cuda.synchronize()
            w_s = time.perf_counter() - s0
            for t in ts_:
                qs.release(t)
        qs.close()
        return {"iters_per_s": sum(r["iters"] for r in rs_) / w_s, "wall_s": w_s,
                "coarse_iters_per_solve": rs_[0]["scaling_iters"],
                "converged": sum(1 for r in rs_ if r["status"] == native.SE2_CONVERGED),
                "marg_l1_mean": float(np.mean([r["marg_l1"] for r in rs_])),
                "marg_l1_f64_mean": float(np.mean([r["marg_l1_f64"] for r in rs_])),
                "fallback_groups": int(sum(r["fallbacks"] for r in rs_)),
                "phase_switch_iter_median": float(np.median([r["phase_switch_iter"] for r in rs_]))}

    rec = {"schedule": {"eps_start": a.eps_start, "factor": a.eps_factor, "stage_iters": a.stage_iters},
           **eps_run(),
           "matrix_core_bulk": {"f32_mfma": eps_run(native.SE2_F32_MFMA), "bf16": eps_run(native.SE2_BF16)}}
    if plain_curve:
        rec["plain_curve"] = [{"iters": n, **{key: v for key, v in eps_run(scaled=False, max_iter=n).items()
                                              if key in ("wall_s", "marg_l1_mean")}} for n in (2000, 3000, 4000)]
    return rec


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 (sharding a solve or the "
                                   "request stream across GPUs is not implemented)"}))
        sys.exit(2)
    if a.oracle_timing:
        # CPU only (no GPU work in this process): all threads, then a one-thread child for the
        # convolutions
        import platform
        import subprocess
        import oracle
        model = platform.processor()
        try:
            with open("/proc/cpuinfo") as fh:
                model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), model)
        except OSError:
            pass
        rec = {"mode": "oracle_timing", "kind": "oracle", "host": {"nproc": os.cpu_count(), "cpu_model": model},
               "all_threads": dict(threads=oracle.num_threads(), **oracle_timing())}
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-timing-one-core"], env=env,
                           capture_output=True, text=True, timeout=600)
        rec["one_thread"] = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else {"error": r.stderr[-500:]}
        print(json.dumps(rec), flush=True)
        return
    if a.oracle_timing_one_core:
        import oracle
        print(json.dumps(dict(threads=oracle.num_threads(), **oracle_timing(one_conv_only=True))), flush=True)
        return
    import numpy as np
    import torch

    from paper_2402_15322_amd import native, synth

    # inputs of the class-barycenter leg, drawn in forked workers before any GPU work
    class_images = None
    workers = min(16, os.cpu_count() or 1)
    if a.bary_n > 0 and not (a.conv_only or a.serving):
        class_images = synth.stroke_images(a.bary_n, workers=workers)
    trace = trace_conv = None
    if (a.serving and not a.converging) or not (a.serving or a.conv_only or a.no_serving):
        trace = synth.serving_trace(a.requests, a.rate, workers=workers)
    if (a.serving and a.converging) or not (a.serving or a.conv_only or a.no_serving):
        # the 16-orientation grids: theta-motion pairs on 32x32x8 stay above 1e-6 after 3000
        # iterations (the oracle gives 9e-6 to 2.6e-5 there)
        trace_conv = synth.serving_trace(a.requests, a.conv_rate, seed=3100, paired="theta",
                                         grids=synth.SERVE_GRIDS[1:], workers=workers)

    torch.cuda.set_device(0)
    native.se2_init()
    if a.copy_ref_mb > 0:
        src = torch.ones(a.copy_ref_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.conv_only:
        print(json.dumps({"se2_conv": conv_measurements(native, torch, a.batch, a.conv_reps),
                          "lift_project": field_measurements(native, torch, a.conv_reps)}), flush=True)
        return
    if a.serving:
        print(json.dumps(serving(native, torch, synth, a, trace_conv if a.converging else trace,
                                 converging=a.converging)), flush=True)
        return
    if a.converged_only:
        print(json.dumps(converged_leg(native, torch, synth, a)[0]), flush=True)
        return
    if a.fields_only:
        print(json.dumps(barycenter_workloads(native, torch, synth, a.c4_iters, ("fields256x256x32_axial_n4",))),
              flush=True)
        return
    if a.halo_spread:
        print(json.dumps(halo_spread(native, torch, synth)), flush=True)
        return
    k = native.Kernel(NX, NX, NT, False, W_METRIC, EPS, R)
    insts = [synth.lines64(i, paired=True) for i in range(a.batch)]
    mus = [torch.from_numpy(x.mu).cuda() for x in insts]
    nus = [torch.from_numpy(x.nu).cuda() for x in insts]
    fs = [torch.empty_like(m) for m in mus]
    gs = [torch.empty_like(m) for m in mus]
    torch.cuda.synchronize()
    if a.eps_only:
        print(json.dumps({"eps_scaling": eps_scaling_leg(native, torch, k, mus, nus, fs, gs, a, plain_curve=True)}),
              flush=True)
        return
    o = native.opts(tol=a.tol, max_iter=a.max_iter, check_every=a.check_every, final_check=True,
                    prune=not a.no_prune)
    # the budget admits the whole batch (each solve keeps its potentials and pruning state resident)
    q = native.SolveQueue(hbm_budget_bytes=native.ot_request_bytes(k, o) * a.batch + (64 << 20), max_slots=a.batch)

    def one_step(lat):
        tickets = [q.submit_ot(k, mus[i], nus[i], o, fs[i], gs[i]) for i in range(a.batch)]
        reps = [q.wait(t) for t in tickets]
        for t in tickets:
            ts, _, td = q.times(t)
            lat.append(td - ts)
            q.release(t)
        return reps

    for _ in range(a.warmup):
        one_step([])
    q.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_r, lat, step_ms = [], [], []
    for _ in range(a.steps):
        s0 = time.perf_counter()
        all_r += one_step(lat)
        step_ms.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    kt = q.kernel_time()
    q.profile(False)
    lat = np.array(lat)
    q.close()

    iters = sum(r["iters"] for r in all_r)
    conv = sum(1 for r in all_r if r["status"] == native.SE2_CONVERGED)
    value = iters / wall

    # roofline of the dominant kernel (log-domain convolution, one launch = one batched
    # half-step of every resident solve): algorithmic HBM bytes per launch over its average
    # duration (HIP events on the queue's streams, union over the lanes, timed region)
    roof = log_conv_roofline(kt["seconds"], kt["launches"], kt["outputs"], sum(r["terms_dense"] for r in all_r),
                             sum(r["terms_sparse"] for r in all_r),
                             "log-domain convolution (k_sparse + k_rebuild), one batched half-step per launch",
                             measured_traffic())
    roof["window_terms_per_launch"] = kt["terms"] / max(1.0, kt["launches"])

    # the same solves one at a time (plain per-solve FP32 Sinkhorn on the same engine)
    plain_iters, plain_wall = 0, 0.0
    o_plain = native.opts(tol=a.tol, max_iter=a.max_iter, check_every=a.check_every, final_check=True, prune=False)
    for i in range(min(a.plain, a.batch)):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        rep = native.se2_sinkhorn(k, mus[i], nus[i], o_plain, fs[i], gs[i])
        torch.cuda.synchronize()
        plain_wall += time.perf_counter() - s0
        plain_iters += rep["iters"]
    plain_rate = plain_iters / plain_wall if plain_wall > 0 else None

    # eps-scaling leg (outside the timed region): the same batch with the same iteration budget,
    # stage_iters iterations at each eps of eps_start * factor^s above 0.1, the rest at 0.1
    eps_leg = None
    if a.eps_start > EPS:
        eps_leg = {**eps_scaling_leg(native, torch, k, mus, nus, fs, gs, a),
                   "plain_marg_l1_mean": float(np.mean([r["marg_l1"] for r in all_r])),
                   "plain_step_wall_s": wall / a.steps}

    # kernel tables (built once per grid and metric, host FP64 then uploaded)
    build_ms = {}
    for n, nt, rad, axial, w, eps, _ in CONV_SHAPES:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kk = native.Kernel(n, n, nt, axial, w, eps, rad)
        torch.cuda.synchronize()
        build_ms[f"{n}x{n}x{nt}{' axial' if axial else ''}, {2 * rad + 1}x{2 * rad + 1}"] = (time.perf_counter() - t0) * 1e3
        del kk
    conv_leg, conv_pots, conv_inst = (None, None, None) if a.conv_batch <= 0 else converged_leg(native, torch, synth, a)
    class_meas = None if class_images is None else class_barycenter(native, torch, class_images, a.bary_iters)
    flow_meas = None if a.flow_steps <= 0 else gradient_flow(native, torch, synth, a.flow_steps)
    bary_meas = None if a.c4_iters <= 0 else barycenter_workloads(native, torch, synth, a.c4_iters)
    serving_meas = None if a.no_serving else serving(native, torch, synth, a, trace)
    serving_conv = None if a.no_serving else serving(native, torch, synth, a, trace_conv, converging=True)
    conv_meas = None if a.no_conv else conv_measurements(native, torch, a.batch, a.conv_reps)
    field_meas = None if a.no_conv else field_measurements(native, torch, a.conv_reps)

    cpu = None
    if not a.no_cpu:
        cpu = cpu_baseline(insts[0], a.cpu_iters, native, torch, k, conv_pots, conv_inst)

    out = {
        "metric": "Sinkhorn iters/sec & solves/sec at 64x64x16 (marg err<=1e-6); p50/p99 latency",
        "value": value,
        "unit": "Sinkhorn iterations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "lines64x64x16-paired OT: w=(1,3,1), eps=0.1, 11x11 window, tol 1e-6, "
                               "max_iter 1000, serving queue", "grid": "64x64x16", "batch": a.batch,
                   "check_every": a.check_every},
        "solves_per_s": len(all_r) / wall,
        "converged_solves_per_s": conv / wall,
        "converged": conv,
        "solves": len(all_r),
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "marg_l1_mean": float(np.mean([r["marg_l1"] for r in all_r])),
        "marg_l1_f64_mean": float(np.mean([r["marg_l1_f64"] for r in all_r])),
        "plain_one_at_a_time_iters_per_s": plain_rate,
        "speedup_vs_plain": (value / plain_rate) if plain_rate else None,
        "step_ms": step_ms,
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernel_build_ms": build_ms,
        "converged_instance": conv_leg,
        "eps_scaling": eps_leg,
        "lift_project": field_meas,
        "class_barycenter": class_meas,
        "gradient_flow": flow_meas,
        "barycenters": bary_meas,
        "serving": serving_meas,
        "serving_converging": serving_conv,
        "se2_conv": {"bound": "mfma", "peak_bf16_tflops": PEAK_BF16_TFLOPS, "peak_f32_tflops": PEAK_F32_TFLOPS,
                     "flops": "2 * batch * nx * ny * ntheta^2 * window", "launches": conv_meas},
    }
    print(json.dumps(out), flush=True)


def serving(native, torch, synth, a, trace, converging=False):
    """Poisson stream of OT requests with mixed grid sizes (32x32x8, 64x64x16, 128x128x16),
    eps and w2, submitted at their arrival times to one queue; latency = completion -
    submission.  Beside it, the same kind of solve one at a time (blocking, dense FP32
    engine) on a stratified sample, extrapolated to the whole trace.  converging: the
    theta-motion trace (eps 0.1, w2 = 3, at most conv_max_iter iterations), whose requests
    reach the tolerance."""
    import numpy as np
    kernels = {}

    def kern(inst):
        g = inst.grid
        key = (g.nx, g.nt, inst.radius, inst.eps, inst.w)
        if key not in kernels:
            kernels[key] = native.Kernel(g.nx, g.ny, g.nt, False, inst.w, inst.eps, inst.radius)
        return kernels[key]

    dev = []
    for r in trace:
        mu = torch.from_numpy(r.inst.mu).cuda()
        nu = torch.from_numpy(r.inst.nu).cuda()
        dev.append((kern(r.inst), mu, nu, torch.empty_like(mu), torch.empty_like(mu)))
    torch.cuda.synchronize()
    max_iter = a.conv_max_iter if converging else a.max_iter
    o = native.opts(tol=a.tol, max_iter=max_iter, check_every=a.check_every, final_check=True, prune=not a.no_prune)
    q = native.SolveQueue(hbm_budget_bytes=int(a.budget_gb * (1 << 30)), max_slots=a.slots)
    tickets = []
    t0 = time.perf_counter()
    for r, (k, mu, nu, f, g) in zip(trace, dev):
        dt = r.arrival_s - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(q.submit_ot(k, mu, nu, o, f, g))
    reps = [q.wait(t) for t in tickets]
    wall = time.perf_counter() - t0
    lat = np.array([q.times(t)[2] - q.times(t)[0] for t in tickets])
    st = q.stats()
    q.close()
    iters = sum(r["iters"] for r in reps)
    conv = sum(1 for r in reps if r["status"] == native.SE2_CONVERGED)
    # one at a time: plain FP32 engine, blocking, a few requests of each grid size
    o_plain = native.opts(tol=a.tol, max_iter=max_iter, check_every=a.check_every, final_check=True, prune=False)
    by_size = {}
    for i, r in enumerate(trace):
        by_size.setdefault(r.inst.grid.nx, []).append(i)
    per_size = {}
    for n, idx in sorted(by_size.items()):
        ts = []
        for i in idx[:a.plain_sample]:
            k, mu, nu, f, g = dev[i]
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            native.se2_sinkhorn(k, mu, nu, o_plain, f, g)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - s0)
        per_size[n] = (float(np.mean(ts)), len(idx))
    plain_total = sum(m * c for m, c in per_size.values())
    workload = ("serving trace, converging: theta-motion pairs on 64x64x16 r5, 128x128x16 r7; "
                f"eps 0.1, w = (1, 3, 1); 4-12 segments; tol 1e-6, max_iter {max_iter}" if converging else
                "serving trace: 32x32x8 r4, 64x64x16 r5, 128x128x16 r7; eps in {0.05, 0.1, 0.2}; "
                f"w = (1, 2 or 3, 1); 4-12 segments; tol 1e-6, max_iter {max_iter}")
    lat_conv = np.array([lt for lt, r in zip(lat, reps) if r["status"] == native.SE2_CONVERGED])
    by_grid = {}
    for r, rep in zip(trace, reps):
        c = by_grid.setdefault(str(r.inst.grid.nx), [0, 0])
        c[0] += rep["status"] == native.SE2_CONVERGED
        c[1] += 1
    return {
        "metric": "serving: p50/p99 latency and solves/s, Poisson OT requests of mixed sizes",
        "mode": "serving",
        "requests": len(trace), "rate_per_s": a.conv_rate if converging else a.rate, "wall_s": wall,
        "solves_per_s": len(reps) / wall, "converged_solves_per_s": conv / wall, "converged": conv,
        "iters_per_s": iters / wall,
        "p50_latency_ms": float(np.percentile(lat, 50) * 1e3), "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
        "converged_p50_p99_latency_ms": ([float(np.percentile(lat_conv, 50) * 1e3),
                                          float(np.percentile(lat_conv, 99) * 1e3)] if lat_conv.size else None),
        "marg_l1_max": float(max(r["marg_l1"] for r in reps)),
        "converged_by_grid": {n: {"converged": c[0], "requests": c[1]} for n, c in sorted(by_grid.items())},
        "iters_median": float(np.median([r["iters"] for r in reps])),
        "queue": st, "budget_gb": a.budget_gb, "max_slots": a.slots,
        "plain_one_at_a_time_solves_per_s_est": len(trace) / plain_total if plain_total > 0 else None,
        "plain_seconds_per_solve": {str(n): m for n, (m, c) in per_size.items()},
        "speedup_vs_plain": (len(reps) / wall) / (len(trace) / plain_total) if plain_total > 0 else None,
        "config": {"workload": workload, "seed": 3100 if converging else 3000},
        "data": "synthetic",
    }


def cpu_baseline(inst, iters: int, native=None, torch=None, kernel=None, conv_pots=None, conv_inst=None):
    """FP64 oracle Sinkhorn on this host, a bounded sample of the same workload; with the
    library given, the same solve on the GPU at the same iteration count beside it, and the
    GPU result's errors against the oracle's (plan L1, marginal L1, relative cost).  With the
    converged leg's potentials (the theta-motion instance its first engine solved in the fewest
    iterations, per engine), the oracle runs that instance to marginal L1 1e-6 as well and the
    converged plans are compared."""
    import numpy as np
    import oracle
    logk, cost = oracle.kernel_table(NT, False, W_METRIC, EPS, R)
    if iters <= 0:
        t = time.perf_counter()
        oracle.sinkhorn(logk, inst.mu, inst.nu, 1, -1.0)
        one = time.perf_counter() - t  # 3 convolutions
        iters = max(2, int(15.0 / max(one * 2.0 / 3.0, 1e-3)))
    t = time.perf_counter()
    phi_o, psi_o, it, err_o, _ = oracle.sinkhorn(logk, inst.mu, inst.nu, iters, -1.0)
    dt = time.perf_counter() - t
    out = {"value": it / dt, "unit": "Sinkhorn iterations/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"one 64x64x16 solve, {it} iterations, FP64 log-domain C + OpenMP"}
    if native is not None:
        mu = torch.from_numpy(inst.mu).cuda()
        nu = torch.from_numpy(inst.nu).cuda()
        f, g = torch.empty_like(mu), torch.empty_like(mu)
        rep = native.se2_sinkhorn(kernel, mu, nu, native.opts(tol=-1.0, max_iter=it, check_every=10), f, g)
        phi_g = f.cpu().numpy() / EPS
        psi_g = g.cpu().numpy() / EPS
        c_o = oracle.plan_stats(logk, cost, phi_o, psi_o)[0]
        out["gpu_vs_oracle"] = {
            "iterations": it, "plan_l1": oracle.plan_l1(logk, phi_g, psi_g, phi_o, psi_o),
            "marg_l1_gpu": rep["marg_l1"], "marg_l1_oracle": err_o,
            "marg_l1_diff": abs(rep["marg_l1"] - err_o), "rel_cost_diff": abs(rep["cost"] - c_o) / c_o,
            "engine": "FP32-exp log-domain engine with certified pruning"}
        # the 128x128x16 interpolation at t = 1/2: 2 IBP iterations on the GPU (blocking call)
        # against the oracle's 2 iterations
        from paper_2402_15322_amd import synth
        ci = synth.curves128(0, t=0.5)
        g = ci.grid
        kc = native.Kernel(g.nx, g.ny, g.nt, g.axial, ci.w, ci.eps, ci.radius)
        dev = [torch.from_numpy(m).cuda() for m in ci.mus]
        b = torch.empty_like(dev[0])
        rep = native.se2_barycenter(kc, dev, ci.lambdas, native.opts(tol=-1.0, max_iter=2, check_every=2), b)
        logk_c, _ = oracle.kernel_table(g.nt, g.axial, ci.w, ci.eps, ci.radius)
        bar_o, it_o, err_o, _ = oracle.ibp(logk_c, ci.mus, ci.lambdas, 2, -1.0)
        out["gpu_vs_oracle_curves128"] = {"t": 0.5, "iterations": it_o,
                                          "barycenter_l1": float(np.abs(b.cpu().numpy() - bar_o).sum()),
                                          "marg_l1_diff": abs(rep["marg_l1"] - err_o)}
        # the same 2 IBP iterations on bfloat16 operands (the configured precision of this workload)
        rep = native.se2_barycenter(kc, dev, ci.lambdas, engine_opts(native, "bf16", tol=-1.0, max_iter=2,
                                                                     check_every=2), b)
        out["gpu_vs_oracle_curves128"]["bf16"] = {"barycenter_l1": float(np.abs(b.cpu().numpy() - bar_o).sum()),
                                                  "fallbacks": rep["fallbacks"]}
        # the 256x256x32 field barycenter's 64x64x8 downsample, 4 IBP iterations: exact engine and
        # bfloat16 operands against the oracle (FP32 on the matrix cores needs 16 or 32 orientations)
        fi = synth.fields256(0, n=64, nt=8)
        g = fi.grid
        kf = native.Kernel(g.nx, g.ny, g.nt, g.axial, fi.w, fi.eps, fi.radius)
        devf = [torch.from_numpy(m).cuda() for m in fi.mus]
        bf = torch.empty_like(devf[0])
        logk_f, _ = oracle.kernel_table(g.nt, g.axial, fi.w, fi.eps, fi.radius)
        bar_f, it_f, err_f, _ = oracle.ibp(logk_f, fi.mus, fi.lambdas, 4, -1.0)
        rec = {"iterations": it_f}
        for ename in ("f32", "bf16"):
            rep = native.se2_barycenter(kf, devf, fi.lambdas, engine_opts(native, ename, tol=-1.0, max_iter=4,
                                                                          check_every=4), bf)
            rec[ename] = {"barycenter_l1": float(np.abs(bf.cpu().numpy() - bar_f).sum()),
                          "marg_l1_diff": abs(rep["marg_l1"] - err_f), "fallbacks": rep["fallbacks"]}
        out["gpu_vs_oracle_fields64x64x8"] = rec
    if conv_pots:
        gi = conv_inst.grid
        logk_t, cost_t = oracle.kernel_table(gi.nt, False, conv_inst.w, conv_inst.eps, conv_inst.radius)
        t = time.perf_counter()
        phi_o, psi_o, it_o, err_o, _ = oracle.sinkhorn(logk_t, conv_inst.mu, conv_inst.nu, 3000, 1e-6)
        c_o = oracle.plan_stats(logk_t, cost_t, phi_o, psi_o)[0]
        rec = {"instance": conv_inst.name, "oracle_iters": it_o, "oracle_marg_l1": err_o,
               "oracle_seconds": time.perf_counter() - t, "engines": {}}
        for name, ((f, g),) in conv_pots.items():
            phi, psi = f / conv_inst.eps, g / conv_inst.eps
            m1, m2, c, _ = oracle.marginal_errors(logk_t, cost_t, phi, psi, conv_inst.mu, conv_inst.nu)
            rec["engines"][name] = {"plan_l1": oracle.plan_l1(logk_t, phi, psi, phi_o, psi_o),
                                    "marg_l1_first": m1, "marg_l1_second": m2, "rel_cost_diff": abs(c - c_o) / c_o}
        out["gpu_vs_oracle_converged"] = rec
    return out


def oracle_timing(one_conv_only: bool = False):
    """The FP64 oracle timed on this host's cores for every configuration of the paper's
    workloads, beside the GPU figures: seconds per log-domain convolution, per iteration
    (Sinkhorn: 2 convolutions; IBP with n measures: 2n) and per 1000-iteration solve
    (extrapolated from the iterations timed).  The serving trace is sampled by 8 requests of
    each grid size (first ones of the trace), each timed over 2 iterations and extrapolated
    to 1000 iterations; the trace total is the per-size mean times the requests of that size.
    With one_conv_only (the one-core run) only the convolutions are timed."""
    import numpy as np
    import oracle
    from paper_2402_15322_amd import synth

    def t_conv(logk, x, reps):
        lx = oracle.safe_log(x)
        oracle.conv_log(logk, lx)
        t = time.perf_counter()
        for _ in range(reps):
            oracle.conv_log(logk, lx)
        return (time.perf_counter() - t) / reps

    cfgs = []
    c0 = synth.tiny_ot(0)
    c1 = synth.lines64(0, paired=True)
    c2 = synth.curves128(0, t=0.5)
    c4 = synth.fields256(0, n=64, nt=8)
    for name, inst, kind, iters, reps in (
            ("16x16x8 OT (200 iterations)", c0, "ot", 200, 20),
            ("64x64x16 OT, paired lines", c1, "ot", 3, 3),
            ("128x128x16 interpolation, t = 1/2", c2, "ibp", 1, 1),
            ("64x64x8 axial downsample of the 256x256x32 fields", c4, "ibp", 2, 3)):
        g = inst.grid
        logk, _ = oracle.kernel_table(g.nt, g.axial, inst.w, inst.eps, inst.radius)
        x = inst.mu if kind == "ot" else inst.mus[0]
        rec = {"config": name, "grid": f"{g.nx}x{g.ny}x{g.nt}", "window": f"{2 * inst.radius + 1}x{2 * inst.radius + 1}",
               "s_per_conv": t_conv(logk, x, reps)}
        convs = 2 if kind == "ot" else 2 * len(inst.mus)
        if one_conv_only:
            rec["s_per_iter_from_convs"] = convs * rec["s_per_conv"]
        else:
            t = time.perf_counter()
            if kind == "ot":
                oracle.sinkhorn(logk, inst.mu, inst.nu, iters, -1.0)
            else:
                oracle.ibp(logk, inst.mus, inst.lambdas, iters, -1.0)
            rec["s_per_iter"] = (time.perf_counter() - t) / iters
            rec["iters_timed"] = iters
            rec["solve_iters"] = 200 if name.startswith("16x16x8") else 1000
            rec["s_per_solve"] = rec["s_per_iter"] * rec["solve_iters"]
        cfgs.append(rec)
    out = {"configs": cfgs}
    if not one_conv_only:
        trace = synth.serving_trace(512, 200.0)
        sizes = {}
        for r in trace:
            sizes.setdefault(r.inst.grid.nx, []).append(r)
        per = {}
        total = 0.0
        for n, reqs in sorted(sizes.items()):
            ts = []
            for r in reqs[:8]:
                g = r.inst.grid
                logk, _ = oracle.kernel_table(g.nt, g.axial, r.inst.w, r.inst.eps, r.inst.radius)
                t = time.perf_counter()
                oracle.sinkhorn(logk, r.inst.mu, r.inst.nu, 2, -1.0)
                ts.append((time.perf_counter() - t) / 2 * 1000)
            per[f"{n}x{n}"] = {"requests_in_trace": len(reqs), "sampled": len(ts),
                               "s_per_1000_iter_solve": float(np.mean(ts))}
            total += len(reqs) * float(np.mean(ts))
        out["serving_trace"] = {"per_grid": per, "s_for_all_512_requests": total,
                                "solves_per_s": 512 / total, "note": "extrapolated from 2 timed iterations"}
    return out


if __name__ == "__main__":
    main()
