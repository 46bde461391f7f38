#!/usr/bin/env python3
"""Benchmark of the RSR Stage-2 hot path on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
sample (Philox) -> classify (dominance, LABEL mode) -> evaluate the
unclassified samples (batched BFS) -> gradient counts -> estimate.  Workload:
the 119-node / 295-edge random geometric graph with 1e4 lower + 1e4 upper
reference rows and N = 1e6 samples.  The metric is dominance tests per
second, counting every (sample, reference row) pair once: N * (R_L + R_U)
per step.

Besides the step, the dominant kernel (classification) is timed in COUNT mode,
where every (sample, row) test is evaluated in full, against the vector-ALU
roofline, and the CPU oracle is timed on a bounded sample of the same
workload.  Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz 32-bit vector ops per second.
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK_BYTES = 8e12
# MI355X dense int8 matrix-core peak (AMD's published figure, no sparsity).
MFMA_I8_PEAK_OPS = 5.0e15
# MI355X dense FP4 (and FP6) matrix-core peak, flops.
MFMA_FP4_PEAK_FLOPS = 10.1e15
# HBM bytes per launch of the COUNT-mode classification on the graph2 workload,
# from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a 1 GiB copy
# (profiles/classify_hbm_traffic.md).  Set an entry to None when its kernel
# changes, until the counters are taken again.
COUNT_TRAFFIC_BYTES = {
    "popcount": (50.42 + 0.95) * 2 ** 20,
    "mfma": (434.04 + 0.95) * 2 ** 20,
    "mfma_fp4": (63.48 + 0.95) * 2 ** 20,
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target duration of the CPU-oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", default="auto", choices=["auto", "popcount", "mfma", "mfma_fp4", "persist"],
                    help="classification form of the graph2 step and of the multi-state leg")
    ap.add_argument("--skip-legs", action="store_true",
                    help="only the graph2 step (no scaling / multi-state / batched legs)")
    ap.add_argument("--only-legs", default="", metavar="LIST",
                    help="comma-separated legs (scaling, multi, batched, stage1, global, flow) to "
                         "run alone, without the step; prints their results as one JSON line")
    ap.add_argument("--batched-scale", type=float, default=1.0,
                    help="reference rows of the batched workload, as a fraction of its sizes")
    ap.add_argument("--batched-reps", type=int, default=3)
    ap.add_argument("--batched-n", default="262144,1e6", metavar="LIST",
                    help="samples per job of the batched leg (comma-separated)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 4 times (calibrates the HBM "
                         "byte counters of rocprofv3) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.empty(args.copy_calibration << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB x 4")
        return
    if args.only_legs:
        import paper_2604_17066_amd as R
        ctx = R.Context(0)
        form = {"auto": R.RSR_AUTO, "popcount": R.RSR_POPCOUNT, "mfma": R.RSR_MFMA,
                "mfma_fp4": R.RSR_MFMA_FP4, "persist": R.RSR_PERSIST}[args.form]
        runs = {"scaling": lambda: scaling_leg(ctx, 5), "multi": lambda: multi_leg(ctx, 5, form),
                "batched": lambda: batched_leg(ctx, args.batched_scale, args.batched_reps,
                                               tuple(int(float(v)) for v in args.batched_n.split(","))),
                "stage1": lambda: stage1_leg(ctx, False), "global": lambda: global_leg(ctx),
                "flow": lambda: flow_leg(ctx)}
        print(json.dumps({name: runs[name]() for name in args.only_legs.split(",")}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2604_17066_amd as R
    import workloads as WL

    form = {"auto": R.RSR_AUTO, "popcount": R.RSR_POPCOUNT, "mfma": R.RSR_MFMA,
            "mfma_fp4": R.RSR_MFMA_FP4, "persist": R.RSR_PERSIST}[args.form]
    t0 = time.time()
    cfg = WL.configs.graph2()
    N, n, K = cfg["N"], cfg["n"], cfg["K"]
    R_L, R_U = cfg["lower"].shape[0], cfg["upper"].shape[0]
    log(f"workload built in {time.time() - t0:.1f}s: n={n} R_L={R_L} R_U={R_U} N={N}")

    ctx = R.Context(0)
    model = R.Model(ctx, cfg["p"])
    refs = R.Refs(ctx, n, K, cfg["lower"], cfg["upper"])
    system = R.System(ctx, cfg["graph"])
    buf = R.Buffers(ctx, n, K, N)
    lib = R.lib()
    P = R.api._ptr
    h = ctx.h

    # The step's calls with their arguments marshalled once: the host time
    # between calls is then the library's, not the harness's.
    p_x, p_f, p_Y, p_ne, p_G = P(buf.samples), P(buf.flags), P(buf.Y), P(buf.n_eval), P(buf.G)
    est_c = R._abi.rsr_estimate_t()
    est_ref = ctypes.byref(est_c)
    f_sample, f_classify, f_eval = lib.rsr_sample, lib.rsr_classify, lib.rsr_eval_unknown
    f_grad, f_est = lib.rsr_grad, lib.rsr_estimate
    seed, LABEL, UNKNOWN = cfg["seed"], R.RSR_LABEL, R.RSR_UNKNOWN_ONLY
    mh, rh, sh = model.h, refs.h, system.h

    def step():
        for st in (f_sample(h, mh, seed, 0, 0, N, p_x),
                   f_classify(h, rh, p_x, N, LABEL, form, p_f, None),
                   f_eval(h, sh, p_x, N, p_f, UNKNOWN, p_Y, p_ne),
                   f_grad(h, mh, p_x, p_Y, N, p_G, None),
                   f_est(h, p_f, p_Y, N, est_ref)):
            if st:
                ctx.check(st)
        return est_c

    for _ in range(args.warmup):
        step()
    est = est_c.as_dict()
    log(f"warmup done: P={est['P']:.6f} p_u={est['p_u']:.3e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    est = est_c.as_dict()
    ms_per_step = (t2 - t1) * 1e3 / args.steps
    tests = N * (R_L + R_U)
    value = tests / (ms_per_step * 1e-3)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")

    # Classification kernels timed alone (HIP events on the context stream).
    reps = max(3, min(args.steps, 10))

    def time_classify(mode, f):
        cev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps)]
        ctx.check(lib.rsr_classify(h, refs.h, P(buf.samples), N, mode, f, P(buf.flags), None))
        for i in range(reps):
            cev[i][0].record()
            ctx.check(lib.rsr_classify(h, refs.h, P(buf.samples), N, mode, f, P(buf.flags), None))
            cev[i][1].record()
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in cev]))

    W = model.words
    # Work per test of the contraction: 2 Kpad ops, Kpad = the packed bits
    # rounded up to 64.  The FP4 instruction contracts 128 k at a time, so its
    # issued work is 2 KP4 (bits rounded up to 128); that figure is reported
    # beside the algorithmic one, never as it.
    KP = 64 * ((32 * W + 63) // 64)
    KP4 = 128 * ((32 * W + 127) // 128)
    kern = {}
    for fname, f in (("popcount", R.RSR_POPCOUNT), ("mfma", R.RSR_MFMA),
                     ("mfma_fp4", R.RSR_MFMA_FP4)):
        kern[fname] = {"count_ms": time_classify(R.RSR_COUNT, f),
                       "label_ms": time_classify(R.RSR_LABEL, f)}
    # Popcount form: one 32-bit AND-OR per packed word per test on the vector ALU.
    kern["popcount"]["count_achieved"] = float(tests) * W / (kern["popcount"]["count_ms"] * 1e-3)
    kern["popcount"]["count_frac"] = kern["popcount"]["count_achieved"] / VALU_PEAK_OPS
    # Matrix-core form: 2 KP int8 operations per test (KP = packed bits rounded to 64).
    kern["mfma"]["count_achieved"] = float(tests) * 2 * KP / (kern["mfma"]["count_ms"] * 1e-3)
    kern["mfma"]["count_frac"] = kern["mfma"]["count_achieved"] / MFMA_I8_PEAK_OPS
    # FP4 form: 2 KP flops per test against the dense FP4 peak (the issued
    # instruction work, 2 KP4 per test, is reported separately).
    kern["mfma_fp4"]["count_achieved"] = float(tests) * 2 * KP / (kern["mfma_fp4"]["count_ms"] * 1e-3)
    kern["mfma_fp4"]["count_frac"] = kern["mfma_fp4"]["count_achieved"] / MFMA_FP4_PEAK_FLOPS
    kern["mfma_fp4"]["issued_ops_per_test"] = 2 * KP4
    kern["mfma_fp4"]["issued_frac"] = (float(tests) * 2 * KP4 / (kern["mfma_fp4"]["count_ms"] * 1e-3)
                                       / MFMA_FP4_PEAK_FLOPS)
    for k, v in kern.items():
        log(f"{k}: COUNT {v['count_ms']:.3f} ms ({v['count_frac'] * 100:.1f}% of peak), "
            f"LABEL {v['label_ms']:.3f} ms")
    # LABEL classification of the step's own form, timed alone.
    label_ms = time_classify(R.RSR_LABEL, form)
    peaks = {"popcount": VALU_PEAK_OPS, "mfma": MFMA_I8_PEAK_OPS, "mfma_fp4": MFMA_FP4_PEAK_FLOPS}
    ops_per_test = {"popcount": W, "mfma": 2 * KP, "mfma_fp4": 2 * KP}
    # The roofline kernel is the COUNT-mode classification of the form the step
    # uses; the automatic form classifies in COUNT mode with the FP4 form.
    dom = args.form if args.form != "auto" else "mfma_fp4"
    count_ms = kern[dom]["count_ms"]
    achieved = kern[dom]["count_achieved"]
    # Restore LABEL flags so the buffers hold a consistent pass.
    step()
    torch.cuda.synchronize()

    # The other stages of the step, each timed alone (HIP events on the context
    # stream), with the rate their own bound is stated in.
    def run_sample():
        ctx.check(lib.rsr_sample(h, model.h, cfg["seed"], 0, 0, N, P(buf.samples)))

    def run_eval():
        ctx.check(lib.rsr_eval_unknown(h, system.h, P(buf.samples), N, P(buf.flags),
                                       R.RSR_UNKNOWN_ONLY, P(buf.Y), P(buf.n_eval)))

    def run_grad():
        ctx.check(lib.rsr_grad(h, model.h, P(buf.samples), P(buf.Y), N, P(buf.G), None))

    def run_estimate():
        R.rsr_estimate(ctx, buf.flags, buf.Y, N)

    st_reps = max(5, reps)
    sample_ms = _event_ms(run_sample, st_reps)
    eval_ms = _event_ms(run_eval, st_reps)
    grad_ms = _event_ms(run_grad, st_reps)
    est_ms = _event_ms(run_estimate, st_reps)
    n_eval = int(buf.n_eval.item())
    philox_blocks = N * ((n + 7) // 8)   # one block per eight components of a sample
    step_kernels = {
        # Philox4x32-10: 10 rounds of two 32x32->64-bit products and two
        # three-input XORs per block of eight 16-bit halves (the second block,
        # drawn with probability 2^-16 per threshold, is left out); a compare,
        # a bit insert and a tie test per draw and plane.
        "sample": {"ms": sample_ms, "draws_per_s": N * n / (sample_ms * 1e-3),
                   "philox_blocks_per_s": philox_blocks / (sample_ms * 1e-3),
                   "algorithmic_valu_frac": (philox_blocks * 40 + 3 * N * n * (K - 1))
                   / (sample_ms * 1e-3) / VALU_PEAK_OPS,
                   "write_GBps": 4.0 * W * N / (sample_ms * 1e-3) / 1e9},
        "classify_label": {"ms": label_ms},
        "eval_unknown": {"ms": eval_ms, "evaluated": n_eval,
                         "phi_evals_per_s": n_eval / (eval_ms * 1e-3)},
        # Gradient: every sample's packed words once, plus its flag and Y bytes.
        "grad": {"ms": grad_ms, "read_GBps": (4.0 * W * N + 2.0 * N) / (grad_ms * 1e-3) / 1e9,
                 "hbm_frac": (4.0 * W * N + 2.0 * N) / (grad_ms * 1e-3) / HBM_PEAK_BYTES},
        # Estimate: flags and Y once, then fp64 sums on the host-visible counts.
        "estimate": {"ms": est_ms, "read_GBps": 2.0 * N / (est_ms * 1e-3) / 1e9},
    }
    log("stages: " + ", ".join(f"{k} {v['ms']:.3f} ms" for k, v in step_kernels.items()))

    # Plain Monte Carlo on the GPU (the system function on every sample, no
    # reference states): the method's own baseline, on the same samples.
    Y_plain = torch.empty(N, dtype=torch.uint8, device=ctx.device)
    def run_plain():
        ctx.check(lib.rsr_eval_unknown(h, system.h, P(buf.samples), N, None, R.RSR_ALL,
                                       P(Y_plain), None))
    plain_ms = _event_ms(run_plain, st_reps)
    plain_P = int(Y_plain.sum(dtype=torch.int64).item()) / N
    step_kernels["plain_mc_eval_all"] = {
        "ms": plain_ms, "phi_evals_per_s": N / (plain_ms * 1e-3), "P": plain_P,
        "equals_rsr_P": plain_P == est["P"],
        "rsr_step_speedup": (plain_ms + sample_ms + grad_ms + est_ms) / ms_per_step}
    log(f"plain MC (BFS on every sample): {plain_ms:.3f} ms, P={plain_P:.6f}")

    # The same step as a one-job plan: its kernels captured once into a HIP
    # graph, one graph launch and one synchronisation per step.
    gbuf = R.Buffers(ctx, n, K, N)
    plan = R.Plan(ctx, [{"model": model, "refs": refs, "system": system, "seed": seed, "N": N,
                         "buffers": gbuf}], tune=False)
    for _ in range(args.warmup):
        plan.run()
        g_est = plan.results()[0][0]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        plan.run()
        g_est = plan.results()[0][0]
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t1) * 1e3 / args.steps
    plan.close()
    step_kernels["graph_step"] = {"ms_per_step": graph_ms, "tests_per_s": tests / (graph_ms * 1e-3),
                                  "identical_estimate": g_est["P"] == est["P"] and g_est["n_u"] == est["n_u"]}
    log(f"step as a one-job captured plan: {graph_ms:.3f} ms/step "
        f"(identical estimate: {step_kernels['graph_step']['identical_estimate']})")
    del gbuf

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        # The buffers hold the last pass of the step (same seed every pass).
        est_now = R.rsr_estimate(ctx, buf.flags, buf.Y, N)
        G_now, c_now = R.rsr_grad(ctx, model, buf.samples, buf.Y, N, want_counts=True)
        I_now = R.rsr_importance(ctx, model, buf.samples, buf.Y, N)
        torch.cuda.synchronize()
        cpu, parity = oracle_check(cfg, R_L + R_U, args.cpu_seconds, est_now, c_now.cpu().numpy(),
                                   G_now.cpu().numpy(), I_now.cpu().numpy())
    extra = {}
    if not args.skip_legs:
        extra["scaling_count_mode"] = scaling_leg(
            ctx, reps, None if args.no_cpu_baseline else args.cpu_seconds)
        cpu_s = None if args.no_cpu_baseline else args.cpu_seconds
        extra["multi_state"] = multi_leg(ctx, reps, form, cpu_s)
        extra["batched_vs_plain"] = batched_leg(ctx, args.batched_scale, args.batched_reps,
                                                tuple(int(float(v)) for v in args.batched_n.split(",")),
                                                cpu_s)
        extra["stage1"] = stage1_leg(ctx, not args.no_cpu_baseline)
        extra["global_connectivity"] = global_leg(ctx)
        extra["max_flow"] = flow_leg(ctx)

    out = {
        "metric": "dominance tests/s (samples x reference states), whole Stage-2 step",
        "value": value,
        "unit": "tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+fp4",
        "data": "synthetic",
        "config": {
            "workload": "graph2: seeded 119-node / 295-edge random geometric graph, s-t "
                        "connectivity, p_fail ~ U[0.01,0.20], 1e4 lower + 1e4 upper reference "
                        "rows, N = 1e6 Philox samples; step = sample + classify (LABEL) + "
                        "evaluate unknowns + gradient + estimate",
            "n": n, "K": K, "R_L": R_L, "R_U": R_U, "N": N, "form": args.form,
            "P": est["P"], "p_u": est["p_u"], "se": est["se"],
        },
        "roofline": {
            "kernel": f"rsr_classify {dom} form, COUNT mode (every test in full), same workload",
            "bound": "alu" if dom == "popcount" else "mfma",
            "achieved": achieved / 1e12,
            "peak": peaks[dom] / 1e12,
            "unit": "TFLOP/s" if dom == "mfma_fp4" else "TOP/s",
            "frac": achieved / peaks[dom],
            "traffic": COUNT_TRAFFIC_BYTES.get(dom),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE)",
            "algorithmic_bytes": 4.0 * W * N + (R_L + R_U) * 4.0 * W + N,
            "ops_per_test": ops_per_test[dom],
            "issued_ops_per_test": 2 * KP4 if dom == "mfma_fp4" else ops_per_test[dom],
            "kernel_ms": count_ms,
        },
        "classify_forms": kern,
        "step_kernels": step_kernels,
        "label_classify": {
            "kernel_ms": label_ms,
            "nominal_tests_per_s": tests / (label_ms * 1e-3),
            "multiple_of_exhaustive_roofline": (tests / (label_ms * 1e-3)) / (VALU_PEAK_OPS / W),
        },
        "cpu_baseline": cpu,
        "parity": parity,
        **extra,
    }
    print(json.dumps(out), flush=True)


def _event_ms(fn, reps):
    import numpy as np
    import torch
    fn()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs]))


def scaling_leg(ctx, reps, cpu_seconds=None):
    """Kernel-only workload (n = 295, 1e5 + 1e5 Bernoulli rows, N = 1e6), every
    classification form in COUNT mode (every test in full) against its
    roofline, and in LABEL mode (these rows are not a consistent reference
    set, so the cascade does not apply)."""
    import paper_2604_17066_amd as R
    import workloads as WL
    cfg = WL.configs.scaling()
    N, n = cfg["N"], cfg["n"]
    model = R.Model(ctx, cfg["p"])
    refs = R.Refs(ctx, n, 2, cfg["lower"], cfg["upper"])
    xs = R.rsr_sample(ctx, model, cfg["seed"], 0, 0, N)
    flags = R.rsr_classify(ctx, refs, xs, N)
    tests = float(N) * (refs.R_L + refs.R_U)
    W = model.words
    KP = 64 * ((32 * W + 63) // 64)
    out = {"workload": "n=295, 1e5 upper Bernoulli(0.05) + 1e5 lower Bernoulli(0.9) rows, "
                       "N=1e6, COUNT mode", "tests": tests}
    KP4 = 128 * ((32 * W + 127) // 128)
    for name, form, ops, peak in (("popcount", R.RSR_POPCOUNT, W, VALU_PEAK_OPS),
                                  ("mfma", R.RSR_MFMA, 2 * KP, MFMA_I8_PEAK_OPS),
                                  ("mfma_fp4", R.RSR_MFMA_FP4, 2 * KP, MFMA_FP4_PEAK_FLOPS)):
        ms = _event_ms(lambda: R.rsr_classify(ctx, refs, xs, N, R.RSR_COUNT, form, flags=flags),
                       reps)
        ach = tests * ops / (ms * 1e-3)
        label_ms = _event_ms(lambda: R.rsr_classify(ctx, refs, xs, N, R.RSR_LABEL, form,
                                                    flags=flags), reps)
        out[name] = {"kernel_ms": ms, "tests_per_s": tests / (ms * 1e-3), "achieved_TOPs": ach / 1e12,
                     "peak_TOPs": peak / 1e12, "frac": ach / peak, "ops_per_test": ops,
                     "label_ms": label_ms}
        if name == "mfma_fp4":
            out[name]["issued_ops_per_test"] = 2 * KP4
            out[name]["issued_frac"] = tests * 2 * KP4 / (ms * 1e-3) / peak
        log(f"scaling COUNT {name}: {ms:.2f} ms, {ach / peak * 100:.1f}% of peak; "
            f"LABEL {label_ms:.2f} ms")
    if cpu_seconds:
        out["cpu_baseline"] = cpu_baseline_scaling(cfg, cpu_seconds)
    return out


def multi_leg(ctx, reps, form=None, cpu_seconds=None):
    """Three-state edges on graph2, bottleneck levels 1 and 2 (5e4 rows per
    level), N = 1e6: P(S >= 1), P(S >= 2), the PMF by differences and the fp32
    gradients, full path per level, classified in `form` (default: the
    automatic form).  With cpu_seconds, also the oracle's baseline on the
    first samples (cpu_baseline_multi)."""
    import paper_2604_17066_amd as R
    form = R.RSR_AUTO if form is None else form
    import workloads as WL
    cfg = WL.configs.multi()
    N, n, K = cfg["N"], cfg["n"], cfg["K"]
    model = R.Model(ctx, cfg["p"])
    buf = R.Buffers(ctx, n, K, N)
    res = {}
    levels = {}
    for k in (1, 2):
        lv = cfg["levels"][k]
        refs = R.Refs(ctx, n, K, lv["lower"], lv["upper"])
        system = R.System(ctx, cfg["graph"], K=K, level=k)
        levels[k] = (refs, system)
    def one_pass():
        ests = {}
        for k, (refs, system) in levels.items():
            ests[k], _ = R.stage2(ctx, model, refs, system, N, cfg["seed"], form=form, buffers=buf)
        return ests
    ests = one_pass()
    import time as _t
    import torch
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    for _ in range(reps):
        ests = one_pass()
    torch.cuda.synchronize()
    ms = (_t.perf_counter() - t0) * 1e3 / reps
    P1, P2 = ests[1]["P"], ests[2]["P"]
    res = {"workload": "graph2 with states {0,1,2}, levels 1 and 2, 5e4 rows per level, N=1e6",
           "form": int(form), "ms_both_levels": ms, "P_ge1": P1, "P_ge2": P2,
           "pmf": [1.0 - P1, P1 - P2, P2], "p_u": [ests[1]["p_u"], ests[2]["p_u"]],
           "tests_per_s": float(N) * sum(r.R_L + r.R_U for r, _ in levels.values()) / (ms * 1e-3)}
    log(f"multi-state: {ms:.2f} ms for both levels, P(S>=1)={P1:.5f} P(S>=2)={P2:.5f}")
    if cpu_seconds:
        res["cpu_baseline"] = cpu_baseline_multi(ctx, cfg, model, levels, buf, form, cpu_seconds)
    return res


def stage1_leg(ctx, with_cpu):
    """Stage 1 on graph2 from empty reference sets (section 3.5): 1e5 samples
    per iteration, 1024 boundary searches per iteration, until p_u < 1e-3 or
    2e4 rows or 100 iterations; plus the boundary search alone on 2^17 start
    samples, and (with_cpu) the oracle's search on 256 of them as its CPU
    baseline."""
    import time as _t
    import torch
    import paper_2604_17066_amd as R
    import workloads as WL
    cfg = WL.configs.graph2(N=1, R_U=10, R_L=10)
    model = R.Model(ctx, cfg["p"])
    system = R.System(ctx, cfg["graph"])
    R.stage1(ctx, model, system, 10_000, 64, 1e-3, 200, 3, 1)   # warm-up
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    lo, up, info = R.stage1(ctx, model, system, 100_000, 1024, 1e-3, 20_000, 100, 5)
    loop_s = _t.perf_counter() - t0
    N = 1 << 17
    xs = R.rsr_sample(ctx, model, 9, 0, 0, N)
    picks = torch.arange(0, N, dtype=torch.int64, device=ctx.device)
    rows, side = R.rsr_boundary_search(ctx, system, xs, N, picks)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(5):
        R.rsr_boundary_search(ctx, system, xs, N, picks, rows=rows, side=side)
    e1.record(st)
    torch.cuda.synchronize()
    search_ms = e0.elapsed_time(e1) / 5
    # The Stage-2 step of the headline workload with these grown rows in place
    # of the structural path / cut rows.
    refs = R.Refs(ctx, cfg["n"], 2, lo, up)
    N2 = 1_000_000
    est2, buf2 = R.stage2(ctx, model, refs, system, N2, 2)
    torch.cuda.synchronize()
    t1 = _t.perf_counter()
    for _ in range(10):
        est2, buf2 = R.stage2(ctx, model, refs, system, N2, 2, buffers=buf2)
    torch.cuda.synchronize()
    grown_ms = (_t.perf_counter() - t1) * 1e3 / 10
    out = {"workload": "graph2 (295 edges) from empty reference sets; 1e5 samples and 1024 searches "
                       "per iteration; stop at p_u < 1e-3, 2e4 rows or 100 iterations",
           "loop_s": loop_s, **info, "rows": int(info["R_L"] + info["R_U"]),
           "boundary_searches_per_s": N / (search_ms * 1e-3), "boundary_search_ms_2e17": search_ms,
           "stage2_step_grown_rows": {"ms": grown_ms, "N": N2, "P": est2["P"], "p_u": est2["p_u"],
                                      "nominal_tests_per_s": N2 * (len(lo) + len(up))
                                      / (grown_ms * 1e-3)}}
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline_boundary(cfg, 9, 256)
    log(f"stage 1: {info['iterations']} iterations, {out['rows']} rows, p_u {info['p_u']:.2e}, "
        f"{loop_s:.2f} s; boundary search {out['boundary_searches_per_s']:.3g}/s")
    return out


def global_leg(ctx):
    """Global connectivity (sections 4.2 and 4.5) on graph2 (119 nodes / 295
    edges): Stage 1 from empty reference sets (1e5 samples and 8192 searches
    per iteration, until 1e5 rows or p_u < 1e-5), then Stage 2 with those rows
    on 1e6 samples, for the connected level; and the boundary-search rate of
    both levels."""
    import time as _t
    import torch
    import paper_2604_17066_amd as R
    import workloads as WL
    cfg = WL.configs.global2(N=1)
    model = R.Model(ctx, cfg["p"])
    out = {"workload": "global connectivity of graph2 (119 nodes / 295 edges), p_fail ~ U[0.01, 0.20]"}
    for level in (1, 2):
        system = R.System(ctx, cfg["graph"], level=level, kind="global")
        N = 1 << 16
        xs = R.rsr_sample(ctx, model, 9, 0, 0, N)
        picks = torch.arange(0, N, dtype=torch.int64, device=ctx.device)
        rows, side = R.rsr_boundary_search(ctx, system, xs, N, picks)
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        R.rsr_boundary_search(ctx, system, xs, N, picks, rows=rows, side=side)
        torch.cuda.synchronize()
        out[f"level{level}_boundary_searches_per_s"] = N / (_t.perf_counter() - t0)
    system = R.System(ctx, cfg["graph"], level=1, kind="global")
    R.stage1(ctx, model, system, 10_000, 64, 1e-5, 200, 3, 1)  # warm-up
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    lo, up, info = R.stage1(ctx, model, system, 100_000, 8192, 1e-5, 100_000, 200, 7)
    stage1_s = _t.perf_counter() - t0
    refs = R.Refs(ctx, cfg["n"], 2, lo, up)
    N2 = 1_000_000
    est, buf = R.stage2(ctx, model, refs, system, N2, 99)
    torch.cuda.synchronize()
    t1 = _t.perf_counter()
    reps = 5
    for _ in range(reps):
        est, buf = R.stage2(ctx, model, refs, system, N2, 99, buffers=buf)
    torch.cuda.synchronize()
    stage2_ms = (_t.perf_counter() - t1) * 1e3 / reps
    out.update({"stage1_s": stage1_s, "stage1": info, "rows": len(lo) + len(up),
                "stage2_ms_N1e6": stage2_ms, "P_connected": est["P"], "p_u": est["p_u"],
                "se": est["se"]})
    log(f"global connectivity: stage 1 {info['iterations']} iterations, {len(lo) + len(up)} rows, "
        f"{stage1_s:.2f} s; stage 2 (N=1e6) {stage2_ms:.2f} ms, P={est['P']:.5f}, "
        f"p_u={est['p_u']:.3e}; boundary search {out['level1_boundary_searches_per_s']:.3g}/s "
        f"(level 1), {out['level2_boundary_searches_per_s']:.3g}/s (level 2)")
    return out


def flow_leg(ctx):
    """Single-OD maximum flow on graph2 with edge capacities {0, 1, 2} (the
    three-state model of the multi-state workload), demand d = 2: Stage 1 from
    empty reference sets (the rows are d-minimal path and cut vectors), Stage 2
    on 1e6 samples with them, plain Monte Carlo (max flow on every sample) for
    comparison, and the boundary-search rate."""
    import time as _t
    import torch
    import paper_2604_17066_amd as R
    import workloads as WL
    cfg = WL.configs.multi(N=1, R_per_level=4)
    d = 2
    model = R.Model(ctx, cfg["p"])
    system = R.System(ctx, cfg["graph"], K=3, level=d, kind="flow")
    R.stage1(ctx, model, system, 10_000, 64, 1e-4, 200, 3, 1)  # warm-up
    torch.cuda.synchronize()
    t0 = _t.perf_counter()
    lo, up, info = R.stage1(ctx, model, system, 100_000, 4096, 1e-4, 50_000, 200, 11)
    stage1_s = _t.perf_counter() - t0
    refs = R.Refs(ctx, cfg["n"], 3, lo, up)
    N2 = 1_000_000
    est, buf = R.stage2(ctx, model, refs, system, N2, 99)
    torch.cuda.synchronize()
    reps = 5
    t1 = _t.perf_counter()
    for _ in range(reps):
        est, buf = R.stage2(ctx, model, refs, system, N2, 99, buffers=buf)
    torch.cuda.synchronize()
    stage2_ms = (_t.perf_counter() - t1) * 1e3 / reps
    t2 = _t.perf_counter()
    Y = R.rsr_eval_unknown(ctx, system, buf.samples, N2, None, which=R.RSR_ALL)
    torch.cuda.synchronize()
    plain_ms = (_t.perf_counter() - t2) * 1e3
    plain_P = float(Y.float().mean().item())
    N = 1 << 16
    picks = torch.arange(0, N, dtype=torch.int64, device=ctx.device)
    rows, side = R.rsr_boundary_search(ctx, system, buf.samples, N, picks)
    torch.cuda.synchronize()
    t3 = _t.perf_counter()
    R.rsr_boundary_search(ctx, system, buf.samples, N, picks, rows=rows, side=side)
    torch.cuda.synchronize()
    searches = N / (_t.perf_counter() - t3)
    out = {"workload": "max s-t flow >= 2 on graph2 (119 nodes / 295 edges), capacities {0,1,2} "
                       "with (p0,p1,p2) = reversed Dirichlet(8,2,1)",
           "stage1_s": stage1_s, "stage1": info, "rows": len(lo) + len(up),
           "stage2_ms_N1e6": stage2_ms, "P": est["P"], "p_u": est["p_u"], "se": est["se"],
           "plain_mc_ms_N1e6": plain_ms, "plain_mc_P": plain_P,
           "boundary_searches_per_s": searches}
    log(f"max flow >= {d}: stage 1 {info['iterations']} iterations, {len(lo) + len(up)} rows, "
        f"{stage1_s:.2f} s, p_u {info['p_u']:.2e}; stage 2 (N=1e6) {stage2_ms:.2f} ms, "
        f"P={est['P']:.5f}; plain MC {plain_ms:.2f} ms; boundary search {searches:.3g}/s")
    return out


def batched_leg(ctx, ref_scale, reps, Ns=(1 << 18, 1_000_000), cpu_seconds=None):
    """64 hazard scenarios x 8 graphs = 512 jobs, at N = 2^18 (SE <= 9.8e-4 <
    1e-3 for any P) and at N = 1e6: P_sys and the gradient of every job by the
    batched plan (one graph launch, tuned configurations) against the plain
    form (the library's calls job by job, with a host synchronisation per job
    for its estimate), in the library's default (automatic) form and, for
    reference, in the popcount form.  Plan creation is timed with an empty
    tuning cache and again with the cache it wrote.  With cpu_seconds, also
    the oracle's baseline on the first samples of one job per graph
    (cpu_baseline_batched, against the plan's outputs at the first N)."""
    import tempfile
    import time as _t
    import torch
    import paper_2604_17066_amd as R
    import workloads as WL
    t0 = _t.time()
    cfg = WL.configs.batched(n_scen=64, N=1, ref_scale=ref_scale)
    log(f"batched workload built in {_t.time() - t0:.1f}s")
    systems = []
    for sd in cfg["systems"]:
        systems.append((sd, R.Refs(ctx, sd["n"], 2, sd["lower"], sd["upper"]), R.System(ctx, sd["graph"])))
    models = [R.Model(ctx, jd["p"]) for jd in cfg["jobs"]]
    rows = [r.R_L + r.R_U for _, r, _ in systems]
    out = {"workload": f"64 hazard scenarios x 8 graphs (50-500 nodes, 120-1250 edges), "
                       f"{len(cfg['jobs'])} jobs, reference rows x{ref_scale} of 1e3..2e5 per graph "
                       f"({', '.join(str(r) for r in rows)}); P_sys and gradient per job",
           "ref_rows": rows}
    tmp = tempfile.mkdtemp(prefix="rsr_tune_")
    for N in Ns:
        jobs = []
        for jd, m in zip(cfg["jobs"], models):
            sd, refs, system = systems[jd["system"]]
            jobs.append({"model": m, "refs": refs, "system": system, "seed": jd["seed"], "N": N,
                         "buffers": R.Buffers(ctx, sd["n"], 2, N)})

        def plain(form):
            res = []
            for jb in jobs:
                est, _ = R.stage2(ctx, jb["model"], jb["refs"], jb["system"], N, jb["seed"],
                                  form=form, buffers=jb["buffers"])
                res.append(est)
            return res

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t = _t.perf_counter()
            for _ in range(reps):
                r = fn()
            torch.cuda.synchronize()
            return (_t.perf_counter() - t) * 1e3 / reps, r

        plain_ms, plain_est = timed(lambda: plain(R.RSR_AUTO))
        pop_ms, _ = timed(lambda: plain(R.RSR_POPCOUNT))
        cache = f"{tmp}/tune_{N}.json"
        t2 = _t.time()
        plan = R.Plan(ctx, jobs, tune=cache)
        create_s = _t.time() - t2
        plan.close()
        t2 = _t.time()
        plan = R.Plan(ctx, jobs, tune=cache)
        create_cached_s = _t.time() - t2

        def run_plan():
            plan.run()
            return plan.results()[0]

        batched_ms, est = timed(run_plan)
        # What the tuner chose per segment (one segment per graph): the
        # cache's entries in the order of the graphs' reference rows.
        with open(cache) as f:
            entries = json.load(f)
        names = {0: "cascade", 1: "popcount per job", 2: "int8 per job", 3: "fp4 per job",
                 4: "persistent cascade"}
        choices = sorted(({"key": k.split("/", 2)[2], "choice": names.get(v["choice"], "?"),
                           "tail": v["tail"], "first": v["first"], "growth": v["growth"],
                           "split": v["split"], "chunks": v.get("chunks", 0),
                           "classify_ms": v["ms"]} for k, v in entries.items()),
                         key=lambda e: e["key"])
        same = all(a["P"] == b["P"] and a["n_u"] == b["n_u"] for a, b in zip(est, plain_est))
        plan.close()
        se = max(e["se"] for e in est)
        total_tests = float(N) * sum(len(cfg["jobs"]) // len(systems) * r for r in rows)
        log(f"batched N={N}: plain (automatic form) {plain_ms:.1f} ms, plain popcount "
            f"{pop_ms:.1f} ms, plan {batched_ms:.1f} ms ({plain_ms / batched_ms:.2f}x), "
            f"identical={same}, max SE {se:.2e}, plan creation {create_s:.1f}s "
            f"({create_cached_s:.2f}s from the tuning cache)")
        out[f"N{N}"] = {"plain_ms": plain_ms, "plain_popcount_ms": pop_ms, "batched_ms": batched_ms,
                        "speedup_vs_plain": plain_ms / batched_ms,
                        "speedup_vs_plain_popcount": pop_ms / batched_ms,
                        "plan_create_s": create_s, "plan_create_from_cache_s": create_cached_s,
                        "identical_estimates": same, "max_se": se, "tuned_segments": choices,
                        "nominal_tests_per_s_batched": total_tests / (batched_ms * 1e-3)}
        if cpu_seconds and N == Ns[0]:
            out["cpu_baseline"] = cpu_baseline_batched(cfg, jobs, cpu_seconds)
        del jobs
        torch.cuda.empty_cache()
    return out


def cpu_baseline_boundary(cfg, seed, count):
    """The oracle's componentwise boundary search (one system evaluation per
    single step) from the first `count` samples of the same model and seed as
    the GPU timing, on the host cores."""
    import oracle
    x = oracle.sample(cfg["p"], seed, 0, 0, count)
    t = time.perf_counter()
    oracle.boundary_st(cfg["graph"], x)
    dt = time.perf_counter() - t
    return {"value": count / dt, "unit": "boundary searches/s", "cores": oracle.get_threads(),
            "kind": "oracle", "sample": f"{count} start samples of graph2, {dt:.2f} s"}


def _fit_to_budget(run, seconds, n0, cap):
    """Runs run(n) (returning (time, result)) on growing sample counts from n0
    until one takes at least a quarter of `seconds` or reaches `cap` samples,
    so that fixed per-call costs do not inflate the per-sample time; returns
    (n, time, result) of the last run."""
    n = min(n0, cap)
    t, res = run(n)
    while t < 0.25 * seconds and n < cap:
        n = min(cap, int(n * min(16.0, max(2.0, 0.6 * seconds / max(t, 1e-6)))))
        t, res = run(n)
    return n, t, res


def cpu_baseline_multi(ctx, cfg, model, levels, buf, form, seconds):
    """The oracle's whole hot path (sample, classify, evaluate, estimate,
    gradient) for both levels of the multi-state workload on its first
    samples, sized to about `seconds` (_fit_to_budget); the time of all 1e6
    samples is a linear extrapolation.  The GPU's flags and Y for those samples, at
    each level, are compared with the oracle's."""
    import numpy as np
    import oracle
    import torch
    import paper_2604_17066_amd as R
    cores = oracle.get_threads()

    def run(n_sub):
        t = time.perf_counter()
        x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, n_sub)
        out = {}
        for k in (1, 2):
            lv = cfg["levels"][k]
            fl, _, _ = oracle.classify(lv["lower"], lv["upper"], x, mode=0)
            Y, _ = oracle.eval_unknown(cfg["graph"], x, fl, which=0, level=k)
            oracle.estimate(oracle.counts(fl, Y))
            oracle.grad(cfg["p"], x, Y)
            out[k] = (fl, Y)
        return time.perf_counter() - t, out

    n_sub, t, res = _fit_to_budget(run, seconds, 1024, cfg["N"])
    same = True
    for k, (refs, system) in levels.items():
        R.stage2(ctx, model, refs, system, cfg["N"], cfg["seed"], form=form, buffers=buf)
        torch.cuda.synchronize()
        same = same and np.array_equal(buf.flags[:n_sub].cpu().numpy(), res[k][0]) and \
            np.array_equal(buf.Y[:n_sub].cpu().numpy(), res[k][1])
    full = t * cfg["N"] / n_sub
    log(f"cpu oracle, multi-state: {n_sub} samples x 2 levels in {t:.2f}s on {cores} threads "
        f"(flags and Y equal the GPU's: {same})")
    return {"value": n_sub / t, "unit": "samples/s (both levels, whole hot path)", "cores": cores,
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"first {n_sub} of the {cfg['N']} samples, both levels, sample + classify + "
                      f"evaluate + estimate + gradient, {t:.1f} s; the full workload's time is "
                      f"extrapolated linearly: {full:.0f} s",
            "extrapolated_full_s": full, "gpu_flags_and_Y_equal": bool(same)}


def cpu_baseline_batched(cfg, jobs, seconds):
    """The oracle's whole hot path on the first samples of the first job of
    each graph (one hazard scenario per graph), sized to about `seconds` in
    all (_fit_to_budget per graph); the time of all 512 jobs at each N is
    extrapolated linearly per graph.  The plan's flags and Y for those samples are
    compared with the oracle's."""
    import numpy as np
    import oracle
    import torch
    cores = oracle.get_threads()
    first = {}
    for k, jd in enumerate(cfg["jobs"]):
        first.setdefault(jd["system"], k)
    per_graph = {g: sum(1 for jd in cfg["jobs"] if jd["system"] == g) for g in first}

    def run(g, n_sub):
        sd, jd = cfg["systems"][g], cfg["jobs"][first[g]]
        t = time.perf_counter()
        x = oracle.sample(jd["p"], jd["seed"], 0, 0, n_sub)
        fl, _, _ = oracle.classify(sd["lower"], sd["upper"], x, mode=0)
        Y, _ = oracle.eval_unknown(sd["graph"], x, fl)
        oracle.estimate(oracle.counts(fl, Y))
        oracle.grad(jd["p"], x, Y)
        return time.perf_counter() - t, (fl, Y)

    share = seconds / len(first)
    rate, same, n_used, t_used = {}, True, 0, 0.0
    torch.cuda.synchronize()
    for g in first:
        n_sub, t, (fl, Y) = _fit_to_budget(lambda n: run(g, n), share, 256, jobs[first[g]]["N"])
        rate[g] = t / n_sub
        n_used += n_sub
        t_used += t
        b = jobs[first[g]]["buffers"]
        same = same and np.array_equal(b.flags[:n_sub].cpu().numpy(), fl) and \
            np.array_equal(b.Y[:n_sub].cpu().numpy(), Y)
    full = {f"N{N}": sum(rate[g] * per_graph[g] * N for g in first) for N in (1 << 18, 1_000_000)}
    log(f"cpu oracle, batched: {n_used} samples over {len(first)} graphs in {t_used:.2f}s on "
        f"{cores} threads (flags and Y equal the plan's: {same}); all {len(cfg['jobs'])} jobs "
        f"extrapolated: "
        + ", ".join(f"{k} {v:.0f} s" for k, v in full.items()))
    return {"value": n_used / t_used,
            "unit": f"samples/s (mix of the {len(first)} graphs, whole hot path)",
            "cores": cores, "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"first samples of one hazard scenario per graph ({n_used} in all, about "
                      f"{share:.1f} s per graph), sample + classify + evaluate + estimate + "
                      f"gradient, {t_used:.1f} s; the time of all {len(cfg['jobs'])} jobs is "
                      f"extrapolated linearly per graph",
            "extrapolated_full_s": full, "plan_flags_and_Y_equal": bool(same)}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_check(cfg, R_total, seconds, est, counts, G, I):
    """The oracle as it stands on the whole graph2 workload (1e6 samples: the
    hot path's sample, classify, evaluate, estimate and gradient) on all host
    threads: its time is the CPU baseline, and its counts, P, gradient
    counts, G (fp32 within 1e-5 of fp64) and binary importance I (within
    1e-5 (|G1| + |G0|)) are compared with the GPU step's.  The single-thread
    rate is timed on the first samples of the same workload, sized to about
    `seconds` / 3 by a pilot run."""
    import numpy as np
    import oracle
    cores = oracle.get_threads()
    g = cfg["graph"]
    N = cfg["N"]

    def run(n_sub):
        t = time.perf_counter()
        x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, n_sub)
        fl, _, _ = oracle.classify(cfg["lower"], cfg["upper"], x, mode=0)
        Y, _ = oracle.eval_unknown(g, x, fl)
        cnt = oracle.counts(fl, Y)
        oest = oracle.estimate(cnt)
        c, Gref = oracle.grad(cfg["p"], x, Y)
        return time.perf_counter() - t, cnt, oest, c, Gref

    t_all, cnt, oest, c, Gref = run(N)
    log(f"cpu oracle: {N} samples in {t_all:.2f}s on {cores} threads")
    names = ["n_L", "n_U", "n_u", "n_both", "n_u_up"]
    counts_ok = all(int(cnt[k]) == int(est[nm]) for k, nm in enumerate(names))
    P_ok = bool(oest[3] == est["P"])
    c_ok = bool(np.array_equal(counts.view(np.uint64), c))
    nz = Gref != 0
    G_rel = float(np.max(np.abs(G[nz].astype(np.float64) - Gref[nz]) / np.abs(Gref[nz])))
    G_ok = G_rel <= 1e-5 and bool(np.all(G[~nz] == 0))
    I64 = Gref[:, 1] - Gref[:, 0]
    I_err = np.abs(I.astype(np.float64) - I64)
    I_ok = bool(np.all(I_err <= 1e-5 * (np.abs(Gref[:, 1]) + np.abs(Gref[:, 0]))))
    parity = {"ok": bool(counts_ok and P_ok and c_ok and G_ok and I_ok),
              "what": "oracle on all 1e6 samples of the step: counts, P (bit-exact), gradient "
                      "counts (exact), G (fp32 vs fp64, rel <= 1e-5), binary importance "
                      "(|I32 - I64| <= 1e-5 (|G1| + |G0|))",
              "counts": counts_ok, "P": P_ok, "P_oracle": oest[3], "grad_counts": c_ok,
              "G_max_rel_err": G_rel, "G": G_ok, "importance": I_ok}
    log(f"parity against the oracle: {parity['ok']} (G max rel err {G_rel:.2e})")
    oracle.set_threads(1)
    try:
        pilot_n = 2000
        pilot = run(pilot_n)[0]
        n1 = int(min(N, max(pilot_n, pilot_n * (seconds / 3.0) / max(pilot, 1e-6))))
        t1 = run(n1)[0]
    finally:
        oracle.set_threads(cores)
    log(f"cpu oracle, one thread: {n1} samples in {t1:.2f}s")
    cpu = {"value": N * R_total / t_all, "unit": "tests/s", "cores": cores, "kind": "oracle",
           "sample": f"all {N} samples of the same workload, whole hot path (sample, classify, "
                     f"evaluate, estimate, gradient), {t_all:.1f} s",
           "cpu_model": _cpu_model(),
           "single_thread": {"value": n1 * R_total / t1, "unit": "tests/s", "cores": 1,
                             "sample": f"first {n1} samples of the same workload, whole hot "
                                       f"path, {t1:.1f} s"}}
    return cpu, parity


def cpu_baseline_scaling(cfg, seconds):
    """The oracle's COUNT-mode classification (exact match counts) of the
    kernel-only workload on its first samples, sized to about `seconds` by a
    pilot; the rate over the full 1e6 samples is a linear extrapolation."""
    import oracle
    cores = oracle.get_threads()

    def run(n_sub):
        x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, n_sub)
        t = time.perf_counter()
        oracle.classify(cfg["lower"], cfg["upper"], x, mode=1)
        return time.perf_counter() - t

    R_total = cfg["lower"].shape[0] + cfg["upper"].shape[0]
    pilot_n = 256
    pilot = run(pilot_n)
    n_sub = int(min(cfg["N"], max(pilot_n, pilot_n * seconds / max(pilot, 1e-6))))
    t = run(n_sub)
    log(f"cpu oracle, kernel-only COUNT: {n_sub} samples in {t:.2f}s on {cores} threads")
    return {"value": n_sub * R_total / t, "unit": "tests/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n_sub} of the {cfg['N']} samples, COUNT-mode classification "
                      f"against all {R_total} rows, {t:.1f} s; the full workload's time is "
                      f"extrapolated linearly: {t * cfg['N'] / n_sub:.0f} s",
            "extrapolated_full_s": t * cfg["N"] / n_sub}


if __name__ == "__main__":
    main()
