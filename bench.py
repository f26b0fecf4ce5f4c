"""Benchmark of the IQP Monte Carlo expectation-value hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input that is
already resident in HBM: the forward estimate (parity bits, phase
contraction, cos / mean / standard error) and the hand-written backward
(gradient of a loss of the estimates), i.e. iqp_expval + iqp_expval_grad.
The MMD workload's step is iqp_mmd_loss_grad (loss and gradient).

Prints ONE JSON line. The metric is phase terms per second, T = l * s * m
(observables x samples x gates) per step divided by the step time; the
headline value is split-BF16 fwd+bwd. Results are checked against the FP64
oracle on sampled observables before the number is printed.

Besides the headline, the default run reports the FP32 path, the sparse-C
form, bitflip circuits, independent sample sets per observable, and the
on-device training step (split-BF16, and with a precision per operator
group), each checked against the oracle (the per-group training step
against the split-BF16 step's loss), plus the oracle's own rate on the host
cores.

The batched workload (64 circuits of uneven size, --workload batch64) runs as
one BatchPlan: a step is the forward and the backward pass over all circuits,
each pass one graph replay with persistent contraction kernels, tiles from
the autotuner. --workload paper_shapes times the paper's benchmark shapes
(context).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload n300|n1000|mmd_n300|batch64|paper_shapes]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "phase terms/s (ops×samples×gates), fwd & fwd+bwd, split-BF16 vs FP32 at tol"
# (dense peak of the kernel's dtype in flop/s, matrix-core flops the form issues
# per phase term). The algorithmic work is one multiply-add, 2 flops, per term
# in every form; split-BF16 issues two BF16 products (hi and lo limb) per term.
PEAK = {"split_bf16": (2.5e15, 4.0), "fp32": (157.3e12, 2.0),
        # two BF16 limbs and one FP8 limb of theta in the forward (the FP8
        # product at twice the BF16 rate: 5 BF16-equivalent flops per term);
        # two INT8 limbs of the backward weights against the dense INT8 peak
        # (5.0 POP/s)
        "split3_bf16_fwd": (2.5e15, 5.0), "split3_bf16_bwd": (5.0e15, 4.0),
        # FP16 limb (2 flops) and FP8 limb (2 flops at twice the rate) of the
        # backward weights: 3 FP16-equivalent flops against the FP16 peak
        "split_bf16_fp8_bwd": (2.5e15, 3.0)}
ALGO_FLOPS_PER_TERM = 2.0
TOL = {"fp32": 1e-5, "split_bf16": 1e-4, "split3_bf16": 1e-4, "split_bf16_fp8": 1e-4,
       "sparse_fp32": 1e-5}


ROOT = os.path.dirname(os.path.abspath(__file__))
# the sources the dense contraction kernels are compiled from
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2501_04776_amd", "csrc", f)
                  for f in ("iqp_kernels.hip", "iqp_device.h")]


def kernel_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def nnz_terms(oracle, w, ops01):
    """Terms the oracle actually evaluates: it skips C_kj = 0, so
    sum_k |J_k| * s."""
    return float(oracle.parity(w.n, ops01, w.gates).sum()) * w.s


def recorded_traffic(workload_name, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 byte-counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE, each scaled by what the
    counter reads for a plain device copy of known size), or None when there is
    none or the kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s.md" % workload_name)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if rec.get("kernel_source_sha256") != kernel_source_sha256() or \
            kernel not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][kernel]
    return k["fetch_bytes"] + k["write_bytes"]


def roofline(T, avg_ms, kernel, traffic, prec="split_bf16"):
    """Roofline of the dominant contraction kernel: algorithmic flops (one
    multiply-add per phase term, T terms per launch) over its average launch
    duration, against the dense matrix-core peak of its dtype; the fraction of
    that peak the form actually issues (its limb products) is reported beside
    it."""
    peak, issued = PEAK[prec]
    t = avg_ms * 1e-3
    achieved = ALGO_FLOPS_PER_TERM * T / t
    unit = "TOP/s" if prec == "split3_bf16_bwd" else "TFLOP/s"  # INT8 products
    return {"bound": "mfma", "kernel": kernel, "achieved": achieved / 1e12,
            "peak": peak / 1e12, "unit": unit, "frac": achieved / peak,
            "traffic": traffic, "traffic_unit": "bytes per launch (HBM read + write)",
            "flops_per_launch": ALGO_FLOPS_PER_TERM * T,
            "flops_per_term": ALGO_FLOPS_PER_TERM,
            "issued_flops_per_term": issued, "issued_frac": issued * T / t / peak,
            "avg_launch_ms": avg_ms}


def make_workload(name):
    import workloads as W
    if name == "n300":
        return W.local_n300()
    if name == "n1000":
        return W.random_n1000()
    if name == "mmd_n300":
        return W.mmd_n300()
    raise SystemExit("unknown workload %s" % name)


class DevWorkload:
    """A workload packed into the library's bit rows and moved to the GPU."""

    def __init__(self, w):
        import torch
        import workloads as W
        from paper_2501_04776_amd import packing

        def rows(r):
            return torch.from_numpy(packing.pack_index_rows(r.ptr, r.idx, w.n)
                                    .view(np.int64)).cuda()

        def dense(b):
            return torch.from_numpy(packing.pack_dense(b).view(np.int64)).cuda()

        self.gens = rows(w.gates)
        self.theta = torch.from_numpy(w.theta).cuda()
        self.ops = rows(w.ops)
        self.samples = dense(w.samples)
        self.data = dense(w.data) if w.data is not None else None
        self.op_weight = torch.from_numpy(w.op_weight).cuda() if w.op_weight is not None else None
        self.ops01 = W.rows_to_dense(w.ops, w.n)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch64",
                    choices=["n300", "n1000", "mmd_n300", "batch64", "paper_shapes"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-split3", action="store_true")
    ap.add_argument("--no-fp8", action="store_true",
                    help="skip the split-BF16 form with FP16 + FP8 backward weights")
    ap.add_argument("--profile-precision", default="split_bf16",
                    choices=["split_bf16", "split3_bf16", "split_bf16_fp8", "fp32"],
                    help="precision of the --profile-pass steps")
    ap.add_argument("--no-bitflip", action="store_true")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-indep", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched workload: keep the default tiles instead of autotuning")
    ap.add_argument("--cpu-sample-ops", type=int, default=0,
                    help="observables in the oracle's timed sample (0 = choose)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="only --steps split-BF16 steps and one plain 256 MiB device copy "
                         "(the reference for hardware byte counters); prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        return main_batch(args)
    if args.workload == "paper_shapes":
        return main_paper_shapes(args)

    import torch
    from paper_2501_04776_amd import api

    t0 = time.time()
    w = make_workload(args.workload)
    dw = DevWorkload(w)
    circ = api.Circuit(w.n, dw.gens, dw.theta)
    T = w.terms
    mmd = args.workload == "mmd_n300"
    log("workload %s: n=%d m=%d l=%d s=%d T=%.4g (setup %.1fs)" % (w.name, w.n, w.m, w.l, w.s, T,
                                                                   time.time() - t0))
    u = torch.from_numpy(np.random.default_rng(7).normal(size=w.l) / w.l).cuda()

    def step(prec, fwd_only=False):
        if mmd:
            return api.iqp_mmd_loss_grad(circ, dw.ops, dw.op_weight, dw.samples, dw.data, True,
                                         not fwd_only, prec)
        mean, se, ph = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=not fwd_only)
        if fwd_only:
            return mean, se
        g = api.iqp_expval_grad(circ, dw.ops, dw.samples, u, ph, prec)
        return mean, se, g

    def timed(prec, fwd_only=False, steps=args.steps, warmup=args.warmup):
        for _ in range(warmup):
            step(prec, fwd_only)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            step(prec, fwd_only)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def kernel_breakdown(prec, steps):
        api.profile_reset()
        api.profile_enable(True)
        for _ in range(steps):
            step(prec)
        torch.cuda.synchronize()
        out = {}
        for name in ("parity", "theta_prep", "phase_fwd", "phase_epilogue", "finalize",
                     "weights", "phase_bwd", "grad_reduce", "mmd"):
            ms, n = api.profile_query(name)
            if n:
                out[name] = {"avg_ms": ms / n, "launches": n, "ms_per_step": ms / steps}
        api.profile_enable(False)
        return out

    if args.profile_pass:
        for _ in range(args.steps):
            step(args.profile_precision)
        torch.cuda.synchronize()
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("profile pass done: %d %s steps, copy of %d bytes" % (args.steps,
                                                                  args.profile_precision,
                                                                  src.numel() * 4))
        return

    result = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
              "data": "synthetic"}

    # --- headline: split-BF16 fwd+bwd -------------------------------------
    ms = timed("split_bf16")
    ms_fwd = timed("split_bf16", fwd_only=True)
    log("split_bf16: fwd+bwd %.3f ms, fwd %.3f ms" % (ms, ms_fwd))
    result["value"] = T / (ms * 1e-3)
    result["unit"] = "terms/s"
    result["ms_per_step"] = ms
    result["fwd_terms_per_s"] = T / (ms_fwd * 1e-3)
    result["fwd_ms"] = ms_fwd

    kb = kernel_breakdown("split_bf16", max(3, min(args.steps, 10)))
    result["kernels"] = kb
    dom = max(("phase_fwd", "phase_bwd"), key=lambda k: kb.get(k, {}).get("avg_ms", 0.0))
    result["roofline"] = roofline(T, kb[dom]["avg_ms"], dom, recorded_traffic(w.name, dom))

    # --- theta in two BF16 limbs and an FP8 one, fixed-point weights on INT8 -
    if not args.no_split3:
        ms3 = timed("split3_bf16")
        ms3f = timed("split3_bf16", fwd_only=True)
        log("split3_bf16: fwd+bwd %.3f ms, fwd %.3f ms" % (ms3, ms3f))
        kb3 = kernel_breakdown("split3_bf16", max(3, min(args.steps, 10)))
        result["split3_bf16"] = {
            "fwd_bwd_terms_per_s": T / (ms3 * 1e-3), "fwd_terms_per_s": T / (ms3f * 1e-3),
            "ms_per_step": ms3, "fwd_ms": ms3f, "kernels": kb3,
            "roofline_fwd": roofline(T, kb3["phase_fwd"]["avg_ms"], "phase_fwd (2 BF16 + 1 FP8 limbs)",
                                     recorded_traffic(w.name, "split3_bf16.phase_fwd"),
                                     "split3_bf16_fwd"),
            "roofline_bwd": roofline(T, kb3["phase_bwd"]["avg_ms"], "phase_bwd (INT8 limbs)",
                                     recorded_traffic(w.name, "split3_bf16.phase_bwd"),
                                     "split3_bf16_bwd")} if not mmd else {
            "fwd_bwd_terms_per_s": T / (ms3 * 1e-3), "ms_per_step": ms3, "kernels": kb3}

    # --- split-BF16 forward, FP16 + FP8 backward weights ----------------------
    if not args.no_fp8:
        ms8 = timed("split_bf16_fp8")
        log("split_bf16_fp8: fwd+bwd %.3f ms" % ms8)
        kb8 = kernel_breakdown("split_bf16_fp8", max(3, min(args.steps, 10)))
        result["split_bf16_fp8"] = {
            "fwd_bwd_terms_per_s": T / (ms8 * 1e-3), "ms_per_step": ms8, "kernels": kb8}
        if not mmd:
            result["split_bf16_fp8"]["roofline_bwd"] = roofline(
                T, kb8["phase_bwd"]["avg_ms"], "phase_bwd (FP16 + FP8 limbs)",
                recorded_traffic(w.name, "split_bf16_fp8.phase_bwd"), "split_bf16_fp8_bwd")

    # --- FP32 path ----------------------------------------------------------
    if not args.no_fp32:
        ms32 = timed("fp32", steps=max(3, args.steps // 4), warmup=2)
        ms32f = timed("fp32", fwd_only=True, steps=max(3, args.steps // 4), warmup=1)
        log("fp32: fwd+bwd %.3f ms, fwd %.3f ms" % (ms32, ms32f))
        result["fp32"] = {"fwd_bwd_terms_per_s": T / (ms32 * 1e-3),
                          "fwd_terms_per_s": T / (ms32f * 1e-3), "ms_per_step": ms32,
                          "fwd_ms": ms32f,
                          "mfma_frac_fwd": 2.0 * T / (ms32f * 1e-3) / PEAK["fp32"][0]}

    # --- sparse-C form (FP32 on the vector units, non-zero entries of C only) -
    import oracle
    pick = np.random.default_rng(11).choice(w.l, size=min(8, w.l), replace=False)
    if not args.no_sparse:
        ms_sp = timed("sparse_fp32", steps=max(3, args.steps // 2), warmup=2)
        ms_spf = timed("sparse_fp32", fwd_only=True, steps=max(3, args.steps // 2), warmup=1)
        dens_pick = np.random.default_rng(12).choice(w.l, size=min(64, w.l), replace=False)
        density = float(oracle.parity(w.n, dw.ops01[dens_pick], w.gates).mean())
        log("sparse_fp32: fwd+bwd %.3f ms, fwd %.3f ms (C density %.4f)" % (ms_sp, ms_spf,
                                                                           density))
        # the sparse contraction kernels alone, against 256 CUs x 64 lanes x
        # 2.4 GHz of 32-bit lane ops. Both read one 16-entry table per 4
        # terms. The backward spends 2.5 lane ops per read (a byte extract,
        # an add and a quarter of the 4 shift-and-mask ops of a 64-bit word):
        # 0.625 per term. The forward spends, per 64 generators x 64 samples,
        # a 35-op bit transpose, 40 ops for its 16 reads and 8 for two folds:
        # 1.3 per term. Both make 0.25 LDS reads per term.
        kb_sp = kernel_breakdown("sparse_fp32", 3)
        nnz = density * T
        valu_peak = 256 * 64 * 2.4e9
        sp_roof = {}
        for fam, ops in (("phase_fwd", 1.3), ("phase_bwd", 0.625)):
            if fam in kb_sp:
                rate = nnz / (kb_sp[fam]["avg_ms"] * 1e-3)
                sp_roof[fam] = {"avg_ms": kb_sp[fam]["avg_ms"], "nnz_terms_per_s": rate,
                                "valu_ops_per_term": ops, "valu_ops_per_s": ops * rate,
                                "peak_valu_ops_per_s": valu_peak,
                                "frac": ops * rate / valu_peak}
        # (the forms these kernels replaced issued 3 and 2 lane ops per term:
        # a per-term extract, mask and add, and a select and an add; the rate
        # in that count is given beside the kernels' own fraction)
        for fam, how, before in (("phase_fwd", "16-entry tables of angle sums per 4 "
                                               "generators, indexed through a 64x64 bit "
                                               "transpose", 3.0),
                                 ("phase_bwd", "16-entry tables of signed S sums per 4 "
                                               "samples", 2.0)):
            if fam in sp_roof:
                r = sp_roof[fam]
                r["method"] = how
                r["lds_reads_per_term"] = 0.25
                r["replaced_form_ops_per_term"] = before
                r["rate_in_replaced_form_ops_per_s_over_peak"] = \
                    before * r["nnz_terms_per_s"] / valu_peak
        result["sparse_fp32"] = {"fwd_bwd_terms_per_s": T / (ms_sp * 1e-3),
                                 "fwd_terms_per_s": T / (ms_spf * 1e-3), "ms_per_step": ms_sp,
                                 "fwd_ms": ms_spf, "c_density": density,
                                 "nnz_terms_per_s_fwd": density * T / (ms_spf * 1e-3),
                                 "kernels": sp_roof, "bound": "alu",
                                 "terms": "dense-equivalent l*s*m; C density sampled on "
                                          "%d observables" % dens_pick.size}

    # --- parity of the timed configuration against the oracle ---------------
    parity = {}
    precs = ["split_bf16"] + ([] if args.no_split3 else ["split3_bf16"]) + \
        ([] if args.no_fp8 else ["split_bf16_fp8"]) + \
        ([] if args.no_fp32 else ["fp32"]) + ([] if args.no_sparse else ["sparse_fp32"])
    for prec in precs:
        if mmd:
            break
        mean, se = step(prec, fwd_only=True)
        up = np.zeros(w.l)
        up[pick] = np.random.default_rng(3).normal(size=pick.size)
        _, _, ph = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=True)
        g = api.iqp_expval_grad(circ, dw.ops, dw.samples, torch.from_numpy(up).cuda(), ph, prec)
        torch.cuda.synchronize()
        om, ose = oracle.expval(w.n, w.gates, w.theta, dw.ops01[pick], w.samples)
        og = oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01[pick], w.samples, up[pick])
        em = float(np.abs(mean.cpu().numpy()[pick] - om).max())
        es = float(np.abs(se.cpu().numpy()[pick] - ose).max())
        ega = float(np.abs(g.cpu().numpy() - og).max())
        eg = ega / max(1.0, np.abs(og).max())
        parity[prec] = {"max_abs_err_mean": em, "max_abs_err_stderr": es,
                        "max_abs_err_grad": ega, "max_rel_err_grad": eg, "tol": TOL[prec],
                        "ok": bool(em < TOL[prec] and es < TOL[prec] and eg < TOL[prec]),
                        "sampled_observables": int(pick.size)}
    result["parity"] = parity

    # --- stochastic bitflip circuits (exact product form, FP64) --------------
    if not mmd and not args.no_bitflip:
        ub = torch.from_numpy(np.random.default_rng(9).normal(size=w.l)).cuda()

        def bf_timed(grad, steps):
            def one():
                if grad:
                    api.iqp_bitflip_expval_grad(circ, dw.ops, ub)
                else:
                    api.iqp_bitflip_expval(circ, dw.ops)
            one()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(steps):
                one()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / steps
        bf_ms = bf_timed(False, max(3, args.steps // 2))
        bfg_ms = bf_timed(True, max(3, args.steps // 2))
        bmean = api.iqp_bitflip_expval(circ, dw.ops).cpu().numpy()[pick]
        ubp = np.zeros(w.l)
        ubp[pick] = np.random.default_rng(4).normal(size=pick.size)
        bg = api.iqp_bitflip_expval_grad(circ, dw.ops, torch.from_numpy(ubp).cuda()).cpu().numpy()
        obm = oracle.bitflip_expval(w.n, w.gates, w.theta, dw.ops01[pick])
        obg = oracle.bitflip_grad(w.n, w.gates, w.theta, dw.ops01[pick], ubp[pick])
        rel_m = float(np.max(np.abs(bmean - obm) / np.maximum(np.abs(obm), 1e-300)))
        rel_g = float(np.abs(bg - obg).max() / max(1e-300, np.abs(obg).max()))
        log("bitflip: expval %.3f ms, expval+grad %.3f ms" % (bf_ms, bfg_ms))
        result["bitflip"] = {"expval_ms": bf_ms, "expval_grad_ms": bfg_ms,
                             "entries_per_s": w.l * w.m / (bf_ms * 1e-3),
                             "entries": "l*m entries of C*Theta per call",
                             "max_rel_err_mean": rel_m, "max_rel_err_grad": rel_g,
                             "ok": bool(rel_m < 1e-10 and rel_g < 1e-9),
                             "sampled_observables": int(pick.size)}

    # --- independent estimates: a sample set per observable ----------------
    if not mmd and not args.no_indep:
        result["indep"] = bench_indep(args, w, dw, circ, pick, T)

    # --- on-device training step (MMD^2 workload shape) ---------------------
    # n = 300 all-local circuit with one parameter per gate, 2000 Bernoulli(0.3)
    # training strings, 2000 operators per bandwidth sigma in {1, 5, 17} and
    # 10000 samples drawn on the device every step, Adam; K steps per graph
    if not args.no_train:
        result["train"] = bench_train(args, w if mmd else None)

    # --- oracle on the host cores -------------------------------------------
    # a bounded sample of the same workload: fwd + bwd for the first k
    # observables over all samples and gates, k sized for ~15 s of CPU time
    if not args.no_cpu_baseline and not mmd:
        def oracle_run(k):
            sel = np.arange(k)
            uu = np.random.default_rng(5).normal(size=k)
            t1 = time.time()
            oracle.expval(w.n, w.gates, w.theta, dw.ops01[sel], w.samples)
            oracle.expval_grad(w.n, w.gates, w.theta, dw.ops01[sel], w.samples, uu)
            return time.time() - t1
        nth = oracle.num_threads()
        k = args.cpu_sample_ops
        if not k:
            k0 = min(w.l, max(nth, 8))
            dt0 = oracle_run(k0)
            k = int(min(w.l, max(k0, round(k0 * 15.0 / max(dt0, 1e-3)))))
            k = max(nth, (k // nth) * nth) if k >= nth else k
        dt = oracle_run(k)
        log("oracle: %d observables in %.2f s on %d threads" % (k, dt, nth))
        result["cpu_baseline"] = {"value": k * w.s * w.m / dt, "unit": "terms/s",
                                  "cores": min(nth, k), "kind": "oracle",
                                  "nnz_terms_per_s": nnz_terms(oracle, w, dw.ops01[:k]) / dt,
                                  "cpu_model": cpu_model(), "wall_s": dt,
                                  "sample": "fwd+bwd of the first %d of %d observables over all "
                                            "%d samples and %d gates (%.1f s); value counts the "
                                            "dense-equivalent l*s*m terms" %
                                            (k, w.l, w.s, w.m, dt)}
    result["config"] = {"workload": w.name, "n_qubits": w.n, "gates": w.m, "observables": w.l,
                        "samples": w.s, "precision": "split_bf16 (hi+lo BF16, FP32 accumulate)",
                        "step": "iqp_mmd_loss_grad" if mmd else "iqp_expval + iqp_expval_grad",
                        "terms_per_step": T}
    print(json.dumps(result), flush=True)


def bench_indep(args, w, dw, circ, pick, T):
    """Independent estimates on the workload's circuit and observables, each
    observable with its own s uniform samples (l s W words drawn on the host
    from a seeded generator); fwd and fwd+bwd timed, 8 sampled observables
    checked against the oracle with their own sample sets."""
    import torch
    import oracle
    import workloads as W
    from paper_2501_04776_amd import api

    words = W.uniform_words(np.random.default_rng(2025), (w.l, w.s), w.n)
    z = torch.from_numpy(words.view(np.int64)).cuda()
    u = torch.from_numpy(np.random.default_rng(9).normal(size=w.l) / w.l).cuda()

    def one(grad):
        _, _, ph = api.iqp_expval_indep(circ, dw.ops, z, phase_save=grad)
        if grad:
            api.iqp_expval_indep_grad(circ, dw.ops, z, u, ph)

    def timed(grad, steps):
        one(grad)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            one(grad)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps
    steps = max(3, args.steps // 2)
    fwd_ms = timed(False, steps)
    ms = timed(True, steps)
    # kernel families: "parity" holds the per-observable bit transposes of the
    # samples (and the C parities), "phase_fwd" / "phase_bwd" the sparse bodies
    api.profile_reset()
    api.profile_enable(True)
    for _ in range(2):
        one(True)
    torch.cuda.synchronize()
    kb = {}
    for fam in ("parity", "phase_fwd", "phase_bwd"):
        tot, n = api.profile_query(fam)
        if n:
            kb[fam] = {"ms_per_step": tot / 2, "launches_per_step": n / 2}
    api.profile_enable(False)
    # parity on sampled observables, each with its own sample set
    up = np.zeros(w.l)
    up[pick] = np.random.default_rng(4).normal(size=pick.size)
    mean, se, ph = api.iqp_expval_indep(circ, dw.ops, z, phase_save=True)
    g = api.iqp_expval_indep_grad(circ, dw.ops, z, torch.from_numpy(up).cuda(), ph)
    torch.cuda.synchronize()
    z01 = np.stack([W.unpack_words(words[k], w.n) for k in pick])
    om, ose = oracle.expval_indep(w.n, w.gates, w.theta, dw.ops01[pick], z01)
    og = oracle.expval_indep_grad(w.n, w.gates, w.theta, dw.ops01[pick], z01, up[pick])
    em = float(np.abs(mean.cpu().numpy()[pick] - om).max())
    es = float(np.abs(se.cpu().numpy()[pick] - ose).max())
    eg = float(np.abs(g.cpu().numpy() - og).max() / max(1.0, np.abs(og).max()))
    tol = 1e-5
    log("indep: fwd %.3f ms, fwd+bwd %.3f ms, mean err %.3g" % (fwd_ms, ms, em))
    return {"fwd_ms": fwd_ms, "ms_per_step": ms, "fwd_terms_per_s": T / (fwd_ms * 1e-3),
            "fwd_bwd_terms_per_s": T / (ms * 1e-3),
            "terms": "dense-equivalent l*s*m with a separate sample set per observable",
            "sample_words_bytes": int(words.nbytes), "kernels": kb,
            "parity": {"max_abs_err_mean": em, "max_abs_err_stderr": es,
                       "max_rel_err_grad": eg, "tol": tol,
                       "ok": bool(em < tol and es < tol and eg < tol),
                       "sampled_observables": int(pick.size)}}


def bench_train(args, w=None):
    import torch
    import oracle
    import workloads as W
    from paper_2501_04776_amd import api, packing

    n, s, N, sigmas, per = 300, 10000, 2000, (1.0, 5.0, 17.0), 2000
    if w is None:
        gates = W.local_gates(n)
        theta = np.random.default_rng(404).normal(0.0, 0.1, size=gates.count)
        data = W.bernoulli_rows(np.random.default_rng(405), N, n, 0.3)
    else:
        gates, theta, data = w.gates, w.theta, w.data
    m = gates.count
    probs = [W.sigma_bit_probability(sg) for sg in sigmas]
    gens = torch.from_numpy(packing.pack_index_rows(gates.ptr, gates.idx, n).view(np.int64)).cuda()
    ddata = torch.from_numpy(packing.pack_dense(data).view(np.int64)).cuda()
    seed = (2025, 4776)
    tr = api.Trainer(n, gens, np.arange(m, dtype=np.int32), m, ddata, [per] * 3, probs, s,
                     precision="split_bf16", optimizer="adam", lr=1e-3, seed=seed)
    params = torch.from_numpy(theta.copy()).cuda()
    K = max(2, args.steps)
    for _ in range(2):
        tr.step(params, n_steps=K)  # warm-up (graph capture on the first call)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    loss = tr.step(params, n_steps=K)
    b.record()
    torch.cuda.synchronize()
    step_ms = a.elapsed_time(b) / K
    t_last = tr.buffers()[2].item() - 1
    z, ops, _ = tr.buffers()
    z01 = packing.unpack(z.cpu().numpy().view(np.uint64), n)
    a01 = packing.unpack(ops.cpu().numpy().view(np.uint64), n)
    exact = bool(np.array_equal(z01, oracle.sample_uniform(s, n, seed, t_last, 0)) and
                 np.array_equal(a01, oracle.sample_bernoulli(n, [per] * 3, probs, seed, t_last,
                                                             1)))
    # the loss and gradient alone on the same draws, for the step's overhead
    circ = api.Circuit(n, gens, params)
    wts = torch.full((3 * per,), 1.0 / (3 * per), dtype=torch.float64, device="cuda")
    zc, oc = z.clone(), ops.clone()
    for _ in range(2):
        api.iqp_mmd_loss_grad(circ, oc, wts, zc, ddata, True, True, "split_bf16")
    torch.cuda.synchronize()
    a.record()
    for _ in range(K):
        api.iqp_mmd_loss_grad(circ, oc, wts, zc, ddata, True, True, "split_bf16")
    b.record()
    torch.cuda.synchronize()
    lg_ms = a.elapsed_time(b) / K
    T = 3.0 * per * s * m
    lo = loss.cpu().numpy()
    log("train: %.3f ms/step (loss+grad alone %.3f ms), draws bit-exact %s, loss %.5g -> %.5g" %
        (step_ms, lg_ms, exact, lo[0], lo[-1]))
    tr.close()
    # the same steps with the precision of each bandwidth group chosen by the
    # plan from the expected density of C: split-BF16 for sigma = 1
    # (operators of weight ~60, a third of C non-zero), the sparse form for
    # sigma = 5 and 17 (weight ~3, and mostly the identity)
    tg = api.Trainer(n, gens, np.arange(m, dtype=np.int32), m, ddata, [per] * 3, probs, s,
                     precision="split_bf16", optimizer="adam", lr=1e-3, seed=seed,
                     group_precision="auto")
    gp = tg.group_precisions()
    pg = torch.from_numpy(theta.copy()).cuda()
    for _ in range(2):
        tg.step(pg, n_steps=K)
    torch.cuda.synchronize()
    pg.copy_(torch.from_numpy(theta.copy()))
    tg.reset(0)
    a.record()
    lg = tg.step(pg, n_steps=K)
    b.record()
    torch.cuda.synchronize()
    group_ms = a.elapsed_time(b) / K
    # the first step's loss and draws are those of the split-BF16 trainer's first step after reset
    tr2 = api.Trainer(n, gens, np.arange(m, dtype=np.int32), m, ddata, [per] * 3, probs, s,
                      precision="split_bf16", optimizer="adam", lr=1e-3, seed=seed)
    p2 = torch.from_numpy(theta.copy()).cuda()
    l2 = tr2.step(p2, n_steps=1)
    torch.cuda.synchronize()
    dl = abs(float(lg[0].item()) - float(l2[0].item()))
    tr2.close()
    tg.close()
    log("train, per-group precision %s: %.3f ms/step (%.2fx), first loss vs split-BF16 %.2g" %
        (gp, group_ms, step_ms / group_ms, dl))
    return {"step_ms": step_ms, "steps_per_s": 1e3 / step_ms, "terms_per_s": T / (step_ms * 1e-3),
            "loss_grad_ms": lg_ms, "overhead_ms": step_ms - lg_ms,
            "draws_bit_exact_vs_oracle": exact, "steps_per_graph": K,
            "group_precision": {"mode": "auto", "precisions": gp, "step_ms": group_ms,
                                "steps_per_s": 1e3 / group_ms,
                                "first_loss_abs_diff_vs_split_bf16": dl},
            "loss_first_last": [float(lo[0]), float(lo[-1])],
            "config": "n=300, m=45150 (one parameter per gate), 3 x 2000 operators ~ P_sigma, "
                      "s=10000 drawn per step, N=2000, split_bf16, Adam lr 1e-3"}


def main_paper_shapes(args):
    """The benchmark shapes of Sec. 4.1 (context: the paper's timings are in a
    figure): n in {100, 1000, 2000, 5000}, m in {1e3, 1e5}, l = s = 1e4,
    generator and observable bits Bernoulli(3/n). Split-BF16 and the sparse
    form, forward and forward + backward, each checked against the oracle on
    4 sampled observables. The JSON value is the split-BF16 fwd+bwd rate over
    all eight shapes together."""
    import torch
    import oracle
    import workloads as W
    from paper_2501_04776_amd import api

    reps, warm = max(1, min(args.steps, 5)), max(1, min(args.warmup, 2))

    def median_ms(fn):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        return float(np.median(ts))

    rows, T_all, t_all = [], 0.0, 0.0
    ok_all = True
    for n in (100, 1000, 2000, 5000):
        for m in (1000, 100000):
            w = W.paper_shape(n, m)
            dw = DevWorkload(w)
            circ = api.Circuit(w.n, dw.gens, dw.theta)
            u = torch.ones(w.l, dtype=torch.float64, device="cuda")
            pick = np.random.default_rng(1).choice(w.l, size=4, replace=False)
            om, _ = oracle.expval(w.n, w.gates, w.theta, dw.ops01[pick], w.samples)
            row = {"n": n, "m": m, "l": w.l, "s": w.s, "terms": w.terms}
            for prec, tol in (("split_bf16", 1e-4), ("sparse_fp32", 1e-5)):
                out = {}

                def fwd():
                    out["m"] = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=True)[0]

                def both():
                    _, _, ph = api.iqp_expval(circ, dw.ops, dw.samples, prec, phase_save=True)
                    api.iqp_expval_grad(circ, dw.ops, dw.samples, u, ph, prec)

                tf, tb = median_ms(fwd), median_ms(both)
                err = float(np.abs(out["m"].cpu().numpy()[pick] - om).max())
                ok_all &= err < tol
                row[prec] = {"fwd_ms": tf, "fwd_bwd_ms": tb, "max_abs_err_mean": err, "tol": tol}
                if prec == "split_bf16":
                    T_all += w.terms
                    t_all += tb
            log("n=%d m=%d: split_bf16 fwd %.3f / fwd+bwd %.3f ms, sparse fwd %.3f / %.3f ms, "
                "errors %.1e / %.1e" % (n, m, row["split_bf16"]["fwd_ms"],
                                       row["split_bf16"]["fwd_bwd_ms"], row["sparse_fp32"]["fwd_ms"],
                                       row["sparse_fp32"]["fwd_bwd_ms"],
                                       row["split_bf16"]["max_abs_err_mean"],
                                       row["sparse_fp32"]["max_abs_err_mean"]))
            rows.append(row)
            del dw, circ, u
            torch.cuda.empty_cache()
    result = {"metric": METRIC, "value": T_all / (t_all * 1e-3), "unit": "terms/s", "n_gpus": 1,
              "steps": reps, "warmup": warm, "ms_per_step": t_all, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
              "parity_ok": bool(ok_all), "shapes": rows,
              "config": {"workload": "paper_shapes_l10000_s10000",
                         "shapes": "n in {100,1000,2000,5000} x m in {1e3,1e5}, Bernoulli(3/n) bits",
                         "step": "the eight shapes' split-BF16 iqp_expval + iqp_expval_grad"}}
    print(json.dumps(result), flush=True)


def main_batch(args):
    """The 64-circuit batched workload: n ~ U{50..2000}, m ~ U{1e3..2e5},
    l ~ U{100..5000}, s = 4096, all circuits in one pass per direction. The
    headline is split-BF16; the three-limb form (split3_bf16) and the FP32
    path run the same step beside it."""
    import torch
    import oracle
    import workloads as W
    from paper_2501_04776_amd import api

    t0 = time.time()
    ws = [W.batch64_circuit(i) for i in range(64)]
    dws = [DevWorkload(w) for w in ws]
    T = float(sum(w.terms for w in ws))
    name = "batch64_s4096_seed505"
    log("workload %s: 64 circuits, T=%.4g terms per pass (setup %.1fs)" % (name, T,
                                                                           time.time() - t0))
    rng = np.random.default_rng(7)
    us = [torch.from_numpy(rng.normal(size=w.l) / w.l).cuda() for w in ws]

    def make_plan(prec):
        plan = api.BatchPlan([(api.Circuit(w.n, d.gens, d.theta), d.ops, d.samples)
                              for w, d in zip(ws, dws)], prec)
        if args.no_tune:
            log("%s: workspace %.2f GB, default tiles %s" % (prec, plan.ws_bytes / 1e9,
                                                             plan.config()))
            return plan
        t1 = time.time()
        plan.expval()
        cfg = plan.tune(us)
        log("%s: workspace %.2f GB, tuned %s in %.1fs" % (prec, plan.ws_bytes / 1e9, cfg,
                                                          time.time() - t1))
        return plan

    def timed(plan, fwd_only=False, steps=args.steps, warmup=args.warmup):
        def one():
            plan.expval()
            if not fwd_only:
                plan.expval_grad(us)
        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            one()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def kernel_times(plan, nprof):
        # with timing on, a pass runs its launches one by one, each bracketed
        # by events on its stream
        api.profile_reset()
        api.profile_enable(True)
        for _ in range(nprof):
            plan.expval()
            plan.expval_grad(us)
        torch.cuda.synchronize()
        kb = {}
        for k in ("parity", "theta_prep", "phase_fwd", "phase_epilogue", "finalize", "weights",
                  "phase_bwd", "grad_reduce"):
            tot, n = api.profile_query(k)
            if n:
                kb[k] = {"avg_ms": tot / n, "launches": n, "ms_per_step": tot / nprof}
        api.profile_enable(False)
        return kb

    # parity: 3 sampled observables of 8 sampled circuits, means and the
    # gradient of a loss that weights only those observables
    pick_c = np.random.default_rng(0).choice(64, size=8, replace=False)
    prng = np.random.default_rng(1)
    sel, upick = {}, []
    for i, w in enumerate(ws):
        u = np.zeros(w.l)
        if i in pick_c:
            sel[i] = prng.choice(w.l, size=3, replace=False)
            u[sel[i]] = prng.normal(size=3)
        upick.append(torch.from_numpy(u).cuda())
    ref = {}
    for i, k in sel.items():
        w, d = ws[i], dws[i]
        om, ose = oracle.expval(w.n, w.gates, w.theta, d.ops01[k], w.samples)
        og = oracle.expval_grad(w.n, w.gates, w.theta, d.ops01[k], w.samples,
                                upick[i].cpu().numpy()[k])
        ref[i] = (om, ose, og)

    def parity(plan, prec):
        plan.expval()
        plan.expval_grad(upick)
        torch.cuda.synchronize()
        e = {"max_abs_err_mean": 0.0, "max_abs_err_stderr": 0.0, "max_abs_err_grad": 0.0,
             "max_rel_err_grad": 0.0}
        for i, k in sel.items():
            om, ose, og = ref[i]
            dg = float(np.abs(plan.grads[i].cpu().numpy() - og).max())
            e["max_abs_err_mean"] = max(e["max_abs_err_mean"],
                                        float(np.abs(plan.means[i].cpu().numpy()[k] - om).max()))
            e["max_abs_err_stderr"] = max(e["max_abs_err_stderr"], float(
                np.abs(plan.stderrs[i].cpu().numpy()[k] - ose).max()))
            e["max_abs_err_grad"] = max(e["max_abs_err_grad"], dg)
            e["max_rel_err_grad"] = max(e["max_rel_err_grad"], dg / max(1.0, np.abs(og).max()))
        tol = TOL[prec]
        ok = (e["max_abs_err_mean"] < tol and e["max_abs_err_stderr"] < tol and
              e["max_rel_err_grad"] < tol)
        return dict(e, tol=tol, ok=bool(ok), sampled="3 observables of 8 circuits",
                    grad_bar="tol * max(1, |g|_inf)")

    plan = make_plan("split_bf16")
    if args.profile_pass:
        prec = args.profile_precision
        if prec != "split_bf16":
            plan.close()
            plan = make_plan(prec)
        for _ in range(args.steps):
            plan.expval()
            plan.expval_grad(us)
        torch.cuda.synchronize()
        src = torch.ones(1 << 26, dtype=torch.float32, device="cuda")  # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("profile pass done: %d %s steps, copy of %d bytes" % (args.steps, prec,
                                                                  src.numel() * 4))
        return

    result = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
              "data": "synthetic"}
    ms = timed(plan)
    ms_fwd = timed(plan, fwd_only=True)
    log("split_bf16 batched: fwd+bwd %.3f ms, fwd %.3f ms" % (ms, ms_fwd))
    result.update({"value": T / (ms * 1e-3), "unit": "terms/s", "ms_per_step": ms,
                   "fwd_terms_per_s": T / (ms_fwd * 1e-3), "fwd_ms": ms_fwd,
                   "tiles": plan.config()})
    kb = kernel_times(plan, max(2, min(args.steps, 4)))
    result["kernels"] = kb
    dom = max(("phase_fwd", "phase_bwd"), key=lambda k: kb[k]["avg_ms"])
    result["roofline"] = roofline(T, kb[dom]["avg_ms"], dom + " (persistent, all 64 circuits)",
                                  recorded_traffic(name, dom))
    par = {"split_bf16": parity(plan, "split_bf16")}
    plan.close()
    del plan

    # theta in two BF16 limbs and an FP8 one, fixed-point weights on the INT8
    # matrix cores
    if not args.no_split3:
        p3 = make_plan("split3_bf16")
        ms3 = timed(p3)
        ms3f = timed(p3, fwd_only=True)
        log("split3_bf16 batched: fwd+bwd %.3f ms, fwd %.3f ms" % (ms3, ms3f))
        kb3 = kernel_times(p3, max(2, min(args.steps, 4)))
        fwd3 = roofline(T, kb3["phase_fwd"]["avg_ms"], "phase_fwd (persistent, 2 BF16 + 1 FP8 limbs)",
                        recorded_traffic(name, "split3_bf16.phase_fwd"), "split3_bf16_fwd")
        bwd3 = roofline(T, kb3["phase_bwd"]["avg_ms"], "phase_bwd (persistent, INT8 limbs)",
                        recorded_traffic(name, "split3_bf16.phase_bwd"), "split3_bf16_bwd")
        result["split3_bf16"] = {"fwd_bwd_terms_per_s": T / (ms3 * 1e-3),
                                 "fwd_terms_per_s": T / (ms3f * 1e-3), "ms_per_step": ms3,
                                 "fwd_ms": ms3f, "tiles": p3.config(), "kernels": kb3,
                                 "roofline_fwd": fwd3, "roofline_bwd": bwd3}
        par["split3_bf16"] = parity(p3, "split3_bf16")
        p3.close()
        del p3

    # split-BF16 forward, FP16 + FP8 backward weights
    if not args.no_fp8:
        p8 = make_plan("split_bf16_fp8")
        ms8 = timed(p8)
        log("split_bf16_fp8 batched: fwd+bwd %.3f ms" % ms8)
        kb8 = kernel_times(p8, max(2, min(args.steps, 4)))
        bwd8 = roofline(T, kb8["phase_bwd"]["avg_ms"], "phase_bwd (persistent, FP16 + FP8 limbs)",
                        recorded_traffic(name, "split_bf16_fp8.phase_bwd"), "split_bf16_fp8_bwd")
        result["split_bf16_fp8"] = {"fwd_bwd_terms_per_s": T / (ms8 * 1e-3), "ms_per_step": ms8,
                                    "tiles": p8.config(), "kernels": kb8, "roofline_bwd": bwd8}
        par["split_bf16_fp8"] = parity(p8, "split_bf16_fp8")
        p8.close()
        del p8

    if not args.no_fp32:
        plan32 = make_plan("fp32")
        ms32 = timed(plan32, steps=max(2, args.steps // 4), warmup=1)
        ms32f = timed(plan32, fwd_only=True, steps=max(2, args.steps // 4), warmup=1)
        log("fp32 batched: fwd+bwd %.3f ms, fwd %.3f ms" % (ms32, ms32f))
        result["fp32"] = {"fwd_bwd_terms_per_s": T / (ms32 * 1e-3),
                          "fwd_terms_per_s": T / (ms32f * 1e-3), "ms_per_step": ms32,
                          "fwd_ms": ms32f, "tiles": plan32.config(),
                          "mfma_frac_fwd": 2.0 * T / (ms32f * 1e-3) / PEAK["fp32"][0]}
        par["fp32"] = parity(plan32, "fp32")
        plan32.close()
        del plan32
    result["parity"] = par

    if not args.no_cpu_baseline:
        # the oracle on a bounded sample: fwd + bwd of whole circuits in order
        # (all their samples and gates; the last one cut to its first
        # observables) until about 15 s of host time
        def oracle_run(w, ops01, k):
            uu = np.random.default_rng(5).normal(size=k)
            t1 = time.time()
            oracle.expval(w.n, w.gates, w.theta, ops01[:k], w.samples)
            oracle.expval_grad(w.n, w.gates, w.theta, ops01[:k], w.samples, uu)
            return time.time() - t1
        nth = oracle.num_threads()
        w0, d0 = ws[0], dws[0]
        k0 = min(w0.l, max(nth, 8))
        rate = k0 * w0.s * w0.m / max(oracle_run(w0, d0.ops01, k0), 1e-3)  # calibration
        budget, spent, terms, nnz, parts, cores = 15.0, 0.0, 0.0, 0.0, [], 1
        for i, (w, d) in enumerate(zip(ws, dws)):
            k = int(min(w.l, (budget - spent) * rate / (w.s * w.m)))
            if k < w.l:
                k = max(min(nth, w.l), (k // nth) * nth)
            dt = oracle_run(w, d.ops01, k)
            spent += dt
            terms += k * w.s * w.m
            nnz += nnz_terms(oracle, w, d.ops01[:k])
            cores = max(cores, min(nth, k))
            rate = terms / spent
            parts.append("%d of %d observables of circuit %d (n=%d, m=%d)" % (k, w.l, i, w.n, w.m))
            if k < w.l or spent >= 0.8 * budget:
                break
        log("oracle: %s in %.2f s on %d threads" % ("; ".join(parts), spent, nth))
        result["cpu_baseline"] = {"value": terms / spent, "unit": "terms/s",
                                  "cores": cores, "kind": "oracle",
                                  "nnz_terms_per_s": nnz / spent,
                                  "cpu_model": cpu_model(), "wall_s": spent,
                                  "sample": "fwd+bwd of %s, each over its 4096 samples and all "
                                            "its gates (%.1f s); value counts the "
                                            "dense-equivalent l*s*m terms" %
                                            ("; ".join(parts), spent)}
    result["config"] = {"workload": name, "circuits": 64, "samples": 4096,
                        "n_qubits": "U{50..2000}", "gates": "U{1e3..2e5}",
                        "observables": "U{100..5000}",
                        "precision": "split_bf16 (hi+lo BF16, FP32 accumulate)",
                        "step": "BatchPlan.expval + BatchPlan.expval_grad (graph replays)",
                        "terms_per_step": T}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
