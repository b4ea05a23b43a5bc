#!/usr/bin/env python3
"""Throughput of the RPY mobility matvec on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cube-15M]

A step is one full matvec over all right-hand sides (tree reused): permute,
near field (P2P + overlap correction), S->M, M->M, M->L, S->L, L->L, target
evaluation (eq. 2.8) and un-permute, over device-resident forces.  The default
workload is the largest single-GPU one: 15,000,000 beads uniform in a cube of
side 2,000 (a = 0.5, eta = 1) with 20 right-hand sides per matvec, eps 1e-6,
timed in the plain FP64 form and the mixed-precision form.  Each timed call
is bracketed by HIP events on the plan's stream; ms_per_step is the median.
After the timed region each form may draw Brownian displacement directions
D^{1/2} z once (rpy_sqrt_matvec, z = the force vectors) when that fits the
time budget, reported under "brownian".  Prints one JSON line with the
metric, the live roofline of the dominant kernel (HIP events around each
phase inside the timed region), the M2L and bead-pass rates, and the FP64 CPU
oracle timed on a bounded sample of the same workload (which also gates the
accuracy).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "beads·matvecs/s at 1e-6 rel-L2 vs FP64 direct; mixed/batched vs FP64 FMM"
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector (and FP64 matrix) peak
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector peak
PEAK_MFMA_FP32_TFLOPS = 157.3  # MI355X dense FP32 matrix-core peak
PEAK_MFMA_FP64_TFLOPS = 78.6   # MI355X dense FP64 matrix-core peak
PEAK_HBM_GBS = 8000.0

WORKLOADS = {"cube-2k": 1, "cube-1M": 2, "blobs-4M": 3, "batched-64": 4, "cube-15M": 5, "sphere-8M": 6}


def progress(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_counts(P, p, nrc):
    """Algorithmic flops per launch of the P2P and M2L kernels, from the
    plan's lists (host arithmetic on exported integers only); nrc is the
    number of right-hand sides one launch carries."""
    ex = P.export()
    boxes = ex["boxes"]
    cnt = boxes[:, 5] - boxes[:, 4]
    uo, ue = ex["lists"]["U"]
    leaves = np.where(boxes[:, 7] < 0)[0]
    src = np.add.reduceat(cnt[ue], uo[:-1]) if len(ue) else np.zeros(len(cnt))
    # reduceat on empty segments returns the element at the offset; mask them
    seg = uo[1:] - uo[:-1]
    src = np.where(seg > 0, src, 0)
    pairs = int(np.sum(cnt[leaves] * src[leaves]))
    vo, _ = ex["lists"]["V"]
    npair_v = int(vo[-1])
    T = (p + 1) * (p + 2) // 2
    # P2P, the measurement's per-pair count: about 16 flops and a reciprocal
    # square root of geometry shared by the right-hand sides, and 12 flops
    # per right-hand side (u += A F + B (d.F) d).
    p2p_flops = pairs * (16 + 12 * nrc)
    # This kernel's own count of the same work: 8 flops for the difference
    # and r^2, 12 for the RPY coefficients, and per right-hand side 18 (d.F,
    # the scaled dyad and the three accumulating multiply-adds).
    p2p_flops_kernel = pairs * (20 + 18 * nrc)
    # M2L (dense): per V pair and density, T x (p+1)^2 complex multiply-adds.
    m2l_flops = npair_v * 4 * nrc * T * (p + 1) ** 2 * 8
    # M2L (rotation): per V pair and density, four real-split rotations of
    # 2 (n+1)^2 multiply-adds per degree n and the z translation with
    # 2 (p-l+1)^2 per order l: 10 S multiply-adds, S = sum_n (n+1)^2
    # (the O(p^2) diagonal phase and scale factors are not counted).
    S = (p + 1) * (p + 2) * (2 * p + 3) // 6
    m2l_rot_flops = npair_v * 4 * nrc * 20 * S
    return {"p2p_pairs": pairs, "v_pairs": npair_v, "p2p_flops": p2p_flops, "p2p_flops_kernel": p2p_flops_kernel,
            "m2l_flops": m2l_flops, "m2l_rot_flops": m2l_rot_flops}


def bead_pass_bytes(n, sort_passes):
    """Algorithmic bytes of the plan's bead passes: 24 per bead for the
    bounding cube, 36 for the keys, 24 per radix pass and 48 for the
    position gather."""
    return n * (24 + 36 + 24 * sort_passes + 48)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def source_sha(kernel_file):
    """Hash of a kernel's source file and the headers every kernel includes."""
    h = hashlib.sha256()
    for f in (kernel_file, "common.h", "fmm.h"):
        h.update(open(os.path.join(ROOT, "paper_1711_02976_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_for(kernel_file, launches_key):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current source of the kernel (and the shared headers); else
    None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(launches_key)
    if not rec:
        return None
    if rec.get("source_sha") != source_sha(kernel_file):
        return None
    return rec.get("bytes_per_launch")


def run(args):
    import torch

    import paper_1711_02976_amd as R
    import workloads as W

    cid = WORKLOADS[args.workload]
    k = args.cpu_targets
    if k <= 0:
        w0 = W.config(cid, scale=1e-3)  # bead and rhs counts of the full workload, cheaply
        n_full, r_full = round(w0.n * 1e3), w0.nrhs
        k = int(min(12000, max(200, 6e9 / (n_full * (1 + 0.25 * r_full)))))
    # a batch samples per system (about k targets in all)
    nsys = len(W.config(cid, scale=1e-3).counts)
    w = W.config(cid, nsample=max(1, k // nsys))
    if args.eps:
        import dataclasses
        w = dataclasses.replace(w, eps=args.eps)
    progress(f"{w.name}: {w.n} beads, {w.nrhs} rhs generated")
    dev = torch.device("cuda:0")
    pos = torch.as_tensor(w.pos, device=dev)
    F = torch.as_tensor(w.forces, device=dev)
    U = torch.empty_like(F)
    counts = w.counts if len(w.counts) > 1 else None

    results = {}
    for prec in args.precisions:
        torch.cuda.synchronize()
        P = R.Plan(pos, w.a, w.eta, w.eps, precision=prec, leaf_size=args.leaf_size, order=args.order,
                   max_depth=w.max_depth, counts=counts, m2l=args.m2l, nrhs=F.shape[0])
        st = P.stats()
        progress(f"{w.name} {prec}: plan {st['plan_ms']:.1f} ms, p={st['order']} s={st['leaf_size']} "
                 f"boxes={st['nbox']} depth={st['depth']}")
        for _ in range(args.warmup):
            P.matvec(F, out=U)
            torch.cuda.synchronize()
            progress(f"{w.name} {prec}: warm-up matvec done")
        torch.cuda.synchronize()
        P.set_timing(True)
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e0, e1 in ev:
            e0.record(stream)
            P.matvec(F, out=U)
            e1.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tm = P.timings()
        calls = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        ms = float(np.median(calls))
        wall_ms = (t1 - t0) * 1e3 / args.steps
        progress(f"{w.name} {prec}: {args.steps} timed matvecs, median {ms:.2f} ms (wall mean {wall_ms:.2f} ms)")
        # one more matvec, outside the timed region, with every phase run
        # alone on the plan stream: isolated per-phase times
        P.set_timing(2)
        P.matvec(F, out=U)
        tms = P.timings()
        P.set_timing(False)
        # Brownian displacement directions D^{1/2} z by the Lanczos recurrence
        # (rpy_sqrt_matvec), z = the standard-normal force vectors; skipped
        # when the iteration cap would take more than about 20 s
        brown = None
        if args.brownian_tol > 0 and ms * args.brownian_iters <= args.brownian_budget_s * 1e3:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = P.sqrt_matvec(F, tol=args.brownian_tol, max_iter=args.brownian_iters)
            torch.cuda.synchronize()
            bms = (time.perf_counter() - t0) * 1e3
            brown = {"tol": args.brownian_tol, "max_iter": args.brownian_iters, "nrhs": w.nrhs, **info,
                     "ms": round(bms, 3), "ms_per_iteration": round(bms / max(info["iterations"], 1), 4)}
            progress(f"{w.name} {prec}: sqrt_matvec {info['iterations']} steps, {bms:.1f} ms, "
                     f"converged={info['converged']}")
        nrc = 4 if w.nrhs >= 4 else (2 if w.nrhs >= 2 else 1)
        alg = algorithmic_counts(P, st["order"], nrc)
        results[prec] = {"stats": st, "ms": ms, "wall_ms": wall_ms, "calls_ms": calls, "timings": tm,
                         "serial": tms, "alg": alg, "brownian": brown,
                         "u": U[:, torch.as_tensor(w.sample, device=dev)].cpu().numpy()}
        # plan memory is released before the next form is planned
        P.free()
        torch.cuda.empty_cache()

    # CPU baseline: the FP64 oracle's direct sum on the sampled targets.
    cpu = None
    errs = {}
    if not args.no_cpu:
        import oracle
        oracle.lib()
        k = len(w.sample)
        # each sampled target summed over every bead of its own system
        bounds = np.concatenate([[0], np.cumsum(w.counts)])
        ref = np.zeros((w.nrhs, k, 3))
        pairs = 0
        t0 = time.perf_counter()
        for s0, s1 in zip(bounds[:-1], bounds[1:]):
            sel = np.where((w.sample >= s0) & (w.sample < s1))[0]
            if len(sel):
                ref[:, sel] = oracle.rpy_direct(w.pos[s0:s1], w.forces[:, s0:s1], w.a, w.eta,
                                                targets=w.sample[sel] - s0)
                pairs += len(sel) * int(s1 - s0)
        tc = time.perf_counter() - t0
        full_pairs = float(np.sum(np.asarray(w.counts, dtype=np.float64) ** 2))
        cpu = {"value": k * w.nrhs / tc, "unit": "beads*matvecs/s", "cores": oracle.max_threads(),
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": f"direct O(N^2) FP64 sum for {k} sampled targets of {w.n} (all sources of the "
                         f"target's system, nrhs={w.nrhs}), {tc:.2f} s; value = targets*rhs/s",
               "pairs_per_s": pairs / tc,
               "full_matvec_s_extrapolated": tc * full_pairs / pairs}
        for prec, r in results.items():
            errs[prec] = oracle.rel_l2(r["u"], ref)

    # Optional: the oracle's FMM (same order, leaf size and W-direct threshold
    # as the GPU plan) on the first --oracle-fmm systems of the workload (all
    # of a single-system workload), on the host's cores.  Not part of the
    # default run (minutes of CPU time).
    fmm_cpu = None
    if args.oracle_fmm > 0:
        import oracle
        oracle.lib()
        st = results[args.precisions[-1]]["stats"]
        bounds = np.concatenate([[0], np.cumsum(w.counts)])[:args.oracle_fmm + 1]
        t0 = time.perf_counter()
        for s0, s1 in zip(bounds[:-1], bounds[1:]):
            oracle.fmm(w.pos[s0:s1], w.forces[:, s0:s1], w.a, w.eta, st["order"], st["leaf_size"], st["w_direct"],
                       max_depth=w.max_depth)
        tf = time.perf_counter() - t0
        nb = int(bounds[-1])
        fmm_cpu = {"value": nb * w.nrhs / tf, "unit": "beads*matvecs/s", "seconds": round(tf, 2),
                   "cores": oracle.max_threads(), "cpu_model": cpu_model(), "kind": "oracle FMM",
                   "sample": f"{len(bounds) - 1} of {len(w.counts)} system(s), {nb} of {w.n} beads, nrhs={w.nrhs}, "
                             f"p={st['order']}, s={st['leaf_size']}, W-direct {st['w_direct']}"}
        progress(f"{w.name}: oracle FMM {tf:.1f} s on {fmm_cpu['cores']} threads")

    # Headline: the fastest form that meets the accuracy gate.
    ok = [p for p in results if (not errs) or errs[p] <= w.eps]
    best = min(ok or list(results), key=lambda p: results[p]["ms"])
    r = results[best]
    value = w.n * w.nrhs / (r["ms"] * 1e-3)
    mixed = best == "mixed"

    def rates(q, is_mixed):
        """Live rates of one form from the HIP events of the timed region:
        P2P flop/s by the measurement's per-pair count (16 flops of geometry
        per launch and 12 per right-hand side), in total, for the launches
        on the matrix cores (16 right-hand sides there plus up to 8 on the
        vector units of the same launch, against the matrix-core peak of the
        precision) and for those on the vector units alone (against the
        vector peak, also by the vector kernel's own count);
        M2L flop/s of the rotation operator (20 S flops per V pair and
        density) against the vector peak (no MFMA instruction is issued), in
        the timed region (where it shares the GPU with the near field) and
        alone (the isolated-phase matvec)."""
        tm = q["timings"]
        steps = max(args.steps, 1)
        L_p2p = tm["launches"]["p2p"] / steps
        t_p2p = tm["ms"]["p2p"] / steps * 1e-3
        pairs, npv = q["alg"]["p2p_pairs"], q["alg"]["v_pairs"]
        p = q["stats"]["order"]
        S = (p + 1) * (p + 2) * (2 * p + 3) // 6
        peak = PEAK_FP32_TFLOPS if is_mixed else PEAK_FP64_TFLOPS
        f_p2p = pairs * (16 * L_p2p + 12 * w.nrhs)
        L_mc = tm.get("p2p_mc_launches", 0) / steps
        t_mc = tm.get("p2p_mc_ms", 0.0) / steps * 1e-3
        rhs_mc = tm.get("p2p_mc_rhs", 0) / steps
        L_vec, t_vec, rhs_vec = L_p2p - L_mc, t_p2p - t_mc, w.nrhs - rhs_mc
        f_mc = pairs * (16 * L_mc + 12 * rhs_mc)
        f_vec = pairs * (16 * L_vec + 12 * rhs_vec)
        f_p2p_kernel = pairs * (20 * L_vec + 18 * rhs_vec)
        peak_mc = PEAK_MFMA_FP32_TFLOPS if is_mixed else PEAK_MFMA_FP64_TFLOPS
        t_m2l = tm["ms"]["m2l"] / steps * 1e-3
        t_m2l_alone = q["serial"]["ms"]["m2l"] * 1e-3 if q.get("serial") else 0.0
        f_m2l = npv * 4 * w.nrhs * 20 * S
        out = {"p2p": {"launches_per_matvec": L_p2p, "ms_per_matvec": round(t_p2p * 1e3, 4),
                       "avg_launch_ms": round(t_p2p * 1e3 / max(L_p2p, 1), 4),
                       "pairs": pairs, "flops_per_matvec": f_p2p,
                       "achieved_tflops": round(f_p2p / t_p2p / 1e12, 3) if t_p2p > 0 else None,
                       "frac": round(f_p2p / t_p2p / 1e12 / peak, 4) if t_p2p > 0 else None,
                       "peak_tflops": peak},
               "p2p_mc": {"launches_per_matvec": L_mc, "rhs_per_matvec": rhs_mc,
                          "ms_per_matvec": round(t_mc * 1e3, 4),
                          "avg_launch_ms": round(t_mc * 1e3 / L_mc, 4) if L_mc else None,
                          "flops_per_matvec": f_mc,
                          "achieved_tflops": round(f_mc / t_mc / 1e12, 3) if t_mc > 0 else None,
                          "frac": round(f_mc / t_mc / 1e12 / peak_mc, 4) if t_mc > 0 else None,
                          "peak_tflops": peak_mc},
               "p2p_vec": {"launches_per_matvec": L_vec, "ms_per_matvec": round(t_vec * 1e3, 4),
                           "avg_launch_ms": round(t_vec * 1e3 / L_vec, 4) if L_vec else None,
                           "flops_per_matvec": f_vec,
                           "achieved_tflops": round(f_vec / t_vec / 1e12, 3) if t_vec > 0 else None,
                           "frac": round(f_vec / t_vec / 1e12 / peak, 4) if t_vec > 0 else None,
                           "kernel_count_tflops": round(f_p2p_kernel / t_vec / 1e12, 3) if t_vec > 0 else None,
                           "peak_tflops": peak},
               "m2l": {"ms_per_matvec": round(t_m2l * 1e3, 4), "v_pairs": npv, "flops_per_matvec": f_m2l,
                       "achieved_tflops": round(f_m2l / t_m2l / 1e12, 3) if t_m2l > 0 else None,
                       "frac": round(f_m2l / t_m2l / 1e12 / peak, 4) if t_m2l > 0 else None,
                       "ms_alone": round(t_m2l_alone * 1e3, 4),
                       "frac_alone": round(f_m2l / t_m2l_alone / 1e12 / peak, 4) if t_m2l_alone > 0 else None,
                       "peak_tflops": peak, "mfma_instructions": 0}}
        st = q["stats"]
        if st.get("bead_pass_ms", 0) > 0:
            b = bead_pass_bytes(w.n, st["sort_passes"])
            gbs = b / (st["bead_pass_ms"] * 1e-3) / 1e9
            out["bead_passes"] = {"ms": round(st["bead_pass_ms"], 4), "bytes": b, "achieved_gbs": round(gbs, 1),
                                  "frac": round(gbs / PEAK_HBM_GBS, 4), "sort_passes": st["sort_passes"]}
        return out

    rr = rates(r, mixed)
    # the dominant kernel: P2P on the matrix cores, P2P on the vector units or M->L
    dom = max(("p2p_mc", "p2p_vec", "m2l"), key=lambda k: rr[k]["ms_per_matvec"])
    d = rr[dom]
    count = "per ordered pair: 16 flops + 1 rsqrt per launch, 12 flops per right-hand side"
    if dom == "p2p_mc":
        launches = max(d["launches_per_matvec"], 1)
        roof = {"bound": "mfma", "kernel": "k_p2p_mfma", "achieved": d["achieved_tflops"], "peak": d["peak_tflops"],
                "unit": "TFLOP/s", "frac": d["frac"],
                "traffic": traffic_for("nearfield.hip", f"p2p_mc:{args.workload}:{best}"),
                "avg_launch_ms": d["avg_launch_ms"], "algorithmic_flops_per_launch": d["flops_per_matvec"] / launches,
                "count": count + f" ({d['rhs_per_matvec'] / launches:g} right-hand sides per launch, "
                                 "16 of them on the matrix cores)"}
    elif dom == "p2p_vec":
        launches = max(d["launches_per_matvec"], 1)
        roof = {"bound": "alu", "kernel": "k_p2p", "achieved": d["achieved_tflops"], "peak": d["peak_tflops"],
                "unit": "TFLOP/s", "frac": d["frac"],
                "traffic": traffic_for("nearfield.hip", f"p2p:{args.workload}:{best}"),
                "avg_launch_ms": d["avg_launch_ms"], "algorithmic_flops_per_launch": d["flops_per_matvec"] / launches,
                "count": count, "kernel_count_achieved": d["kernel_count_tflops"]}
    else:
        roof = {"bound": "alu", "kernel": "k_m2l_rot", "achieved": d["achieved_tflops"], "peak": d["peak_tflops"],
                "unit": "TFLOP/s", "frac": d["frac"],
                "traffic": traffic_for("m2l_rot.hip", f"m2l:{args.workload}:{best}"),
                "algorithmic_flops_per_matvec": d["flops_per_matvec"],
                "count": "per V pair and density: 20 S flops, S = sum_n (n+1)^2"}
    tm = r["timings"]
    phase_ms = {k: v / max(args.steps, 1) for k, v in tm["ms"].items()}
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "beads*matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_beads": w.n, "nrhs": w.nrhs, "a": w.a, "eta": w.eta, "eps": w.eps,
                   "precision": best, "order": r["stats"]["order"], "leaf_size": r["stats"]["leaf_size"],
                   "boxes": r["stats"]["nbox"], "depth": r["stats"]["depth"],
                   "plan_ms": round(r["stats"]["plan_ms"], 2)},
        "timing": "median of per-call HIP-event times on the plan stream",
        "rel_l2_vs_direct": errs.get(best),
        "phases_ms": {k: round(v, 4) for k, v in phase_ms.items()},
        "phases_serial_ms": {k: round(v, 4) for k, v in r["serial"]["ms"].items()},
        "forms": {p: {"ms_per_step": round(q["ms"], 4), "ms_mean_wall": round(q["wall_ms"], 4),
                      "ms_min": round(q["calls_ms"][0], 4), "ms_max": round(q["calls_ms"][-1], 4),
                      "value": w.n * w.nrhs / (q["ms"] * 1e-3), "rel_l2_vs_direct": errs.get(p),
                      "plan_ms": round(q["stats"]["plan_ms"], 2), "order": q["stats"]["order"],
                      "leaf_size": q["stats"]["leaf_size"], "rates": rates(q, p == "mixed"),
                      "brownian": q["brownian"]} for p, q in results.items()},
        "speedup_mixed_vs_fp64": (round(results["fp64"]["ms"] / results["mixed"]["ms"], 3)
                                  if "fp64" in results and "mixed" in results else None),
        "roofline": roof,
        "cpu_baseline": cpu,
        **({"cpu_oracle_fmm": fmm_cpu} if fmm_cpu else {}),
    }
    print(json.dumps(line), flush=True)
    if errs and errs[best] > w.eps:
        print(f"accuracy gate failed: rel-L2 {errs[best]:.3e} > {w.eps:.0e}", file=sys.stderr)
        return 3
    return 0


PMC_KERNELS = {  # rocprofv3 kernel-name pattern -> (phase, precision form, source file)
    r"rpy::k_p2p_mfma<true": ("p2p_mc", "mixed", "nearfield.hip"),
    r"rpy::k_p2p_mfma<false": ("p2p_mc", "fp64", "nearfield.hip"),
    r"rpy::k_p2p<\d+, true>": ("p2p", "mixed", "nearfield.hip"),
    r"rpy::k_p2p<\d+, false>": ("p2p", "fp64", "nearfield.hip"),
    r"rpy::k_m2l_rot<\d+, float": ("m2l", "mixed", "m2l_rot.hip"),
    r"rpy::k_m2l_rot<\d+, double": ("m2l", "fp64", "m2l_rot.hip"),
}


def pmc_summary(args):
    """HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (KiB
    per dispatch), each scaled by what the same counter reads for a plain
    device copy of known size (--copy-probe run); writes
    profiles/pmc_traffic.json keyed by phase:workload:form with the kernel
    source hash, so stale figures are not reported."""
    import csv
    import re

    def load(d):
        out = {}
        for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
            name = re.sub(r"\(.*", "", r["Kernel_Name"]).replace("void ", "").strip()
            out.setdefault((name, r["Counter_Name"]), []).append(float(r["Counter_Value"]))
        return out

    fdir, wdir, cfdir, cwdir = args.pmc_summary
    f, w, cf, cw = load(fdir), load(wdir), load(cfdir), load(cwdir)
    copy_bytes = args.copy_probe * (1 << 20)
    mean = lambda v: sum(v) / len(v)
    kf = copy_bytes / (1024.0 * mean(cf[("__amd_rocclr_copyBuffer", "FETCH_SIZE")]))
    kw = copy_bytes / (1024.0 * mean(cw[("__amd_rocclr_copyBuffer", "WRITE_SIZE")]))
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    for pat, (phase, form, src) in PMC_KERNELS.items():
        # the most dispatched kernel of the pattern
        names = sorted({k[0] for k in f if re.match(pat, k[0])}, key=lambda k: -len(f[(k, "FETCH_SIZE")]))
        if not names:
            continue
        name = names[0]
        if (name, "FETCH_SIZE") not in f or (name, "WRITE_SIZE") not in w:
            continue
        fb = mean(f[(name, "FETCH_SIZE")]) * 1024.0 * kf
        wb = mean(w[(name, "WRITE_SIZE")]) * 1024.0 * kw
        sha = source_sha(src)
        rec[f"{phase}:{args.workload}:{form}"] = {
            "kernel": name, "fetch_bytes": round(fb), "write_bytes": round(wb),
            "bytes_per_launch": round(fb + wb), "fetch_scale": round(kf, 4), "write_scale": round(kw, 4),
            "source_sha": sha}
    json.dump(rec, open(path, "w"), indent=1, sort_keys=True)
    print(json.dumps(rec, indent=1, sort_keys=True))
    return 0


def copy_probe(mib):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 3}))
    return 0


def gemm_probe(cols, p=16):
    """The dense alternative to the rotation M->L as a library GEMM: one
    offset's real-split operator [2T x 2T] (T = (p+1)(p+2)/2) applied to
    `cols` gathered (source, density) columns, through torch.matmul
    (hipBLASLt), in FP32 and in BF16.  Prints the rates (HIP events, median
    of 10 after 3 warm-ups)."""
    import torch
    torch.backends.cuda.matmul.allow_tf32 = False
    k = (p + 1) * (p + 2)
    out = {"gemm_probe": f"[{k}x{k}] x [{k}x{cols}]", "order": p}
    for name, dt in (("fp32", torch.float32), ("bf16", torch.bfloat16)):
        a = torch.randn(k, k, device="cuda:0").to(dt)
        b = torch.randn(k, cols, device="cuda:0").to(dt)
        for _ in range(3):
            c = a @ b
        ts = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            c = a @ b
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = sorted(ts)[len(ts) // 2]
        out[name] = {"ms": round(ms, 4), "tflops": round(2.0 * k * k * cols / (ms * 1e-3) / 1e12, 2)}
        del a, b, c
    print(json.dumps(out))
    return 0


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cube-15M", choices=sorted(WORKLOADS))
    ap.add_argument("--precisions", default="fp64,mixed", help="comma list of forms to time: fp64,mixed")
    ap.add_argument("--leaf-size", type=int, default=0)
    ap.add_argument("--brownian-tol", type=float, default=1e-3,
                    help="after the timed matvecs, one rpy_sqrt_matvec at this tolerance (0: skip)")
    ap.add_argument("--brownian-iters", type=int, default=60, help="iteration cap of that call")
    ap.add_argument("--brownian-budget-s", type=float, default=20.0,
                    help="skip that call when the iteration cap times the matvec time exceeds this many seconds")
    ap.add_argument("--order", type=int, default=0)
    ap.add_argument("--eps", type=float, default=0.0,
                    help="accuracy target in place of the workload's (e.g. 1e-9, the 9-digit setting)")
    ap.add_argument("--cpu-targets", type=int, default=0,
                    help="sampled targets of the oracle's direct sum (CPU baseline and accuracy gate); 0: a "
                         "sample of about 6e9 pair evaluations times right-hand sides, at least 200 targets")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--oracle-fmm", type=int, default=0, metavar="SYSTEMS",
                    help="also time the oracle's FMM (same order and leaf size) on the first SYSTEMS systems")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device three times (calibrates rocprofv3 byte counters)")
    ap.add_argument("--gemm-probe", type=int, default=0, metavar="COLS",
                    help="only time the dense M->L operator of one offset (p = 16) as a library GEMM on COLS "
                         "columns, FP32 and BF16, then exit")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="turn four rocprofv3 --pmc output folders (FETCH_SIZE and WRITE_SIZE of a benchmark run "
                         "and of a --copy-probe run of the size given by --copy-probe) into "
                         "profiles/pmc_traffic.json, then exit")
    ap.add_argument("--m2l", default="auto", choices=["auto", "dense", "rotation"],
                    help="multipole-to-local operator (auto = the library's choice per precision)")
    args = ap.parse_args()
    args.precisions = [p.strip() for p in args.precisions.split(",") if p.strip()]
    if args.pmc_summary:
        return pmc_summary(args)
    if args.copy_probe > 0:
        return copy_probe(args.copy_probe)
    if args.gemm_probe > 0:
        return gemm_probe(args.gemm_probe)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        return 2
    return run(args)


if __name__ == "__main__":
    sys.exit(main())
