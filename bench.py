#!/usr/bin/env python3
"""Throughput of the THC-MPO Krylov hot path on one MI355X.

One step = one global Lanczos step (Sec. 2.2) from the current Krylov vector:
the compressed H|v> of Algorithm 1 (all 4N^2 V terms with the prefix reuse of
Sec. 3.2, the 2L kinetic terms of App. D, summed by the pairwise tree of
Fig. 11), the overlaps <v_j|w>, the residual sum-compression and the Ritz
values.  Every step applies H once, so the reported value is H|psi>
applications per second.

Default workload: L = 20 spatial orbitals (40 sites), THC rank N = 80, bond
dimension D = 256, a random normalised real MPS with bonds
min(2^j, 2^(40-j), 256) (seed 0).  The absorb contractions run in BF16x3
(--prec), the QR / SVD factorisations, overlaps and the Lanczos eigensolve
in FP64; --compare-f64 also times the same step with FP64 contractions and
reports the speedup and the Ritz-value difference.  The input sits in device
memory before the timed region starts.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak (vendor figure)
HBM_PEAK_GBS = 8000.0         # MI355X HBM3E peak bandwidth (vendor figure)
# FP64 vector ALU peak: 256 CUs x 4 SIMDs x 16 FP64 FMA lanes x 2 flops x 2.4 GHz
FP64_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# kernel classes whose arithmetic runs on the vector ALUs (the rest on MFMA)
VALU_KERNELS = ("sytrd", "tri_eig")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_FN = {"lq": "k_lq2", "sytrd": "k_sytrd", "tri_eig": "k_tri_eig", "ormtr": "k_ormtr2", "gemm": "k_gemm_mfma"}


def kernel_digest(fn: str):
    """SHA-256 of a kernel's source text (from its signature line to its closing brace)."""
    import hashlib
    path = os.path.join(ROOT, "paper_2409_12708_amd", "csrc", "kernels.hip")
    src = open(path).read().splitlines()
    try:
        i = next(k for k, l in enumerate(src) if f"void {fn}(" in l)
        j = next(k for k in range(i, len(src)) if src[k] == "}")
    except StopIteration:
        return None
    return hashlib.sha256("\n".join(src[i:j + 1]).encode()).hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter runs (profiles/), or None
    when there are none or the kernel's source has changed since they were taken."""
    fn = KERNEL_FN.get(kernel)
    path = os.path.join(ROOT, "profiles", f"traffic_{fn}_{workload}.json")
    if not fn or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != kernel_digest(fn):
        return None
    return int(rec["bytes_per_launch"])


KERNEL_LABEL = {"lq": "k_lq2 (Householder LQ with Q, FP64)", "sytrd": "k_sytrd (tridiagonalisation, FP64)",
                "tri_eig": "k_tri_eig (bisection + inverse iteration, FP64)",
                "ormtr": "k_ormtr2 (eigenvector back-transformation, FP64)", "gemm": "k_gemm_mfma (FP64)"}


def roofline_of(kms, kfl, kby, kn):
    """The dominant kernel class (largest summed device time among those with
    algorithmic flops) against the roof its arithmetic intensity puts it
    under: HBM below the ridge point (FP64 peak / HBM peak), else the FP64
    peak of the unit it computes on.  Inputs per class: summed ms, flops,
    bytes, launches.  The returned dict carries the class under "_class"."""
    dom = max((k for k in kms if kfl[k] > 0), key=lambda k: kms[k])
    sec = kms[dom] * 1e-3
    alu = dom in VALU_KERNELS
    cpeak = FP64_VALU_PEAK_TFLOPS if alu else FP64_MFMA_PEAK_TFLOPS
    intensity = kfl[dom] / kby[dom] if kby[dom] > 0 else float("inf")
    ridge = cpeak * 1e12 / (HBM_PEAK_GBS * 1e9)
    if intensity < ridge:
        achieved, peak, unit, bound = kby[dom] / sec / 1e9, HBM_PEAK_GBS, "GB/s", "hbm"
    else:
        achieved, peak, unit, bound = kfl[dom] / sec / 1e12, cpeak, "TFLOP/s", "alu" if alu else "mfma"
    return {
        "bound": bound,
        "kernel": KERNEL_LABEL.get(dom, dom),
        "achieved": round(achieved, 3),
        "peak": round(peak, 2),
        "unit": unit,
        "frac": round(achieved / peak, 4),
        "traffic": None,
        "algorithmic_bytes_per_launch": int(kby[dom] / max(kn[dom], 1)),
        "intensity_flop_per_byte": round(intensity, 3),
        "ridge_flop_per_byte": round(ridge, 2),
        "achieved_tflops": round(kfl[dom] / sec / 1e12, 3),
        "avg_launch_ms": round(kms[dom] / max(kn[dom], 1), 4),
        "launches": int(kn[dom]),
        "_class": dom,
    }


def cpu_baseline(workload: str, seconds_hint: float = 20.0):
    """Time the FP64 oracle on a bounded sample of the same workload: one
    layer-compression and one add-compression at the full bond dimension,
    extrapolated to the compressions of one H|psi>."""
    import numpy as np

    import synth
    from oracle import hamiltonian as OH

    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover - informational only
        threads = len(os.sched_getaffinity(0))
    w = synth.WORKLOADS[workload]
    L, N, D = w["L"], w["N"], w["D"]
    t, chi, zeta, sites = synth.make_workload(workload)
    t0 = time.perf_counter()
    lay = OH.layer_compress(sites, chi[:, 0], 0, False, D)
    t1 = time.perf_counter()
    OH.add_compress(lay, sites, D)
    t2 = time.perf_counter()
    t_layer, t_add = t1 - t0, t2 - t1
    n_layer = 2 * 2 * N + 2 * 4 * N * N + 2 * 2 * L
    n_add = 4 * N * N + 2 * L - 1
    per_h = n_layer * t_layer + n_add * t_add
    return {
        "value": 1.0 / per_h,
        "unit": "H|psi>/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"one layer-compression ({t_layer:.2f} s) and one add-compression ({t_add:.2f} s) of the "
                   f"{workload} MPS at D={D}, FP64 NumPy/LAPACK, extrapolated to the {n_layer} layer- and "
                   f"{n_add} add-compressions of one H|psi>"),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="L20_N80_D256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--prec", default="bf16x3", choices=["f64", "f32", "bf16x3"],
                    help="contraction precision of the absorb products (factorisations stay FP64)")
    ap.add_argument("--compare-f64", action="store_true",
                    help="also time the step with FP64 contractions (doubles the run time)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}, WORLD_SIZE={world}): the THC-MPO path of "
              f"this library is a single-GPU build; no multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("THCK_PROGRESS", "1")  # the library reports finished compression batches on stderr
    import numpy as np
    import torch

    import synth
    import paper_2409_12708_amd as thck

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    w = synth.WORKLOADS[args.workload]
    L, N, D = w["L"], w["N"], w["D"]
    t, chi, zeta, sites = synth.make_workload(args.workload)
    ctx = thck.Context(t, chi, zeta)
    psi = thck.DeviceMPS.from_sites(sites)
    torch.cuda.synchronize()
    log(f"[bench] workload {args.workload}: L={L} N={N} D={D}, warmup {args.warmup}, steps {args.steps}")

    def run(prec):
        K = args.warmup + args.steps
        kr = thck.Krylov(ctx, psi, K, D=D, flags=thck.FLAG_TIME_KERNELS, prec=prec)
        for s in range(args.warmup):
            st = thck.ThcStats()
            t0 = time.perf_counter()
            kr.step(st)
            log(f"[bench] {prec} warmup step {s}: {time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        stats = []
        ritz = None
        t0 = time.perf_counter()
        for s in range(args.steps):
            st = thck.ThcStats()
            ritz, _, beta = kr.step(st)
            stats.append(st)
            log(f"[bench] {prec} step {s}: {time.perf_counter() - t0:.1f} s elapsed, lowest Ritz value {ritz[0]:.10f}, "
                f"beta {beta:.3e}, compressions {st.n_compressions}, max discarded weight "
                f"{st.discarded_weight_max:.3e}")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kr.close()
        return elapsed, stats, ritz

    elapsed, stats, ritz = run(args.prec)
    f64 = None
    if args.compare_f64 and args.prec != "f64":
        e64, _, r64 = run("f64")
        f64 = {"value": args.steps / e64, "ms_per_step": e64 / args.steps * 1e3, "lowest_ritz": float(r64[0]),
               "speedup_of_mixed": e64 / elapsed,
               "lowest_ritz_rel_diff": abs(float(ritz[0]) - float(r64[0])) / abs(float(r64[0]))}
        log(f"[bench] f64 contractions: {e64:.1f} s per step; mixed speedup {e64 / elapsed:.3f}x")

    # per-kernel device time inside the timed region (HIP events on the call's stream)
    names = thck.ThcStats.KERNELS
    kms = {k: sum(st.kernel_ms[i] for st in stats) for i, k in enumerate(names)}
    kfl = {k: sum(st.kernel_flops[i] for st in stats) for i, k in enumerate(names)}
    kn = {k: sum(st.kernel_launches[i] for st in stats) for i, k in enumerate(names)}
    kby = {k: sum(st.kernel_bytes[i] for st in stats) for i, k in enumerate(names)}
    for k in names:
        if kn[k]:
            sec = kms[k] * 1e-3
            rate = kfl[k] / sec / 1e12 if sec > 0 else 0.0
            bw = kby[k] / sec / 1e9 if sec > 0 else 0.0
            log(f"[bench] {k:8s} launches {kn[k]:7d}  device {sec:8.2f} s  "
                f"avg {kms[k] / kn[k]:8.3f} ms  {rate:6.2f} TFLOP/s  {bw:7.1f} GB/s")
    roofline = roofline_of(kms, kfl, kby, kn)
    roofline["traffic"] = measured_traffic(roofline.pop("_class"), args.workload)
    flops_model = sum(st.flops_model for st in stats)
    n_comp = sum(st.n_compressions for st in stats)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(args.workload)
        log(f"[bench] cpu baseline: {cpu['value']:.3e} H|psi>/s ({cpu['sample']})")

    line = {
        "metric": "THC H|\u03c8\u27e9 applications/sec (L=20, D=256) + fraction of MFMA peak, mixed vs FP64",
        "value": args.steps / elapsed,
        "unit": "H|psi>/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "f64" else f"f64+{args.prec}",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "L": L, "n_sites": 2 * L, "N": N, "D": D,
            "terms": 4 * N * N + 2 * L,
            "input": f"random normalised real MPS, bonds min(2^j, 2^({2 * L}-j), {D}), seed {w['seed']}",
            "step": "one krylov_step: compressed H|v> (tree sum) + residual sum-compression + Ritz values",
            "compressions_per_step": n_comp / args.steps,
            "contraction_precision": args.prec,
        },
        "model_tflops_per_s": flops_model / elapsed / 1e12,
        # model flops of the whole step over its time, against the FP64 matrix peak
        "path_fraction_of_fp64_peak": flops_model / elapsed / 1e12 / FP64_MFMA_PEAK_TFLOPS,
        "lowest_ritz": float(ritz[0]) if ritz is not None else None,
        "fp64_contractions": f64,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
