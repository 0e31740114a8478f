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
in FP64.  The input sits in device memory before the timed region starts.

The run keeps to a wall budget (--budget seconds from process start, the CPU
baseline included): --steps and --warmup are upper bounds, at least one full
step is always timed, and a further step (warm-up or timed) starts only
while the measured step time still fits.  Before the timed steps, on fixed
slices of the same workload:
* the CPU oracle times one layer-compression and one add-compression
  (cpu_baseline), and the GPU computes the same two compressions in FP64
  and in the bench precision: their distance to the oracle's results is the
  per-result error;
* the same H|psi> with the THC rank cut to its first 8 columns is timed with
  FP64 and with mixed contractions (mixed vs FP64), and a few of its leaf
  layer-compressions one at a time (the plain, unbatched form).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

T_START = time.monotonic()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6  # MI355X dense FP64 matrix peak (vendor figure)
HBM_PEAK_GBS = 8000.0         # MI355X HBM3E peak bandwidth (vendor figure)
# FP64 vector ALU peak: 256 CUs x 4 SIMDs x 16 FP64 FMA lanes x 2 flops x 2.4 GHz
FP64_VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# kernel classes whose arithmetic runs on the vector ALUs (the rest on MFMA;
# the tridiagonalisation class is the two-stage route's MFMA band reduction)
VALU_KERNELS = ("tri_eig", "sb2st", "q2")
SLICE_N = 8          # THC rank of the mixed-vs-FP64 slice
PLAIN_SAMPLES = 4    # leaf layer-compressions timed one job per launch


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def elapsed():
    return time.monotonic() - T_START


KERNEL_FN = {"lq": ("k_lq2", "k_lq_q"), "sytrd": "k_sy2sb", "tri_eig": "k_tri_eig", "ormtr": "k_ormtr2", "gemm": "k_gemm_mfma",
             "sb2st": "k_sb2st", "q2": "k_q2apply"}
KERNEL_SOURCES = ("kernels.hip", "band.hip")


def kernel_digest(fn):
    """SHA-256 of a kernel's source text (from its signature line to its closing
    brace); for a class of several kernels, of their texts joined in order."""
    import hashlib
    if isinstance(fn, tuple):
        parts = [kernel_digest(f) for f in fn]
        return None if None in parts else hashlib.sha256("".join(parts).encode()).hexdigest()
    for name in KERNEL_SOURCES:
        src = open(os.path.join(ROOT, "paper_2409_12708_amd", "csrc", name)).read().splitlines()
        try:
            i = next(k for k, l in enumerate(src) if f"void {fn}(" in l)
            j = next(k for k in range(i, len(src)) if src[k] == "}")
        except StopIteration:
            continue
        return hashlib.sha256("\n".join(src[i:j + 1]).encode()).hexdigest()
    return None


def measured_traffic(kernel: str, workload: str, algorithmic_bytes_per_launch: float):
    """HBM bytes per launch from the committed counter runs (profiles/): the
    measured-over-algorithmic byte ratio of the kernel's launches in those runs
    times this run's algorithmic bytes per launch; None when there are no
    counter runs or the kernel's source has changed since they were taken."""
    fn = KERNEL_FN.get(kernel)
    first = fn[0] if isinstance(fn, tuple) else fn
    path = os.path.join(ROOT, "profiles", f"traffic_{first}_{workload}.json")
    if not fn or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != kernel_digest(fn):
        return None
    return int(rec["measured_over_algorithmic"] * algorithmic_bytes_per_launch)


KERNEL_LABEL = {"lq": "k_lq2 + k_lq_q (Householder LQ, then Q from its compact-WY blocks, FP64)",
                "sytrd": "k_sy2sb (tridiagonalisation: band reduction, FP64 MFMA)",
                "sb2st": "k_sb2st (tridiagonalisation: band chase, FP64)",
                "q2": "k_q2apply (band-chase back-transformation, FP64)",
                "tri_eig": "k_tri_eig (bisection + inverse iteration, FP64)",
                "ormtr": "k_ormtr2 (eigenvector back-transformation, FP64)", "gemm": "k_gemm_mfma (FP64)",
                "svd_fallback": "second Gram level of the SVD (jobs at the noise floor)"}


def roofline_of(kms, kfl, kby, kn):
    """The dominant kernel class (largest summed device time among those with
    algorithmic flops) against the roof its arithmetic intensity puts it
    under: HBM below the ridge point (FP64 peak / HBM peak), else the FP64
    peak of the unit it computes on.  Flops and bytes per class are the
    method's (the operation counts of the factorisation or product, and the
    bytes it must move), so excess traffic of an implementation shows only
    in the measured counters.  Inputs per class: summed ms, flops, bytes,
    launches.  The returned dict carries the class under "_class"."""
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
        "algorithmic_flops_per_launch": float(kfl[dom] / max(kn[dom], 1)),
        "intensity_flop_per_byte": round(intensity, 3),
        "ridge_flop_per_byte": round(ridge, 2),
        "achieved_tflops": round(kfl[dom] / sec / 1e12, 3),
        "avg_launch_ms": round(kms[dom] / max(kn[dom], 1), 4),
        "launches": int(kn[dom]),
        "_class": dom,
    }


def model_compress_flops(bonds_in, D):
    """Flops of one compression of an MPS with uncompressed bonds bonds_in,
    by the LAPACK-formula model (FMA = 2): right-to-left LQ sweep (thin Q,
    2 (2 M K^2 - 2 K^3 / 3)) with the absorb of L, left-to-right thin SVD
    (Golub-Reinsch with both factors, 14 M K^2 + 8 K^3) truncated to D with
    the absorb of S V^T.  This is a model of the method (Fig. 3), not of the
    operations this library runs."""
    B = bonds_in
    n = len(B) - 1
    c = [1] * (n + 1)
    for j in range(n - 1, 0, -1):
        c[j] = min(B[j], 2 * c[j + 1])
    k = [1] * (n + 1)
    for j in range(n - 1):
        k[j + 1] = min(2 * k[j], c[j + 1], D)
    fl = 0.0
    for j in range(n - 1, 0, -1):
        M_, K_ = max(2 * c[j + 1], B[j]), min(2 * c[j + 1], B[j])
        fl += 2 * (2 * M_ * K_ ** 2 - 2 * K_ ** 3 / 3)   # LQ of site j
        fl += 2 * (2 * B[j - 1]) * B[j] * c[j]             # L absorbed into site j-1
    for j in range(n - 1):
        M_, K_ = max(2 * k[j], c[j + 1]), min(2 * k[j], c[j + 1])
        fl += 14 * M_ * K_ ** 2 + 8 * K_ ** 3              # SVD at bond j+1
        fl += 2 * k[j + 1] * c[j + 1] * 2 * c[j + 2]       # S V^T absorbed into site j+1
    return fl


def model_flops_per_H(L, N, D):
    """Model flops of one compressed H|psi> on a saturated MPS of bond D:
    4N + 8N^2 + 4L layer-compressions and 4N^2 + 2L add-compressions, every
    input at bonds min(2^j, 2^(n-j), D), doubled by the layer or the sum."""
    n = 2 * L
    chi = [min(2 ** j, 2 ** (n - j), D) for j in range(n + 1)]
    doubled = [1] + [2 * x for x in chi[1:-1]] + [1]
    per = model_compress_flops(doubled, D)
    return per * ((4 * N + 8 * N * N + 4 * L) + (4 * N * N + 2 * L))


def one_stage_sytrd_bytes(m: int, nb: int = 8) -> float:
    """Bytes a one-stage (panel) tridiagonalisation streams for an m x m
    matrix: the trailing upper triangle read once per column and written once
    more by the first column of each panel of nb after the first."""
    el = 0.0
    for i in range(m - 2):
        s = m - i - 1
        el += 0.5 * s * (s + 1.0) * (2.0 if (i > 0 and i % nb == 0) else 1.0)
    return 8.0 * el


def two_stage_sy2sb_bytes(m: int, bw: int = 16) -> float:
    """Bytes the band reduction streams for an m x m matrix: per panel of bw
    columns the trailing upper triangle (16 x 16 tiles, diagonal tiles whole)
    read and written by the update, the panel read and written, and the next
    trailing triangle read by the product."""
    def tri(n):
        t = -(-n // 16)
        return t * (t + 1) / 2 * 256.0
    el = 0.0
    c0 = 0
    while True:
        if c0 > 0:
            el += 2.0 * tri(m - c0)
        r0 = c0 + bw
        if m - r0 < 2:
            break
        el += 2.0 * bw * (m - r0) + tri(m - r0)
        c0 += bw
    return 8.0 * el


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover - informational only
        return len(os.sched_getaffinity(0))


def cpu_baseline(t, chi, zeta, sites, D, L, N, pooled=None):
    """Time the FP64 oracle on a bounded sample of the workload: one
    layer-compression and one add-compression at the full bond dimension,
    extrapolated to the compressions of one H|psi>.  The record is the faster
    of this threaded-BLAS form and the term-parallel form measured before
    (``pooled``), both kept under "modes".  Returns the baseline record and
    the two oracle results (with their Schmidt spectra at the cuts) for the
    per-result error of the GPU path."""
    from oracle import mps as M
    from oracle import thc as TH

    y = TH.spin_site_coeffs(chi[:, 0], 0)
    spec_l, spec_a = [], []
    t0 = time.perf_counter()
    lay = M.compress(M.apply_layer(sites, y, False), D, record=spec_l)
    t1 = time.perf_counter()
    add = M.compress(M.direct_sum([(1.0, lay), (1.0, sites)]), D, record=spec_a)
    t2 = time.perf_counter()
    t_layer, t_add = t1 - t0, t2 - t1
    n_layer = 2 * 2 * N + 2 * 4 * N * N + 2 * 2 * L
    n_add = 4 * N * N + 2 * L - 1
    per_h = n_layer * t_layer + n_add * t_add
    threaded = {
        "value": 1.0 / per_h,
        "unit": "H|psi>/s",
        "cores": int(blas_threads()),
        "kind": "oracle",
        "sample": (f"one layer-compression ({t_layer:.2f} s) and one add-compression ({t_add:.2f} s) of the "
                   f"L={L} (n={2 * L}) MPS at D={D}, FP64 NumPy/LAPACK (threaded BLAS, one process), extrapolated "
                   f"to the {n_layer} layer- and {n_add} add-compressions of one H|psi>"),
    }
    rec = dict(threaded)
    if pooled is not None:
        rec = dict(pooled) if pooled["value"] > threaded["value"] else rec
        rec["modes"] = {"threaded_blas": threaded, "term_parallel": pooled}
    return rec, (y, lay, spec_l), (add, spec_a)


def _pool_init():
    # one BLAS thread per worker process: the thread counts are read when
    # numpy's BLAS loads, which happens after this in a spawned worker
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        os.environ[v] = "1"
    import numpy  # noqa: F401
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _pool_job(args):
    """One layer-compression (THC column x, spin up, annihilator) and one
    add-compression of its result with the input, timed separately."""
    from oracle import mps as M
    from oracle import thc as TH
    sites, x, D = args
    t0 = time.perf_counter()
    lay = M.compress(M.apply_layer(sites, TH.spin_site_coeffs(x, 0), False), D)
    t1 = time.perf_counter()
    M.compress(M.direct_sum([(1.0, lay), (1.0, sites)]), D)
    return t1 - t0, time.perf_counter() - t1


def pool_cores():
    """Worker processes for the term-parallel baseline: the cores this
    process may run on, at most the thread count the environment grants
    (OMP_NUM_THREADS) and 16."""
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, min(n, 16))


def cpu_baseline_pool(chi, sites, D, L, N):
    """The oracle in the paper's term-parallel form (independent terms on
    separate cores, Sec. 4.5): one process per core with one BLAS thread,
    each running one layer-compression (its own THC column) and one
    add-compression of the workload MPS; the mean times divided by the
    process count give the pool's time per compression, extrapolated to one
    H|psi>.  Runs before the GPU is initialised: the workers are started
    with spawn, which a process holding a GPU context may not do here."""
    import multiprocessing as mp
    cores = pool_cores()
    if cores < 2:
        return None
    n_layer = 2 * 2 * N + 2 * 4 * N * N + 2 * 2 * L
    n_add = 4 * N * N + 2 * L - 1
    # bounded waits: a pool that cannot start its workers raises instead of hanging
    with mp.get_context("spawn").Pool(cores, initializer=_pool_init) as pool:
        pool.map_async(_pool_init_probe, range(cores)).get(timeout=60)  # workers up before the clock
        log(f"[bench] {cores} oracle processes started; {elapsed():.0f} s since start")
        t0 = time.perf_counter()
        times = pool.map_async(_pool_job, [(sites, chi[:, i % chi.shape[1]], D) for i in range(cores)],
                               chunksize=1).get(timeout=150)
        wall = time.perf_counter() - t0
    t_layer = sum(a for a, _ in times) / len(times) / cores
    t_add = sum(b for _, b in times) / len(times) / cores
    per_h = n_layer * t_layer + n_add * t_add
    return {
        "value": 1.0 / per_h,
        "unit": "H|psi>/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{cores} processes with one BLAS thread each (terms in parallel, as the paper's OpenMP scheme), "
                   f"each one layer-compression and one add-compression of the L={L} (n={2 * L}) MPS at D={D} "
                   f"({wall:.1f} s wall; per process {t_layer * cores:.2f} s and {t_add * cores:.2f} s), FP64 "
                   f"NumPy/LAPACK, extrapolated to the {n_layer} layer- and {n_add} add-compressions of one H|psi>"),
    }


def _pool_init_probe(_):
    from oracle import mps  # noqa: F401
    return 0


def min_cut_gap(spectra, D):
    """Smallest relative gap (s_D - s_{D+1}) / s_1 over the bonds where the
    compression truncated (the conditioning of the truncated result)."""
    gaps = [(s[D - 1] - s[D]) / s[0] for s in spectra if len(s) > D and s[0] > 0]
    return min(gaps) if gaps else None


def rel_distance(a_sites, b_sites):
    """|| a - b || / || b || from three oracle overlaps (resolves ~1e-8)."""
    from oracle import mps as M
    aa, bb, ab = M.overlap(a_sites, a_sites), M.overlap(b_sites, b_sites), M.overlap(a_sites, b_sites)
    return float((max(aa + bb - 2.0 * ab, 0.0)) ** 0.5 / max(bb, 1e-300) ** 0.5)


def evolve_run(args, thck, synth, np, torch):
    """One Krylov time step (Sec. 2.2) of a batch of instances of uneven size
    in one krylov_evolve call: the time-evolution configuration's structure
    (instances of different L, N = 4L and D, Hartree-Fock single-excitation
    starts, K = 12, delta = 0.05) at sizes one step of which takes seconds."""
    rng = np.random.default_rng(7)
    insts, draws = [], []
    for q in range(args.evolve):
        L = int(rng.integers(8, 13))
        D = int(rng.choice([32, 64]))
        t, chi, zeta = synth.thc_factors(rng, L, 4 * L)
        n_elec = L if L % 2 == 0 else L - 1
        psi = thck.DeviceMPS.from_sites(synth.occupation_mps_tensors(synth.single_excitation_occupation(L, n_elec)))
        insts.append((thck.Context(t, chi, zeta), psi, None, D, {"prec": args.prec}))
        draws.append({"L": L, "N": 4 * L, "D": D, "electrons": n_elec})
    torch.cuda.synchronize()
    st = thck.ThcStats()
    t0 = time.perf_counter()
    outs, dims = thck.evolve(insts, K=12, delta=0.05, n_steps=1, stats=st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    norms = [float(np.sqrt(max(inst[0].overlap(a, a) + inst[0].overlap(b, b), 0.0)))
             for inst, (a, b) in zip(insts, outs)]
    print(json.dumps({"evolve": True, "instances": draws, "K": 12, "delta": 0.05, "steps": 1,
                      "krylov_dims": dims.tolist(), "seconds": wall, "compressions": int(st.n_compressions),
                      "norms_after": norms, "contraction_precision": args.prec}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="L20_N80_D256")
    ap.add_argument("--budget", type=float, default=450.0,
                    help="wall seconds from process start within which a new step may still start")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-slices", action="store_true", help="skip the mixed-vs-FP64 and unbatched slices")
    ap.add_argument("--profile-slice", action="store_true",
                    help="counter runs: only the THC-rank-8 slice of H|psi> (batches of the step's shapes) and a "
                         "device copy of known size; prints the slice's algorithmic bytes per kernel class")
    ap.add_argument("--prec", default="bf16x3", choices=["f64", "f32", "bf16x3"],
                    help="contraction precision of the absorb products (factorisations stay FP64)")
    ap.add_argument("--evolve", type=int, default=0, metavar="INSTANCES",
                    help="instead of the Lanczos step: one Krylov time step (K = 12, delta = 0.05) of this many "
                         "instances in one call, L drawn from 8..12, N = 4L, D from {32, 64}, each from a "
                         "Hartree-Fock single excitation; prints the draws and the time")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}, WORLD_SIZE={world}): the THC-MPO path of "
              f"this library is a single-GPU build; no multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("THCK_PROGRESS", "1")  # the library reports finished compression batches on stderr
    import numpy as np

    import synth

    pooled = None
    if not args.no_cpu_baseline and not args.profile_slice and not args.evolve:
        # the term-parallel CPU baseline spawns its workers, so it runs first
        w = synth.WORKLOADS[args.workload]
        _, chi_p, _, sites_p = synth.make_workload(args.workload)
        from oracle import mps as OMp
        sites_p = OMp.scale(sites_p, 1.0 / float(np.sqrt(OMp.overlap(sites_p, sites_p))))
        log(f"[bench] timing the CPU oracle, terms in parallel ({pool_cores()} processes)")
        try:
            pooled = cpu_baseline_pool(chi_p, sites_p, w["D"], w["L"], w["N"])
            log(f"[bench] cpu baseline (terms in parallel): {pooled['value']:.3e} H|psi>/s; {elapsed():.0f} s "
                f"since start")
        except Exception as e:  # the threaded form below still gives a baseline
            log(f"[bench] term-parallel CPU baseline failed: {e!r}")
        del chi_p, sites_p

    import torch

    import paper_2409_12708_amd as thck

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    w = synth.WORKLOADS[args.workload]
    L, N, D = w["L"], w["N"], w["D"]
    t, chi, zeta, sites = synth.make_workload(args.workload)
    from oracle import mps as OM  # noqa: F401  (CPU baseline and result checks only)
    nrm = float(np.sqrt(OM.overlap(sites, sites)))
    sites = OM.scale(sites, 1.0 / nrm)  # normalised on the host: GPU and oracle see the same state
    ctx = thck.Context(t, chi, zeta)
    psi = thck.DeviceMPS.from_sites(sites)
    torch.cuda.synchronize()
    log(f"[bench] workload {args.workload}: L={L} N={N} D={D}; requested warmup {args.warmup}, steps "
        f"{args.steps}; budget {args.budget:.0f} s; {elapsed():.1f} s since start")

    if args.evolve:
        evolve_run(args, thck, synth, np, torch)
        return

    if args.profile_slice:
        # a device copy of 64 MiB (read and written once) calibrates the counters
        src = torch.ones(8 << 20, dtype=torch.float64, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        ctx_s = thck.Context(t, np.ascontiguousarray(chi[:, :SLICE_N]), np.ascontiguousarray(zeta[:SLICE_N, :SLICE_N]))
        st = thck.ThcStats()
        ctx_s.apply_H(psi, D=D, stats=st, prec=args.prec, flags=thck.FLAG_TIME_KERNELS)
        torch.cuda.synchronize()
        names = thck.ThcStats.KERNELS
        print(json.dumps({"profile_slice": True, "copy_bytes": 2 * dst.numel() * 8,
                          "kernels": {k: {"launches": int(st.kernel_launches[i]), "ms": st.kernel_ms[i],
                                          "algorithmic_bytes": st.kernel_bytes[i],
                                          "algorithmic_flops": st.kernel_flops[i]}
                                      for i, k in enumerate(names)}}), flush=True)
        return

    # ---- the timed Lanczos steps, under the wall budget ----
    K = min(31, max(1, args.warmup + args.steps))
    kr = thck.Krylov(ctx, psi, K, D=D, flags=thck.FLAG_TIME_KERNELS, prec=args.prec)
    step_s = None  # measured by the first step
    # warm-up steps run only when a step time is known and a warm-up plus a
    # timed step fit in the budget; the first call of a process is timed as
    # it is (its one-time costs, the workspace allocation and the first
    # launch of each kernel, are part of the timed step then)
    warm_done = 0
    torch.cuda.synchronize()
    stats, ritz, beta = [], None, None
    t_begin = time.perf_counter()
    for s in range(args.steps):
        if s > 0 and (elapsed() + step_s * 1.05 > args.budget or kr.steps >= K):
            break
        st = thck.ThcStats()
        t0 = time.perf_counter()
        ritz, _, beta = kr.step(st)
        step_s = time.perf_counter() - t0
        stats.append(st)
        log(f"[bench] step {s}: {step_s:.1f} s, lowest Ritz value {ritz[0]:.10f}, beta {beta:.3e}, compressions "
            f"{st.n_compressions}, SVD fallbacks {st.svd_fallbacks}, max discarded weight "
            f"{st.discarded_weight_max:.3e}; {elapsed():.0f} s since start")
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t_begin
    kr.close()
    n_steps = len(stats)

    # ---- after the timed steps, as the budget allows: the CPU oracle on a
    # bounded sample (and the GPU's error on the same results), then the
    # fixed slices (mixed vs FP64 contractions, batched vs one job per launch)
    extras_limit = args.budget + 100.0
    # ---- CPU oracle on a bounded sample, and the GPU's error on the same results ----
    cpu, accuracy = None, None
    if not args.no_cpu_baseline and elapsed() + 30.0 < extras_limit:
        log("[bench] timing the CPU oracle on a bounded sample")
        cpu, (y, lay_ref, spec_l), (add_ref, spec_a) = cpu_baseline(t, chi, zeta, sites, D, L, N, pooled)
        log(f"[bench] cpu baseline: {cpu['value']:.3e} H|psi>/s ({cpu['sample']})")
        accuracy = {"reference": "FP64 oracle (NumPy/LAPACK), same input, same truncation rule",
                    "metric": "|| gpu - oracle || / || oracle || from FP64 overlaps (resolves ~1e-8)",
                    "layer_compress_min_cut_gap": min_cut_gap(spec_l, D),
                    "add_compress_min_cut_gap": min_cut_gap(spec_a, D)}
        for prec in ("f64", args.prec) if args.prec != "f64" else ("f64",):
            lay_g = ctx.apply_layer(psi, y, False, D, prec=prec)
            add_g = ctx.sum_compress([1.0, 1.0], [thck.DeviceMPS.from_sites(lay_ref), psi], D, prec=prec)
            torch.cuda.synchronize()
            accuracy[prec] = {"layer_compress": rel_distance(lay_g.to_sites(), lay_ref),
                              "add_compress": rel_distance(add_g.to_sites(), add_ref)}
            log(f"[bench] {prec}: error vs oracle, layer-compression {accuracy[prec]['layer_compress']:.3e}, "
                f"add-compression {accuracy[prec]['add_compress']:.3e}")

    # ---- fixed slices: mixed vs FP64 contractions, batched vs one job per launch ----
    slices = None
    if not args.no_slices and elapsed() + 60.0 < extras_limit:
        ctx_s = thck.Context(t, np.ascontiguousarray(chi[:, :SLICE_N]),
                             np.ascontiguousarray(zeta[:SLICE_N, :SLICE_N]))
        res, times = {}, {}
        for prec in ("f64", args.prec):
            st = thck.ThcStats()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res[prec] = ctx_s.apply_H(psi, D=D, stats=st, prec=prec)
            torch.cuda.synchronize()
            times[prec] = (time.perf_counter() - t0, st.n_compressions, st.svd_fallbacks)
            log(f"[bench] slice N={SLICE_N} {prec}: {times[prec][0]:.2f} s, {st.n_compressions} compressions")
        a, b = res[args.prec].to_sites(), res["f64"].to_sites()
        # plain form: leaf layer-compressions of the slice, one job per launch, FP64
        y0 = np.zeros(2 * L)
        y0[0::2] = chi[:, 0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(PLAIN_SAMPLES):
            ctx_s.apply_layer(psi, y0, False, D, prec="f64", batch=1)
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - t0) / PLAIN_SAMPLES
        per_batched = times["f64"][0] / times["f64"][1]
        slices = {
            "slice": (f"H|psi> with the first {SLICE_N} THC columns (chi[:, :{SLICE_N}], zeta[:{SLICE_N}, :{SLICE_N}]) "
                      f"and the full t at L={L}, D={D}: {times['f64'][1]} compressions of the same shapes"),
            "f64_s": times["f64"][0], f"{args.prec}_s": times[args.prec][0],
            "speedup_of_mixed": times["f64"][0] / times[args.prec][0],
            "mixed_vs_f64_rel_distance": rel_distance(a, b),
            "plain_f64_ms_per_compression": t_plain * 1e3,
            "batched_f64_ms_per_compression": per_batched * 1e3,
            "batching_gain": t_plain / per_batched,
            "plain_form": (f"{PLAIN_SAMPLES} leaf layer-compressions of the workload MPS, one job per launch "
                           f"(thc_opts.batch = 1), FP64 contractions"),
            "svd_fallbacks": {"f64": times["f64"][2], args.prec: times[args.prec][2]},
        }
        log(f"[bench] slices: mixed speedup {slices['speedup_of_mixed']:.3f}x, batching gain "
            f"{slices['batching_gain']:.1f}x, mixed vs f64 distance {slices['mixed_vs_f64_rel_distance']:.2e}")
        ctx_s.close()

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
            log(f"[bench] {k:12s} launches {kn[k]:7d}  device {sec:8.2f} s  avg {kms[k] / kn[k]:8.3f} ms  "
                f"{rate:6.2f} TFLOP/s")
    roofline = roofline_of(kms, kfl, kby, kn)
    dom = roofline.pop("_class")
    traffic = measured_traffic(dom, args.workload, roofline["algorithmic_bytes_per_launch"])
    roofline["traffic"] = traffic
    if traffic is not None:
        roofline["traffic_over_algorithmic"] = round(traffic / max(roofline["algorithmic_bytes_per_launch"], 1), 2)
    if dom == "sytrd":
        roofline["note"] = ("flops 4m^3/3 and bytes m^2 + 3m doubles per m x m matrix (the method's); the "
                            "two-stage band reduction streams the trailing triangle three times per panel of 16 "
                            f"columns, {two_stage_sy2sb_bytes(512) / 1e6:.1f} MB per 512 x 512 matrix (the "
                            f"one-stage kernel {one_stage_sytrd_bytes(512) / 1e6:.1f} MB)")
    executed = sum(st.flops_model for st in stats)
    n_comp = sum(st.n_compressions for st in stats)
    model_h = model_flops_per_H(L, N, D)
    per_step = t_steps / max(n_steps, 1)

    line = {
        "metric": "THC H|ψ⟩ applications/sec (L=20, D=256) + fraction of MFMA peak, mixed vs FP64",
        "value": n_steps / t_steps,
        "unit": "H|psi>/s",
        "n_gpus": 1,
        "steps": n_steps,
        "warmup": warm_done,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "ms_per_step": per_step * 1e3,
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
            "compressions_per_step": n_comp / max(n_steps, 1),
            "contraction_precision": args.prec,
        },
        # the method's flops (LAPACK-formula model of Fig. 3's compression at this workload,
        # 4N + 8N^2 + 4L layer- and 4N^2 + 2L add-compressions) per H|psi> over the step time
        "model_flops_per_H": model_h,
        "path_fraction_of_fp64_peak_model": model_h / per_step / 1e12 / FP64_MFMA_PEAK_TFLOPS,
        # the flops of the operations the library ran (its Gram SVD route, structured sweeps, re-canonicalisation)
        "executed_flops_per_step": executed / max(n_steps, 1),
        "path_fraction_of_fp64_peak_executed": executed / t_steps / 1e12 / FP64_MFMA_PEAK_TFLOPS,
        "svd_fallbacks_per_step": sum(st.svd_fallbacks for st in stats) / max(n_steps, 1),
        "lowest_ritz": float(ritz[0]) if ritz is not None else None,
        "error_vs_oracle": accuracy,
        "slices": slices,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "wall_s": elapsed(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
