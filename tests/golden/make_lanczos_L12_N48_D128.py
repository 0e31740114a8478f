#!/usr/bin/env python3
"""Write lanczos_L12_N48_D128.json: the FP64 oracle's MPS-Lanczos run of the
Hartree-Fock-started ground-state workload (Sec. 2.2 with eq. eff_H).

Workload: L = 12 spatial orbitals (24 spin-orbital sites), THC rank N = 48,
bond dimension D = 128, t / chi / zeta drawn by ``synth.thc_factors`` from
``default_rng(0)``, start vector the closed-shell determinant with 12
electrons (orbitals 0..5 doubly occupied).  Every H application is the
oracle's tree-summed H|psi> (``oracle.hamiltonian.apply_H_mapped``, the same
pairs as ``apply_H(mode="tree")``; its independent compressions run in a
process pool), the residual is one tree-summed sum-compression, and the
Ritz values come from ``oracle.lanczos``.  The file is rewritten after every
step, so an interrupted run still leaves the steps it finished.

Only ``oracle/`` and ``synth/`` are used.

    python tests/golden/make_lanczos_L12_N48_D128.py --steps 20 --procs 6
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import hamiltonian as OH  # noqa: E402
from oracle import lanczos as OL  # noqa: E402
from oracle import mps as M  # noqa: E402

OUT = os.path.join(HERE, "lanczos_L12_N48_D128.json")


def _one_thread():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--procs", type=int, default=max(1, (os.cpu_count() or 2) - 2))
    args = ap.parse_args()
    w = synth.WORKLOADS["L12_N48_D128"]
    L, N, D, ne = w["L"], w["N"], w["D"], w["n_elec"]
    t, chi, zeta = synth.thc_factors(np.random.default_rng(w["seed"]), L, N)
    hf = synth.occupation_mps_tensors(synth.hartree_fock_occupation(L, ne))
    rec = {"workload": "L12_N48_D128", "L": L, "N": N, "D": D, "n_elec": ne, "seed": w["seed"],
           "sum": "tree", "cutoff": M.CUTOFF, "steps": []}
    with mp.get_context("fork").Pool(args.procs, initializer=_one_thread) as pool:
        def Hfun(v):
            return OH.apply_H_mapped(v, t, chi, zeta, D, mapper=pool.map, window=256)
        st = OL.KrylovState(hf, args.steps)
        for i in range(args.steps):
            t0 = time.time()
            rg, rt, b = OL.krylov_step(st, t, chi, zeta, D, Hfun=Hfun)
            rec["steps"].append({
                "i": i, "ritz_generalized": [float(x) for x in rg], "ritz_tridiagonal": [float(x) for x in rt],
                "beta": float(b), "w_bonds": M.bonds(st.w[i]),
                "v_next_bonds": M.bonds(st.v[i + 1]) if len(st.v) > i + 1 else None,
                "seconds": time.time() - t0})
            with open(OUT + ".tmp", "w") as f:
                json.dump(rec, f, indent=1)
            os.replace(OUT + ".tmp", OUT)
            print(f"step {i}: lowest Ritz {rg[0]:.12f}, beta {b:.3e}, max bond {max(M.bonds(st.w[i]))}, "
                  f"{time.time() - t0:.0f} s", flush=True)
            if st.breakdown:
                break


if __name__ == "__main__":
    main()
