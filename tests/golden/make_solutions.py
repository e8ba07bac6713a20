"""Write tests/golden/fullsize_solutions.json: fingerprints of the oracle's FP64
CG solutions on the frozen 16^3 x 32 workload (field seed 2000), so that GPU
solutions in every storage precision can be compared with the oracle's without
storing 25 MB fields.

Calls only ``oracle`` and ``synth``.  For each formulation and each delta in
{0.02, 0.05, 0.1} (mass m_c + delta, m_c frozen in workloads.json): plain FP64
CGNR on eq. (2) (Sec. 3) from the point source at the origin (colour 0, spin 0),
x0 = 0, tol 1e-8, and of its solution x*:
  * ||x*||^2;
  * every component of x* at 64 sites drawn without replacement by
    numpy.random.default_rng(SAMPLE_SEED) from the V sites (canonical site
    order: t outermost, x innermost);
  * <v_j, x*> = sum conj(v_j) x* for the four start-vector-like fields
    v_j = synth.gaussian_field(dims, formulation, seed) with seeds PROJ_SEEDS.

Run:  python tests/golden/make_solutions.py [--jobs 6]      (about 15 minutes on 8 cores)
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

TOL = 1e-8
SAMPLE_SEED = 4242
NSITES = 64
PROJ_SEEDS = [901, 902, 903, 904]


def _work(args):
    form, delta = args
    import numpy as np
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import solvers, staggered_wilson

    with open(os.path.join(HERE, "workloads.json")) as f:
        w = json.load(f)
    dims = tuple(w["dims"])
    name = "wilson" if form == synth.WILSON else "staggered_wilson"
    m = w["m_c"][name] + delta
    t0 = time.time()
    with threadpool_limits(limits=1):
        U = synth.gauge_field(dims, "near_identity", w["seed"], w["eps"])
        cor = staggered_wilson.corners(U) if form == synth.STAGGERED_WILSON else None
        chi = synth.point_source(dims, form, 0)
        x, info = solvers.cgnr(form, U, chi, m, TOL, 100000, corners=cor)
    V = int(np.prod(dims))
    flat = x.reshape(V, -1)
    sites = np.random.default_rng(SAMPLE_SEED).choice(V, NSITES, replace=False)
    samp = flat[np.sort(sites)]
    proj = []
    for s in PROJ_SEEDS:
        v = synth.gaussian_field(dims, form, s)
        proj.append(complex(np.vdot(v.ravel(), x.ravel())))
    res = dict(iterations=info["iterations"], true_residual=info["true_residual"],
               norm2=float(np.vdot(x.ravel(), x.ravel()).real),
               sites=[int(i) for i in np.sort(sites)],
               samples_re=[[float(z.real) for z in row] for row in samp],
               samples_im=[[float(z.imag) for z in row] for row in samp],
               proj_re=[p.real for p in proj], proj_im=[p.imag for p in proj],
               seconds=time.time() - t0)
    print(f"{name} delta={delta}: iterations {res['iterations']} in {res['seconds']:.0f}s",
          flush=True)
    return name, str(delta), res


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    a = ap.parse_args()
    with open(os.path.join(HERE, "workloads.json")) as f:
        w = json.load(f)
    jobs = [(form, d) for form in (0, 1) for d in w["deltas"]]
    with mp.Pool(a.jobs) as pool:
        out = pool.map(_work, jobs, chunksize=1)
    res = {"wilson": {}, "staggered_wilson": {}}
    for name, d, r in out:
        res[name][d] = r
    doc = dict(
        description="Fingerprints of the oracle's FP64 CGNR solutions (tol 1e-8, point source "
                    "alpha = 0, x0 = 0) on field seed 2000 of the frozen 16^3x32 workload, masses "
                    "m_c + delta: squared norm, every component at 64 seeded sites, and the "
                    "projections on four seeded Gaussian fields.",
        dims=w["dims"], seed=w["seed"], eps=w["eps"], m_c=w["m_c"], tol=TOL,
        sample_seed=SAMPLE_SEED, proj_seeds=PROJ_SEEDS, solutions=res,
        generated_by="tests/golden/make_solutions.py (oracle only)")
    with open(os.path.join(HERE, "fullsize_solutions.json"), "w") as f:
        json.dump(doc, f, indent=0)
    print("wrote fullsize_solutions.json", flush=True)


if __name__ == "__main__":
    main()
