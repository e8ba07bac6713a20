"""Write tests/golden/fullsize.json: oracle FP64 CG iteration counts and 200-step
Lanczos condition numbers on the frozen 16^3 x 32 workload (field seed 2000).

Calls only ``oracle`` and ``synth``.  For each formulation and each
delta in {0.02, 0.05, 0.1} (mass m_c + delta, m_c frozen in workloads.json):
  * plain FP64 CGNR on eq. (2) (Sec. 3) from the point source at the origin
    (colour 0, spin 0), x0 = 0, tol 1e-8: iterations, restarts, the iterated
    and the FP64 true residual;
  * Lanczos with full reorthogonalisation, 200 steps from the seeded start
    vector (seed v0_seed): theta_min, theta_max and kappa = theta_max / theta_min
    (the condition number of (D+m)^dag (D+m), Sec. 3).

Run:  python tests/golden/make_fullsize.py [--jobs 6]      (about an hour on 8 cores)
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
STEPS = 200


def _work(args):
    kind, form, delta = args
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
        if kind == "cg":
            chi = synth.point_source(dims, form, 0)
            _, info = solvers.cgnr(form, U, chi, m, TOL, 100000, corners=cor)
            res = dict(iterations=info["iterations"], restarts=info["restarts"],
                       status=info["status"], iterated_residual=info["iterated_residual"],
                       true_residual=info["true_residual"])
        else:
            v0 = synth.gaussian_field(dims, form, w["v0_seed"])
            lo, hi, kappa, _ = solvers.condition_number(form, U, m, v0, STEPS, corners=cor)
            res = dict(theta_min=float(lo), theta_max=float(hi), kappa=float(kappa))
    res["seconds"] = time.time() - t0
    print(f"{kind} {name} delta={delta}: {res}", flush=True)
    return kind, name, str(delta), res


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=6)
    a = ap.parse_args()
    with open(os.path.join(HERE, "workloads.json")) as f:
        w = json.load(f)
    jobs = [(kind, form, d) for kind in ("lanczos", "cg") for form in (0, 1)
            for d in w["deltas"]]
    with mp.Pool(a.jobs) as pool:
        out = pool.map(_work, jobs, chunksize=1)
    res = {"cg": {"wilson": {}, "staggered_wilson": {}},
           "lanczos": {"wilson": {}, "staggered_wilson": {}}}
    for kind, name, d, r in out:
        res[kind][name][d] = r
    doc = dict(
        description="Oracle FP64 CGNR (tol 1e-8, point source alpha = 0, x0 = 0) and 200-step "
                    "Lanczos (full reorthogonalisation, start vector seed v0_seed) on field seed "
                    "2000 of the frozen 16^3x32 workload, masses m_c + delta.",
        dims=w["dims"], seed=w["seed"], eps=w["eps"], m_c=w["m_c"], v0_seed=w["v0_seed"],
        tol=TOL, lanczos_steps=STEPS, cg=res["cg"], lanczos=res["lanczos"],
        generated_by="tests/golden/make_fullsize.py (oracle only)")
    with open(os.path.join(HERE, "fullsize.json"), "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote fullsize.json", flush=True)


if __name__ == "__main__":
    main()
