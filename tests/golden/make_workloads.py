"""Write tests/golden/workloads.json: the frozen synthetic 16^3 x 32 workload.

Calls only ``oracle`` and ``synth``.  It tunes the near-identity spread epsilon
so that the mean plaquette is 0.594 (a typical quenched beta = 6 value, the
paper's ensemble of Sec. 3), then finds m_c for each formulation as the
minimiser of the 200-step Lanczos lowest Ritz value of (D+m)^dag (D+m).  The
bare masses of the workload are m_c + delta, delta in {0.02, 0.05, 0.1}.

Run:  python tests/golden/make_workloads.py      (about an hour on 8 cores), or
      python tests/golden/make_workloads.py --only W   and   --only SW   in parallel,
      then  python tests/golden/make_workloads.py --merge
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import critical, gauge, staggered_wilson  # noqa: E402

DIMS = (16, 16, 16, 32)
SEED = 2000
V0_SEED = 7
TARGET_PLAQ = 0.594
DELTAS = (0.02, 0.05, 0.1)
STEPS = 200
BRACKET = (-0.8, -0.2)


def _mc(args):
    formulation, eps = args
    U = synth.gauge_field(DIMS, "near_identity", SEED, eps)
    cor = staggered_wilson.corners(U) if formulation == synth.STAGGERED_WILSON else None
    v0 = synth.gaussian_field(DIMS, formulation, V0_SEED)
    tag = "W" if formulation == synth.WILSON else "SW"
    t0 = time.time()
    mc, th, trace = critical.critical_mass(
        formulation, U, v0, BRACKET[0], BRACKET[1], steps=STEPS, ngrid=7, ngolden=6,
        corners=cor, log=lambda s: print(f"[{tag} {time.time() - t0:7.0f}s]{s}", flush=True))
    return tag, dict(m_c=mc, theta_min=th, trace=trace)


def main():
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=["W", "SW"], help="compute one formulation's m_c into "
                    "workload_<W|SW>.json (run both, then --merge)")
    ap.add_argument("--merge", action="store_true", help="combine the two partial files")
    args = ap.parse_args()
    eps, plaq = gauge.tune_epsilon(DIMS, SEED, TARGET_PLAQ)
    print(f"epsilon={eps} plaquette={plaq}", flush=True)
    if args.only:
        form = synth.WILSON if args.only == "W" else synth.STAGGERED_WILSON
        tag, r = _mc((form, eps))
        with open(os.path.join(HERE, f"workload_{tag}.json"), "w") as f:
            json.dump(dict(eps=eps, plaquette=plaq, result=r), f, indent=1)
        return
    if args.merge:
        res = {}
        for tag in ("W", "SW"):
            with open(os.path.join(HERE, f"workload_{tag}.json")) as f:
                part = json.load(f)
            assert part["eps"] == eps
            res[tag] = part["result"]
    else:
        with mp.Pool(2) as pool:
            res = dict(pool.map(_mc, [(synth.WILSON, eps), (synth.STAGGERED_WILSON, eps)]))
    out = dict(
        description="Synthetic 16^3x32 stand-in for the paper's quenched beta=6 ensemble "
                    "(Sec. 3): independent near-identity SU(3) links exp(i eps H), eps tuned "
                    "to mean plaquette 0.594; m_c = argmin_m of the 200-step Lanczos lowest "
                    "Ritz value of (D+m)^dag(D+m); masses m_c + delta.",
        dims=list(DIMS), seed=SEED, eps=eps, plaquette=plaq, lanczos_steps=STEPS,
        v0_seed=V0_SEED, deltas=list(DELTAS), r=1.0, bc=[1, 1, 1, 1],
        m_c={"wilson": res["W"]["m_c"], "staggered_wilson": res["SW"]["m_c"]},
        theta_min_at_m_c={"wilson": res["W"]["theta_min"],
                          "staggered_wilson": res["SW"]["theta_min"]},
        scan={"wilson": res["W"]["trace"], "staggered_wilson": res["SW"]["trace"]},
        batch_seeds=list(range(SEED, SEED + 8)),
        generated_by="tests/golden/make_workloads.py (oracle only)",
    )
    with open(os.path.join(HERE, "workloads.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("eps", "plaquette", "m_c")}))


if __name__ == "__main__":
    main()
