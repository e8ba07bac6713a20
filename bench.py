"""Benchmark: CG solves/s on the 16^3 x 32 workload, mixed-precision batched vs FP64.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision q16|f32]

Workload (synthetic stand-in for the paper's quenched beta = 6 ensemble on
16^3 x 32, Sec. 3): 8 gauge fields of independent near-identity SU(3) links
(seeds 2000..2007, spread tuned to mean plaquette 0.594), point sources at the
origin -- 12 spin-colour sources for Wilson and 3 colour sources for staggered
Wilson, as the paper averages over -- at bare masses m_c + delta, delta in
{0.02, 0.05, 0.1}, with m_c frozen per formulation by the oracle
(tests/golden/workloads.json).  Every system is solved to an FP64 true
residual ||b - A x|| / ||b|| <= 1e-8 on eq. (2), unpreconditioned.

One step = all 360 systems: per field, one batched launch sequence for the 36
Wilson systems and one for the 9 staggered Wilson systems; stencil and Krylov
vectors stored in 16-bit fixed point (or FP32), FP32 arithmetic, FP64
reductions and reliable updates.  `value` is systems solved per second over
the timed steps.  Alongside (outside the timed region): FP64 single-RHS CG on
every system of the same mix, one at a time (the baseline the speed-up is
quoted against); the dominant kernel's roofline figures from HIP events on
non-zero data; the FP64 matvecs (Wilson, staggered Wilson from corners and on
the fly) at 16^3x32 and 32^3x64 against the HBM and FP64 rooflines; the
Lanczos condition numbers at the three masses; the paper's W/SW cost ratios
measured (Sec. 3, eqs. (3)-(4)); and the oracle timed on the host's cores
(before the GPU is touched: its worker processes are spawned).  Last, the
serving loop (`--serving` alone runs just that; `--no-serving` skips it).

Profiling modes (each runs only what a profiler should see):
    --roofline-only --rhs-per-thread K --window W   the dominant stencil alone
    --matvec-only                                   the FP64 matvecs, both sizes
    --copy-calibration                              a 256 MiB device copy x5
    --summarize-profile TRACE FETCH WRITE CFETCH CWRITE
        reads rocprofv3 output of the two modes above and writes the
        counter-based traffic figures the roofline line reports
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = os.path.join(ROOT, "tests", "golden", "workloads.json")
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
TOL = 1e-8
DELTAS = (0.02, 0.05, 0.1)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_workload():
    with open(WORKLOADS) as f:
        w = json.load(f)
    return w


def bytes_per_site(formulation, precision, links, nrhs, kernel=0, g55=0):
    """Compulsory HBM bytes per site of one stencil launch over nrhs fields:
    the links (and, for the corner form, the corners) once, and per RHS:
    kernel 0 (t = M p + ||t||^2) and kernel 1 (a plain matvec) read the input
    and write the output; kernel 2 (q = M^dag t, r -= alpha q, ||r||^2) reads
    t and reads and writes r, and on every fourth launch also reads the four
    search directions of the group and reads and writes x (FP32 under 16-bit
    storage) -- per launch on average 4 vectors and half an x.  12-real links
    are read as their rows 0 and 1 (in FP64 too); g55 = 1 (staggered Wilson
    on the fly) reads no corners."""
    nc = 12 if formulation == 0 else 3
    per = {0: 16, 1: 8, 2: 4}[precision]
    vec = nc * per + (4 if precision == 2 else 0)            # Q16: per-site float scale
    xvec = nc * (8 if precision == 2 else per)
    link = 4 * (links // 2) * per
    corner = 0 if (formulation == 0 or g55 == 1) else 8 * 9 * (4 if precision == 2 else per)
    per_rhs = 2 * vec if kernel in (0, 1) else 4 * vec + xvec // 2
    return nrhs * per_rhs + link + corner


# flops per site of one FP64 application of D (a complex 3x3 mat-vec with its
# accumulation counted as 66 + 12 = 78): Wilson r = 1, 8 spin-projected hops
# (2 mat-vecs each) plus projection and reconstruction, the paper's 1392
# (Sec. 3, eq. (4)); staggered Wilson from corners: 8 D_st hops + 16 corners
# (24 x 78) + the diagonal and combination (30); on the fly: 8 D_st hops +
# the 32 C applications of the subset recursion (64 mat-vecs) + 30
FLOPS_PER_SITE = {"wilson": 1392, "staggered_wilson_corners": 24 * 78 + 30,
                  "staggered_wilson_onthefly": (8 + 64) * 78 + 30}
FP64_PEAK_TFLOPS = 78.6


NRHS_W = 36                      # Wilson systems per field: 12 sources x 3 masses
PROFILE_JSON = os.path.join(ROOT, "profiles", "stencil_wilson_batched_16x32_traffic.json")
# sources whose change invalidates the stored counter readings of the stencil
STENCIL_SOURCES = ["csrc/common.h", "csrc/dirac.h", "csrc/stencil.h", "csrc/stencil_dispatch.h",
                   "csrc/stencil_tsweep.h", "csrc/k_stencil_wilson.hip", "build.py"]


def stencil_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STENCIL_SOURCES:
        with open(os.path.join(ROOT, "paper_1312_3265_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _cfg_key(cfg):
    return f"K{cfg[0]}_w{cfg[1]}"


def stored_traffic(storage, links, cfg):
    """Bytes per launch beyond L2 (FETCH_SIZE + WRITE_SIZE, calibrated) from the
    committed counter readings of the dominant stencil, if they were taken on
    the current stencil sources, with this storage and in this launch
    configuration (systems per thread, block order); else None."""
    try:
        with open(PROFILE_JSON) as f:
            p = json.load(f)
    except OSError:
        return None
    if p.get("source_sha256") != stencil_source_hash():
        return None
    e = p.get("configs", {}).get(_cfg_key(cfg))
    if not e or e.get("storage") != storage or e.get("links") != links or e.get("nrhs") != NRHS_W:
        return None
    return e["fetch_bytes_per_launch"] + e["write_bytes_per_launch"]


def roofline(lq, g0, lat, mc, prec, links, storage, cfg, stream, reps=48):
    """Average launch time (HIP events on `stream`) of the batched CG's
    dominant kernel -- the Wilson stencil q = M^dag t fused with the x and r
    updates and ||r||^2, over the 36 systems of one field, in the launch
    configuration the autotuner chose -- against the algorithmic bytes of one
    launch; the iteration's other stencil (t = M p + ||t||^2) beside it."""
    K, win = cfg
    out = {}
    for kern in (2, 0):
        ms = lq.time_dslash(g0, 0, mc["wilson"] + 0.1, precision=prec, links=links, nrhs=NRHS_W,
                            reps=reps, rhs_per_thread=K, window=win, stream=stream, kernel=kern)
        per_site = bytes_per_site(0, prec, links, NRHS_W, kern)
        out[kern] = (ms, per_site, per_site * lat.volume)
    ms, per_site, algo = out[2]
    achieved = algo / (ms * 1e-3) / 1e9
    ms0, per0, algo0 = out[0]
    pol = "Q16" if prec == lq.Q16 else "F32"
    traffic = stored_traffic(storage, links, cfg)
    if -16 <= win <= -11 and prec == lq.Q16:
        # the t-sweeping kernel of block orders -11 ... -16
        c = -win - 10
        how = (f"t-sweep, T = {2 << ((c - 1) % 3)} slices per block, x-y neighbours "
               f"{'from LDS' if c <= 3 else 'fetched'}")
        name, name0 = (f"wilson_tsweep_lo_kernel<{pol}, {links}, true, CG_UPDATE> ({how})",
                       f"wilson_tsweep_lo_kernel<{pol}, {links}, false, STORE_NORM> ({how})")
    else:
        name, name0 = (f"stencil_kernel<WilsonOpR1<{pol}, {links}, true>, CG_UPDATE, K={K}>",
                       f"stencil_kernel<WilsonOpR1<{pol}, {links}, false>, STORE_NORM>")
    return {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "traffic_scope": ("bytes leaving L2 per launch (FETCH_SIZE + WRITE_SIZE, scaled by a "
                          "256 MiB device copy), counted in this launch configuration; reads "
                          "served by the Infinity Cache are included"),
        "data": "pseudo-random fields, live solver state (alpha = 1)",
        "kernel": (f"{name}: "
                   f"q = M^dag t, r -= alpha q, ||r||^2, x += the four steps of the group every "
                   f"fourth launch; {NRHS_W} systems; average over the group"),
        "rhs_per_thread": K, "window": win,
        "avg_launch_us": round(ms * 1e3, 2),
        "algorithmic_bytes_per_site": per_site,
        "algorithmic_bytes_per_launch": int(algo),
        "other_stencil": {
            "kernel": f"{name0}: t = M p, ||t||^2",
            "avg_launch_us": round(ms0 * 1e3, 2),
            "algorithmic_bytes_per_site": per0,
            "achieved_GBs": round(algo0 / (ms0 * 1e-3) / 1e9, 1),
        },
    }


def summarize_profile(a, trace, fetch, write, cfetch, cwrite):
    """Profile summary of the dominant stencil: rocprofv3 kernel-trace stats and
    the FETCH_SIZE / WRITE_SIZE counters per dispatch, scaled by what the same
    counters read for a device copy of known size."""
    import csv
    import glob

    def rows(d, pat):
        f = glob.glob(os.path.join(d, "**", pat), recursive=True)
        if not f:
            raise SystemExit(f"no {pat} under {d}")
        with open(f[0]) as fh:
            return list(csv.DictReader(fh))

    def per_dispatch(d, counter, match):
        tot, ids = 0.0, set()
        for r in rows(d, "*counter_collection.csv"):
            if match(r["Kernel_Name"]) and r["Counter_Name"] == counter:
                tot += float(r["Counter_Value"])
                ids.add(r["Dispatch_Id"])
        return tot / len(ids), len(ids)

    stencil = lambda n: "stencil_kernel" in n or "tsweep_lo_kernel" in n
    stats = [r for r in rows(trace, "*kernel_stats.csv") if stencil(r["Name"])]
    copy_f, _ = per_dispatch(cfetch, "FETCH_SIZE", lambda n: "copyBuffer" in n)
    copy_w, _ = per_dispatch(cwrite, "WRITE_SIZE", lambda n: "copyBuffer" in n)
    fs, wsz = 256 << 20, 256 << 20
    fscale = fs / (copy_f * 1024.0)
    wscale = wsz / (copy_w * 1024.0)
    # the CG-update stencil: M^dag with epilogue 2 (one-site or t-sweeping kernel)
    dom = lambda n: (("stencil_kernel" in n and ", true>, 2," in n) or
                     ("tsweep_lo_kernel" in n and ", true, 2," in n))
    f_kib, nf = per_dispatch(fetch, "FETCH_SIZE", dom)
    w_kib, nw = per_dispatch(write, "WRITE_SIZE", dom)
    entry = {
        "storage": a.precision, "links": a.links, "rhs_per_thread": a.rhs_per_thread,
        "window": a.window, "nrhs": NRHS_W,
        "kernel_stats": stats,
        "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
        "copy_fetch_kib_per_256MiB": copy_f, "copy_write_kib_per_256MiB": copy_w,
        "fetch_scale": fscale, "write_scale": wscale,
        "fetch_bytes_per_launch": int(f_kib * 1024 * fscale),
        "write_bytes_per_launch": int(w_kib * 1024 * wscale),
        "dispatches_counted": [nf, nw],
    }
    # one entry per launch configuration, all taken on the same sources
    try:
        with open(PROFILE_JSON) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        doc = {}
    if doc.get("source_sha256") != stencil_source_hash() or "configs" not in doc:
        doc = {"source_sha256": stencil_source_hash(), "configs": {}}
    doc["scope"] = ("bytes leaving L2 (TCC FETCH_SIZE / WRITE_SIZE): HBM traffic plus "
                    "Infinity Cache hits")
    doc["configs"][_cfg_key((a.rhs_per_thread, a.window))] = entry
    with open(PROFILE_JSON, "w") as fh:
        json.dump(doc, fh, indent=1)
    print(json.dumps(entry, indent=1))


SERVING_DIMS = [(8, 8, 8, 16), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]


def serving(a, w):
    """Continuous batching: requests drawn over four lattice sizes (one
    resident near-identity field each, same spread as the workload), both
    formulations, delta in {0.02, 0.05, 0.1} above the workload's m_c, point
    or Z2 sources, tolerances log-uniform in [1e-10, 1e-6].  First all
    requests at once (capacity, solves/s), then Poisson arrivals at 50% and
    90% of that rate; p50/p99 latency from arrival to result."""
    import numpy as np
    import paper_1312_3265_amd as lq
    import synth
    from paper_1312_3265_amd import serve

    eps = w["eps"]
    mc = {0: w["m_c"]["wilson"], 1: w["m_c"]["staggered_wilson"]}
    fields = {d: synth.gauge_field(d, "near_identity", 3000 + i, eps)
              for i, d in enumerate(SERVING_DIMS)}
    descs = synth.serving_requests(a.serving_requests, seed=42, dims_choices=SERVING_DIMS,
                                   tol_range=(1e-10, 1e-6))
    sources = []
    for d in descs:
        f = d["formulation"]
        sources.append(synth.point_source(d["dims"], f, d["alpha"]) if d["source"] == "point"
                       else synth.z2_source(d["dims"], f, d["source_seed"]))
    opts = lq.solve_opts(precision=lq.Q16, links=12, poll_interval=16)

    def run(arrivals):
        reqs = [serve.Request(d["id"], d["dims"], d["formulation"], mc[d["formulation"]] + d["delta"],
                              src, d["tol"], arrival=float(t), maxiter=20000)
                for d, src, t in zip(descs, sources, arrivals)]
        srv = serve.SolveServer(fields, opts=opts, mem_budget=96 << 30, slots=a.serving_slots,
                                chunk=16, evenodd=a.serving_evenodd, min_pool=a.serving_min_pool)
        results = srv.run(reqs)
        rep = srv.report()
        rep.pop("groups", None)
        byid = {d["id"]: d for d in descs}
        rep["not_converged"] = [
            dict(dims=list(byid[r.id]["dims"]), formulation=byid[r.id]["formulation"],
                 delta=byid[r.id]["delta"], tol=byid[r.id]["tol"], status=r.info["status"],
                 iterations=r.info["iterations"], true_residual=r.info["true_residual"])
            for r in results if r.info["status"] != 0]
        return rep

    log("serving: warm-up (tuning every group)")
    run([0.0] * len(descs))
    cap = run([0.0] * len(descs))
    log(f"serving: capacity {cap['solves_per_s']:.2f} solves/s")
    out = {"requests": len(descs), "dims": [list(d) for d in SERVING_DIMS], "storage": "q16",
           "wilson_evenodd": bool(a.serving_evenodd), "slots_per_pool": a.serving_slots,
           "min_pool": a.serving_min_pool, "capacity": cap}
    for frac in (0.5, 0.9):
        rate = frac * cap["solves_per_s"]
        out[f"offered_{int(frac * 100)}pct"] = dict(
            offered_per_s=rate, **run(synth.poisson_arrivals(rate=rate, n=len(descs), seed=43)))
        log(f"serving: {int(frac * 100)}% done")
    return out


def evenodd_wilson(lq, fields, src, masses, dims, mc, prec, links, stream, t64w):
    """The Wilson part of the mix with and without even-odd preconditioning
    (the footnote to eq. (2), Sec. 3): the 36 systems of each of the 8 fields
    batched in the benchmark's storage, one batch at a time on one stream, and
    FP64 single-RHS on field 0 (t64w: the unpreconditioned FP64 seconds).  Both
    stop on eq. (2)'s residual ||b - A x|| / ||b|| <= TOL for the whole solution
    (b = M^dag chi), which is recomputed here in FP64 for every system."""
    import numpy as np
    import torch

    def eq2_residual(g, m, chi, x):
        b = lq.apply(g, 0, m, chi, op=lq.OP_MDAG, stream=stream)
        ax = lq.apply(g, 0, m, x, op=lq.OP_MDAGM, stream=stream)
        return float(torch.linalg.vector_norm(b - ax) / torch.linalg.vector_norm(b))

    n = len(masses[0])
    out = {}
    props0 = None
    for eo in (0, 1):
        opts = lq.solve_opts(precision=prec, links=links, poll_interval=16, use_graph=1,
                             evenodd=eo)
        ws = torch.empty(lq.solve_workspace_bytes(fields[0], 0, opts, n), dtype=torch.uint8,
                         device="cuda")
        tol = TOL
        lq.cg_solve_batch(fields[0], 0, masses[0], src[0], [tol] * n, opts=opts, stream=stream,
                          workspace=ws)
        torch.cuda.synchronize()
        t0 = time.time()
        res, its = [], []
        for g in fields:
            x, infos = lq.cg_solve_batch(g, 0, masses[0], src[0], [tol] * n, opts=opts,
                                         stream=stream, workspace=ws)
            if any(i["status"] != lq.OK for i in infos):
                raise RuntimeError(f"even-odd={eo}: a Wilson system did not converge")
            its.append([i["iterations"] for i in infos])
            res.append(x)
        torch.cuda.synchronize()
        el = time.time() - t0
        worst = max(eq2_residual(g, masses[0][k], src[0][k], x[k])
                    for g, x in zip(fields, res) for k in range(n))
        if worst > TOL:
            raise RuntimeError(f"even-odd={eo}: eq. (2) residual {worst:.2e} above {TOL}")
        props0 = res[0]
        out["evenodd" if eo else "unpreconditioned"] = {
            "solves_per_s": round(len(fields) * n / el, 2),
            "mean_iterations": round(float(np.mean(its)), 1),
            "worst_eq2_residual": worst,
        }
    # FP64 single-RHS, point source alpha = 0 on field 0
    opts = lq.solve_opts(evenodd=1)
    t64e, it64e = {}, {}
    for d in DELTAS:
        m = mc["wilson"] + d
        chi = src[0][DELTAS.index(d) * 12]
        lq.cg_solve(fields[0], 0, m, chi, TOL, opts=opts, stream=stream)
        torch.cuda.synchronize()
        ts = time.time()
        x, inf = lq.cg_solve(fields[0], 0, m, chi, TOL, opts=opts, stream=stream)
        torch.cuda.synchronize()
        t64e[str(d)] = time.time() - ts
        it64e[str(d)] = inf["iterations"]
        r = eq2_residual(fields[0], m, chi, x)
        if inf["status"] != lq.OK or r > TOL:
            raise RuntimeError(f"FP64 even-odd delta={d}: status {inf['status']}, residual {r:.2e}")
    rate0 = 3.0 / sum(t64w[str(d)] for d in DELTAS)
    rate1 = 3.0 / sum(t64e.values())
    out["speedup_batched"] = round(out["evenodd"]["solves_per_s"] /
                                   out["unpreconditioned"]["solves_per_s"], 2)
    # the two even-odd pairs of an iteration alone (HIP events), against their
    # algorithmic bytes per half site: a pair writes one odd and one even
    # site per system; links 2 x 4 x 2 directions of 24 B (16-bit 12-real)
    # or 72 B (FP32 18-real) per pair
    vec = 12 * {0: 16, 1: 8, 2: 4}[prec] + (4 if prec == lq.Q16 else 0)
    xv = 12 * (8 if prec == lq.Q16 else {0: 16, 1: 8}[prec])
    lk = 2 * 8 * (links // 2) * {0: 16, 1: 8, 2: 4}[prec]
    per = {3: n * (2 * vec + 3 * vec) + lk,                                  # p->w, (w, p)->t
           4: n * (2 * vec + 2 * vec + 2 * vec + 0.25 * (4 * vec + 2 * xv)) + lk}
    Vh = fields[0].lattice.volume // 2
    roof = {}
    for kern in (3, 4):
        ms = lq.time_dslash(fields[0], 0, mc["wilson"] + 0.1, precision=prec, links=links, nrhs=n,
                            reps=20, rhs_per_thread=1, window=0, stream=stream, kernel=kern)
        roof[kern] = ms
    def pair(k):
        gbs = per[k] * Vh / (roof[k] * 1e-3) / 1e9
        return {"avg_pair_us": round(roof[k] * 1e3, 1), "bytes_per_half_site": per[k],
                "achieved_GBs": round(gbs, 1), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4)}
    out["pairs"] = {"t = M^p + ||t||^2": pair(3), "M^dag t + CG update": pair(4)}
    out["fp64_single_rhs"] = {"solves_per_s_unpreconditioned": round(rate0, 2),
                              "solves_per_s_evenodd": round(rate1, 2),
                              "speedup": round(rate1 / rate0, 2), "iterations_evenodd": it64e}
    return out, props0


def spectrum_section(lq, g, dims, stream):
    """Fig. 1(c)'s observable on field 0: the eigenvalues of D_SW (m = 0)
    nearest a shift beside the low end of the physical branch (sigma = 0.45;
    that end lies near -m_c) and of the doubler branch (sigma = 1.55), by
    shift-invert Krylov-Schur (basis of 40, up to 8 restarts, FP64 inner
    solves of eq. (2) to 1e-10); each as [Re, Im, relative Ritz estimate],
    nearest first."""
    import synth
    v0 = synth.gaussian_field(dims, 1, 11)
    out = {}
    for sigma in (0.45, 1.55):
        t0 = time.time()
        ev, res = lq.spectrum(g, 1, 0.0, sigma, v0, steps=40, restarts=8, tol=1e-10,
                              stream=stream)
        out[str(sigma)] = {"seconds": round(time.time() - t0, 2), "basis": 40, "restarts_max": 8,
                           "nearest": [[round(float(z.real), 5), round(float(z.imag), 5),
                                        float("%.2g" % r)] for z, r in zip(ev[:10], res[:10])]}
    return out


def pion_section(lq, lat, props, masses, stream):
    """Fig. 1(a)'s observable for the Wilson part of field 0: the pion
    correlator of the 12 point-source propagators at each mass, its effective
    mass averaged over t in [L4/4, L4/2), and the device reduction's rate
    (propagator bytes read per second, HIP events on the stream)."""
    import numpy as np
    import torch
    L4 = lat.dims[3]
    out = {"m_eff_window": [L4 // 4, L4 // 2 - 1], "per_mass": []}
    for di, d in enumerate(DELTAS):
        p = props[12 * di:12 * di + 12]
        C, meff = lq.pion_correlator(lat, p, stream=stream)
        w = meff[L4 // 4:L4 // 2]
        out["per_mass"].append({"delta": d, "mass": masses[12 * di],
                                "m_eff": round(float(np.nanmean(w)), 5),
                                "m_pi2": round(float(np.nanmean(w)) ** 2, 5),
                                "C_over_C0": [round(float(c / C[0]), 8) for c in C[:L4 // 2 + 1]]})
    p = props[:12]
    reps = 20
    lq.pion_correlator(lat, p, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record()
        for _ in range(reps):
            lq.pion_correlator(lat, p, stream=stream)
        e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 12 * lat.volume * 12 * 16
    out["correlator_ms_incl_host_sync"] = round(ms, 4)
    out["correlator_GBs_incl_host_sync"] = round(nbytes / (ms * 1e-3) / 1e9, 1)
    return out


def matvec_rooflines(lq, U16, dims16, mc, stream, reps=50):
    """The FP64 single-system matvecs (the plain M^dag stencil, as the FP64
    solver and every reliable update launch it) at 16^3 x 32 (workload field 0)
    and 32^3 x 64 (that field repeated twice in every direction; the timing does
    not depend on the link values), where the working set no longer fits the
    256 MB Infinity Cache: Wilson, staggered Wilson from corners, and staggered
    Wilson on the fly (an application = the recursion's three level launches
    plus the operator's).  Average over `reps` applications (HIP events on the
    stream), against the algorithmic bytes and flops per site."""
    import numpy as np
    import torch
    out = {}
    for dims in (dims16, tuple(2 * d for d in dims16)):
        U = U16 if dims == dims16 else np.tile(U16, (2, 2, 2, 2, 1, 1, 1))
        lat = lq.Lattice(dims)
        g = lq.Gauge(lat, U, lq.FEAT_CORNERS, stream=stream)
        del U
        V = lat.volume
        key = "x".join(map(str, dims))
        out[key] = {}
        for name, form, g55 in (("wilson", 0, 0), ("staggered_wilson_corners", 1, 0),
                                ("staggered_wilson_onthefly", 1, 1)):
            m = mc["wilson" if form == 0 else "staggered_wilson"] + 0.1
            ms = lq.time_dslash(g, form, m, dagger=True, g55=g55, precision=lq.F64, links=12,
                                reps=reps, window=-3, stream=stream)
            by = bytes_per_site(form, 0, 12, 1, kernel=1, g55=g55)
            by18 = bytes_per_site(form, 0, 18, 1, kernel=1, g55=g55)
            gbs = by * V / (ms * 1e-3) / 1e9
            tfl = FLOPS_PER_SITE[name] * V / (ms * 1e-3) / 1e12
            out[key][name] = {
                "avg_application_us": round(ms * 1e3, 1),
                "algorithmic_bytes_per_site": by, "bytes_per_site_18real_links": by18,
                "achieved_GBs": round(gbs, 1), "frac_of_8TBs": round(gbs / HBM_PEAK_GBS, 4),
                "flops_per_site": FLOPS_PER_SITE[name], "achieved_TFLOPs": round(tfl, 2),
                "frac_of_fp64_peak": round(tfl / FP64_PEAK_TFLOPS, 4)}
            log(f"matvec {key} {name}: {ms * 1e3:.1f} us, {gbs:.0f} GB/s, {tfl:.2f} TFLOP/s")
        del g, lat
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out


def fp64_single_rhs_mix(lq, fields, src, masses, stream):
    """Plain FP64 CG (eq. (2), unpreconditioned) on every system of the mix,
    one system at a time: the baseline the mixed-precision batched rate is
    compared with.  Returns the rate, the FP64 iteration counts of source 0 on
    field 0 per delta, and the mean seconds and iterations per solve per
    formulation and delta over the whole mix."""
    import numpy as np
    import torch
    nsrc = {0: 12, 1: 3}
    lq.cg_solve(fields[0], 0, masses[0][0], src[0][0], TOL, stream=stream)   # warm
    torch.cuda.synchronize()
    secs = {"wilson": {}, "staggered_wilson": {}}
    its = {"wilson": {}, "staggered_wilson": {}}
    iters0 = {"wilson": {}, "staggered_wilson": {}}
    total, n = 0.0, 0
    for gi, g in enumerate(fields):
        for form, name in ((0, "wilson"), (1, "staggered_wilson")):
            for k in range(len(masses[form])):
                d = str(DELTAS[k // nsrc[form]])
                ts = time.time()
                x, inf = lq.cg_solve(g, form, masses[form][k], src[form][k], TOL, stream=stream)
                el = time.time() - ts
                if inf["status"] != lq.OK or inf["true_residual"] > TOL:
                    raise RuntimeError(f"FP64 field {gi} formulation {form} system {k}: {inf}")
                total += el
                n += 1
                secs[name].setdefault(d, []).append(el)
                its[name].setdefault(d, []).append(inf["iterations"])
                if gi == 0 and k % nsrc[form] == 0:
                    iters0[name][d] = inf["iterations"]
    mean = lambda dd: {d: float(np.mean(v)) for d, v in dd.items()}
    return dict(rate=n / total, systems=n, seconds=total, iterations_source0_field0=iters0,
                mean_seconds={k: mean(v) for k, v in secs.items()},
                mean_iterations={k: mean(v) for k, v in its.items()})


def paper_comparison(mv, fp64, kap):
    """The paper's cost comparison (Sec. 3, eqs. (3)-(4)) with measured
    numbers: W / SW ratios of the matvec time, the CG iteration count, the
    cost per iteration and the time per solve (FP64, single system), raw (the
    same lattice for both) and in eq. (4)'s convention, which multiplies a
    per-site ratio by 4 because the Wilson matrix is 4 times larger."""
    out = {"paper_estimates": {
        "cost_per_iteration_W_over_SW_flops_eq4": 3.2,
        "cost_per_iteration_W_over_SW_neighbour_count": 2.67,
        "matvec_speedup_assumed": "2-3", "cg_iteration_ratio": "about 2",
        "inversion_speedup": "4-6", "kappa_ratio": "about 4",
        "convention": "eq. (4): 4 x (per-site ratio); the raw figures below compare the "
                      "two matrices on the same lattice"}}
    mvr = {}
    for key, d in mv.items():
        w = d["wilson"]["avg_application_us"]
        mvr[key] = {}
        for form in ("staggered_wilson_corners", "staggered_wilson_onthefly"):
            raw = w / d[form]["avg_application_us"]
            mvr[key][form] = {"raw": round(raw, 3), "x4": round(4 * raw, 3)}
    out["matvec_time_ratio_W_over_SW_fp64"] = mvr
    it_r, iter_cost, solve = {}, {}, {}
    for d in map(str, DELTAS):
        iw, isw = fp64["mean_iterations"]["wilson"][d], fp64["mean_iterations"]["staggered_wilson"][d]
        tw, tsw = fp64["mean_seconds"]["wilson"][d], fp64["mean_seconds"]["staggered_wilson"][d]
        it_r[d] = round(iw / isw, 3)
        c = (tw / iw) / (tsw / isw)
        iter_cost[d] = {"raw": round(c, 3), "x4": round(4 * c, 3)}
        solve[d] = {"raw": round(tw / tsw, 3), "x4": round(4 * tw / tsw, 3)}
    out["cg_iteration_ratio_W_over_SW_fp64"] = it_r
    out["cost_per_iteration_ratio_W_over_SW_fp64"] = iter_cost
    out["solve_time_ratio_W_over_SW_fp64"] = solve
    out["kappa_lanczos200"] = {d: {k: round(v, 1) for k, v in kk.items()} for d, kk in kap.items()}
    out["kappa_ratio_W_over_SW"] = {d: round(kk["wilson"] / kk["staggered_wilson"], 2)
                                    for d, kk in kap.items()}
    return out


def _cpu_worker(args):
    """One host core's share of the all-cores oracle sample (a spawned process,
    one BLAS thread): the workload field, then n_w CG iterations of Wilson and
    n_sw of staggered Wilson at delta = 0.1 from point source alpha.  Returns
    the wall seconds of each, the closing true-residual application included."""
    alpha, n_w, n_sw = args
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import solvers
    w = load_workload()
    dims = tuple(w["dims"])
    out = {}
    with threadpool_limits(limits=1):
        U = synth.gauge_field(dims, "near_identity", w["seed"], w["eps"])
        for form, name, n in ((0, "wilson", n_w), (1, "staggered_wilson", n_sw)):
            M, Md, A = solvers.operator(form, U, w["m_c"][name] + 0.1)
            b = Md(synth.point_source(dims, form, alpha % (12 if form == 0 else 3)))
            t0 = time.time()
            solvers.cg(A, b, 1e-30, n)
            out[name] = time.time() - t0
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload):
    """The oracle timed on this host's cores on a bounded sample of the
    workload (run before the GPU is touched, so that the worker processes can
    be spawned):
      * one thread: the FP64 matvec of each formulation at 16^3 x 32, median
        of 5 (staggered Wilson by the oracle's subset recursion);
      * all cores (one process per core, one BLAS thread each, at most 16):
        2 Wilson and 1 staggered Wilson CG iterations per process at
        delta = 0.1, timed concurrently -> the aggregate seconds per iteration;
      * projected solves/s on the 360-system mix: the oracle's own FP64
        iteration counts at 16^3 x 32 (tests/golden/fullsize.json, equal to the
        GPU's) times that per-iteration cost, labelled as projected.
    The full oracle solves at delta = 0.1, measured when fullsize.json was
    written (build host, one thread each), are quoted beside it."""
    import multiprocessing as mp
    import statistics

    from threadpoolctl import threadpool_limits

    import synth
    from oracle import staggered_wilson, wilson

    w = workload
    dims = tuple(w["dims"])
    cores = min(len(os.sched_getaffinity(0)), 16)
    t_start = time.time()
    mv = {}
    with threadpool_limits(limits=1):
        U = synth.gauge_field(dims, "near_identity", w["seed"], w["eps"])
        for form, name, fn in ((0, "wilson", wilson.apply), (1, "staggered_wilson",
                                                            staggered_wilson.apply)):
            psi = synth.gaussian_field(dims, form, 3)
            m = w["m_c"][name] + 0.1
            ts = []
            for _ in range(5):
                t0 = time.time()
                fn(U, psi, m)
                ts.append(time.time() - t0)
            mv[name] = statistics.median(ts)
    del U
    n_w, n_sw = 2, 1
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(a, n_w, n_sw) for a in range(cores)], chunksize=1)
    # seconds per iteration of the whole pool: cores iterations run at once
    per_iter = {}
    for name, n in (("wilson", n_w), ("staggered_wilson", n_sw)):
        mean = sum(r[name] for r in res) / len(res)
        per_iter[name] = mean / (n + 1) / cores      # n iterations + 1 residual application
    with open(os.path.join(ROOT, "tests", "golden", "fullsize.json")) as f:
        gold = json.load(f)
    tot, nsys = 0.0, 0
    for name, per_field in (("wilson", 12), ("staggered_wilson", 3)):
        for d in DELTAS:
            it = gold["cg"][name][str(d)]["iterations"]
            tot += 8 * per_field * it * per_iter[name]
            nsys += 8 * per_field
    return dict(
        value=round(nsys / tot, 5), unit="solves/s", cores=cores, kind="oracle",
        cpu_model=cpu_model(), host_cpus=os.cpu_count(),
        sample=(f"oracle FP64 on this host: 2 Wilson + 1 staggered Wilson CG iterations at "
                f"16^3x32, delta=0.1, in each of {cores} processes at once (one BLAS thread "
                f"each); solves/s projected to the 360-system mix with the oracle's FP64 "
                f"iteration counts from tests/golden/fullsize.json"),
        projected=True,
        seconds_per_iteration_all_cores=per_iter,
        matvec_seconds_1thread_median5={k: round(v, 4) for k, v in mv.items()},
        # the oracle reads all 18 reals of each link; staggered Wilson by the
        # subset recursion reads no corners
        matvec_GBs_1thread={k: round(bytes_per_site(0 if k == "wilson" else 1, 0, 18, 1,
                                                     kernel=1, g55=1) * gold_volume(w) / v / 1e9, 3)
                            for k, v in mv.items()},
        full_solve_seconds_delta0_1_build_host={
            k: round(gold["cg"][k]["0.1"]["seconds"], 1) for k in ("wilson", "staggered_wilson")},
        full_solve_note=("measured when tests/golden/fullsize.json was written: one thread per "
                         "solve, six solves at once on an 8-core Xeon build host, not this box"),
        wall_seconds=round(time.time() - t_start, 1),
    )


def oracle_error(lq, g0, dims, mc, stream):
    """Per storage precision, the single-system solve of field 0's point
    source alpha = 0 at each mass against the oracle's FP64 solution x*, from
    its fingerprint in tests/golden/fullsize_solutions.json (written by the
    oracle alone): iterations, and the error on the 64 sampled sites and on
    the four seeded projections, each relative to ||x*||.  Two solutions that
    both meet eq. (2) at tol differ by at most 2 tol kappa ||x*|| (about)."""
    import numpy as np
    import torch

    import synth
    with open(os.path.join(ROOT, "tests", "golden", "fullsize_solutions.json")) as f:
        sols = json.load(f)
    V = int(np.prod(dims))
    out = {}
    for form, name in ((0, "wilson"), (1, "staggered_wilson")):
        chi = synth.point_source(dims, form, 0)
        vs = [torch.from_numpy(synth.gaussian_field(dims, form, s)).to("cuda")
              for s in sols["proj_seeds"]]
        out[name] = {}
        for d in DELTAS:
            ref = sols["solutions"][name][str(d)]
            nrm = float(np.sqrt(ref["norm2"]))
            sites = torch.as_tensor(ref["sites"], device="cuda")
            samp = torch.complex(torch.tensor(ref["samples_re"], dtype=torch.float64),
                                 torch.tensor(ref["samples_im"], dtype=torch.float64)).to("cuda")
            row = {"oracle_iterations": ref["iterations"]}
            for prec, pname in ((lq.F64, "f64"), (lq.F32, "f32"), (lq.Q16, "q16")):
                opts = lq.solve_opts(precision=prec, links=12)
                x, info = lq.cg_solve(g0, form, mc[name] + d, chi, TOL, opts=opts, stream=stream)
                torch.cuda.synchronize()
                e_s = float(torch.linalg.vector_norm(x.reshape(V, -1)[sites] - samp)) / nrm
                e_p = max(abs(complex(torch.vdot(v.reshape(-1), x.reshape(-1))) -
                              complex(pr, pi)) / (float(torch.linalg.vector_norm(v)) * nrm)
                          for v, pr, pi in zip(vs, ref["proj_re"], ref["proj_im"]))
                row[pname] = {"iterations": info["iterations"],
                              "true_residual": info["true_residual"],
                              "err_sampled": float(f"{e_s:.3e}"), "err_projections": float(f"{e_p:.3e}")}
            out[name][str(d)] = row
    return out


def gold_volume(w):
    v = 1
    for d in w["dims"]:
        v *= d
    return v


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="q16", choices=["f32", "q16"],
                    help="storage of the batched CG's stencil and Krylov vectors "
                         "(arithmetic is FP32, reductions and reliable updates FP64)")
    ap.add_argument("--links", type=int, default=12, choices=[12, 18],
                    help="link storage of the batched stencil (16-bit with q16): 18 = 18-real, "
                         "12 = 12-real in the vector storage")
    ap.add_argument("--links-sw", type=int, default=0, choices=[0, 12, 18],
                    help="link storage of the staggered Wilson batches (0: as --links)")
    ap.add_argument("--fields", type=int, default=8)
    ap.add_argument("--reliable-interval", type=int, default=0,
                    help="reliable update at least every this many iterations (0: library default)")
    ap.add_argument("--poll-interval", type=int, default=16)
    ap.add_argument("--reliable-delta", type=float, default=0.0,
                    help="reliable update once the iterated residual has dropped by this factor "
                         "(0: library default)")
    ap.add_argument("--concurrency", type=int, default=3,
                    help="batches (gauge field x formulation) in flight at once")
    ap.add_argument("--order", choices=["wilson-first", "interleave"], default="interleave",
                    help="order in which the batches are taken up (interleave: each Wilson "
                         "batch followed by the same field's staggered Wilson one)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving section at the end of the default run")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only time the dominant stencil (the launches a profiler should see)")
    ap.add_argument("--rhs-per-thread", type=int, default=1, help="with --roofline-only")
    ap.add_argument("--window", type=int, default=0, help="with --roofline-only")
    ap.add_argument("--matvec-only", action="store_true",
                    help="only the FP64 single-system matvecs at 16^3x32 and 32^3x64 (the "
                         "launches a profiler should see for their roofline entries)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device copy five times (counter calibration)")
    ap.add_argument("--serving", action="store_true",
                    help="only the continuous-batching measurement: Poisson arrivals over four "
                         "lattice sizes at 50%% and 90%% of the measured capacity")
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--serving-slots", type=int, default=8, help="with --serving: slots per pool")
    ap.add_argument("--serving-min-pool", type=int, default=1,
                    help="with --serving: slots a new pool asks for at least")
    ap.add_argument("--serving-evenodd", type=int, default=1, choices=[0, 1],
                    help="with --serving: Wilson requests solved even-odd preconditioned")
    ap.add_argument("--summarize-profile", nargs=5, metavar=("TRACE", "FETCH", "WRITE", "CFETCH", "CWRITE"),
                    help="write the profile summary of the dominant stencil from rocprofv3 output "
                         "directories (kernel trace, FETCH_SIZE, WRITE_SIZE of --roofline-only; "
                         "FETCH_SIZE, WRITE_SIZE of --copy-calibration)")
    a = ap.parse_args()
    if a.summarize_profile:
        summarize_profile(a, *a.summarize_profile)
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the workload is a single-GPU batch of "
              "independent solves; splitting it across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    w = load_workload()
    cpu = None
    if not (a.no_cpu or a.copy_calibration or a.serving or a.roofline_only or a.matvec_only):
        # before anything touches the GPU: the oracle's worker processes are spawned
        cpu = cpu_baseline(w)
        log(f"cpu baseline: {cpu}")

    import numpy as np
    import torch

    import paper_1312_3265_amd as lq
    import synth

    if a.copy_calibration:
        x = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 256 << 20, "copies": 5}), flush=True)
        return

    if a.serving:
        print(json.dumps({"serving": serving(a, w)}), flush=True)
        return
    dims = tuple(w["dims"])
    eps = w["eps"]
    mc = w["m_c"]
    seeds = w["batch_seeds"][: a.fields]
    prec = lq.F32 if a.precision == "f32" else lq.Q16
    links = a.links
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()

    if a.roofline_only:
        lat = lq.Lattice(dims)
        U = synth.gauge_field(dims, "near_identity", seeds[0], eps)
        g0 = lq.Gauge(lat, U, lq.FEAT_CORNERS | lq.FEAT_F32 | lq.FEAT_Q16, stream=stream)
        print(json.dumps({"roofline": roofline(lq, g0, lat, mc, prec, links, a.precision,
                                               (a.rhs_per_thread, a.window), stream)}), flush=True)
        return
    if a.matvec_only:
        U = synth.gauge_field(dims, "near_identity", seeds[0], eps)
        print(json.dumps({"matvec_fp64": matvec_rooflines(lq, U, dims, mc, stream)}), flush=True)
        return

    # ---------------------------------------------------------------- setup
    t0 = time.time()
    lat = lq.Lattice(dims)
    fields = []
    U0 = None
    for s in seeds:
        U = synth.gauge_field(dims, "near_identity", s, eps)
        if U0 is None:
            U0 = U
        fields.append(lq.Gauge(lat, U, lq.FEAT_CORNERS | lq.FEAT_F32 | lq.FEAT_Q16 | lq.FEAT_EO,
                               stream=stream))
    plaq = fields[0].plaquette(stream=stream)
    src = {}
    masses = {}
    for form, name, nsrc in ((0, "wilson", 12), (1, "staggered_wilson", 3)):
        chis, ms = [], []
        for d in DELTAS:
            for alpha in range(nsrc):
                chis.append(synth.point_source(dims, form, alpha))
                ms.append(mc[name] + d)
        src[form] = torch.from_numpy(np.stack(chis)).to("cuda")
        masses[form] = ms
    opts = lq.solve_opts(precision=prec, links=links, poll_interval=a.poll_interval, use_graph=1,
                         reliable_interval=a.reliable_interval, reliable_delta=a.reliable_delta)
    links_sw = a.links_sw or links
    opts_f = {0: opts, 1: lq.solve_opts(precision=prec, links=links_sw,
                                        poll_interval=a.poll_interval, use_graph=1,
                                        reliable_interval=a.reliable_interval,
                                        reliable_delta=a.reliable_delta)}
    # `concurrency` batches in flight, each on its own stream with its own
    # workspace: a batch's instruction-bound stencil then shares the device
    # with another batch's bandwidth-bound kernels
    workers = []
    for c in range(a.concurrency):
        wsc = {}
        for form in (0, 1):
            n = len(masses[form])
            wsc[form] = torch.empty(lq.solve_workspace_bytes(fields[0], form, opts_f[form], n),
                                    dtype=torch.uint8, device="cuda")
        workers.append((stream if c == 0 else torch.cuda.Stream(), wsc))
    torch.cuda.synchronize()
    log(f"setup {time.time() - t0:.1f}s plaquette {plaq:.4f} m_c {mc}")

    def one_step(record=None):
        import queue
        import threading
        tasks = queue.Queue()
        if a.order == "interleave":    # each Wilson batch beside a staggered Wilson one
            for gi in range(len(fields)):
                tasks.put((gi, 0))
                tasks.put((gi, 1))
        else:                          # longer Wilson batches first
            for form in (0, 1):
                for gi in range(len(fields)):
                    tasks.put((gi, form))
        done, errors = [], []

        def work(strm, wsc):
            while True:
                try:
                    gi, form = tasks.get_nowait()
                except queue.Empty:
                    return
                try:
                    x, infos = lq.cg_solve_batch(fields[gi], form, masses[form], src[form],
                                                 [TOL] * len(masses[form]), opts=opts_f[form],
                                                 stream=strm, workspace=wsc[form])
                    for k, inf in enumerate(infos):
                        if inf["status"] != lq.OK or inf["true_residual"] > TOL:
                            raise RuntimeError(f"field {gi} formulation {form} system {k}: {inf}")
                    done.append((gi, form, infos))
                except Exception as e:          # reported after the join
                    errors.append(e)
                    return

        th = [threading.Thread(target=work, args=wk) for wk in workers]
        for t in th:
            t.start()
        for t in th:
            t.join()
        if errors:
            raise errors[0]
        n = 0
        for gi, form, infos in done:
            for k, inf in enumerate(infos):
                if record is not None:
                    record.append((gi, form, k, inf["iterations"], inf["reliable_updates"]))
            n += len(infos)
        return n

    # every batch shape is tuned alone, before the concurrent workers start:
    # the autotuner times kernels on its own stream, and other batches
    # running meanwhile would decide its choice
    for form in (0, 1):
        lq.cg_solve_batch(fields[0], form, masses[form], src[form], [TOL] * len(masses[form]),
                          opts=opts_f[form], stream=workers[0][0], workspace=workers[0][1][form])
    torch.cuda.synchronize()
    log(f"tuned launch (K, window): wilson {lq.tuned_launch(fields[0], 0, prec, links, NRHS_W)}")
    for i in range(a.warmup):
        one_step()
        log(f"warmup step {i} done")
    rec = []
    torch.cuda.synchronize()
    t0 = time.time()
    nsolved = 0
    for i in range(a.steps):
        nsolved += one_step(rec if i == 0 else None)
        log(f"step {i} done")
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    value = nsolved / elapsed
    log(f"timed: {value:.2f} solves/s ({nsolved} solves in {elapsed:.2f} s)")

    # ------------------------------ FP64 single-RHS reference over the whole mix
    g0 = fields[0]
    fp64 = fp64_single_rhs_mix(lq, fields, src, masses, stream)
    fp64_rate = fp64["rate"]
    iters64 = fp64["iterations_source0_field0"]
    log(f"fp64 single-RHS: {fp64_rate:.2f} solves/s over {fp64['systems']} systems")
    mixed_iters = {"wilson": {}, "staggered_wilson": {}}
    mixed_ru = {"wilson": {}, "staggered_wilson": {}}
    for gi, form, k, it, ru in rec:
        if gi == 0:
            name = "wilson" if form == 0 else "staggered_wilson"
            d = str(DELTAS[k // (12 if form == 0 else 3)])
            mixed_iters[name].setdefault(d, []).append(it)
            mixed_ru[name].setdefault(d, []).append(ru)
    mixed_iters = {n: {d: float(np.mean(v)) for d, v in dd.items()} for n, dd in mixed_iters.items()}
    mixed_ru = {n: {d: float(np.mean(v)) for d, v in dd.items()} for n, dd in mixed_ru.items()}

    # ------------------ measurements beside the headline (the next rows)
    def beside(name, fn, *args):
        # a failure here is reported in the line, in place of that figure
        try:
            return fn(*args)
        except Exception as e:  # noqa: BLE001
            log(f"{name} failed: {e!r}")
            return {"error": repr(e)}

    eo_res = beside("even-odd", evenodd_wilson, lq, fields, src, masses, dims, mc, prec, links,
                    stream, fp64["mean_seconds"]["wilson"])
    eo_w, props0 = eo_res if isinstance(eo_res, tuple) else (eo_res, None)
    log(f"even-odd Wilson: {eo_w}")
    pion = (beside("pion", pion_section, lq, lat, props0, masses[0], stream)
            if props0 is not None else {"error": "no propagators"})
    spec = beside("spectrum", spectrum_section, lq, fields[0], dims, stream)
    log(f"spectrum: {spec}")
    oerr = beside("error vs oracle", oracle_error, lq, fields[0], dims, mc, stream)
    log(f"error vs oracle: {oerr}")

    # --------------------------------------------- dominant kernel roofline
    cfg = lq.tuned_launch(g0, 0, prec, links, NRHS_W)
    roof = roofline(lq, g0, lat, mc, prec, links, a.precision, cfg or (1, 2), stream)
    mv = beside("matvec rooflines", matvec_rooflines, lq, U0, dims, mc, stream)

    # -------------------------------------- condition numbers (paper context)
    kap = {}
    for d in DELTAS:
        kap[str(d)] = {}
        for form, name in ((0, "wilson"), (1, "staggered_wilson")):
            v0 = synth.gaussian_field(dims, form, w["v0_seed"])
            r = lq.condition_number(g0, form, mc[name] + d, v0, steps=200, stream=stream)
            kap[str(d)][name] = r["kappa"]
    paper = beside("paper comparison", paper_comparison, mv, fp64, kap) \
        if "error" not in mv else {"error": "no matvec figures"}
    # the serving loop of the continuous-batching row, after everything else
    # (its pools and fields are its own)
    serv = None
    if not a.no_serving:
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        serv = beside("serving", serving, a, w)

    line = {
        "metric": "CG solves/s + Dslash HBM GB/s vs peak, 16^3x32, mixed-prec batched vs FP64",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("16^3x32, 8 near-identity SU(3) fields (plaquette 0.594), "
                         "W 12 + SW 3 point sources x 3 masses m_c+{0.02,0.05,0.1}, "
                         "tol 1e-8, batched CG with FP64 reliable updates"),
            "systems_per_step": nsolved // a.steps,
            "storage": a.precision, "links": links, "links_staggered_wilson": links_sw,
            "batches_in_flight": a.concurrency,
            "reliable_interval": a.reliable_interval or "default", "poll_interval": a.poll_interval,
            "reliable_delta": a.reliable_delta or "default",
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp64_single_rhs": {
            "solves_per_s_same_mix": round(fp64_rate, 3),
            "measured_over": f"all {fp64['systems']} systems, one FP64 solve at a time",
            "speedup_mixed_batched_vs_fp64": round(value / fp64_rate, 2),
            "iterations_source0_field0": iters64,
            "mean_iterations": {n: {d: round(v, 1) for d, v in dd.items()}
                                for n, dd in fp64["mean_iterations"].items()},
            "mean_seconds": {n: {d: round(v, 4) for d, v in dd.items()}
                             for n, dd in fp64["mean_seconds"].items()},
        },
        "matvec_fp64": mv,
        "paper_comparison": paper,
        "serving": serv,
        "evenodd_wilson": eo_w,
        "pion_wilson_field0": pion,
        "spectrum_sw_field0": spec,
        "solution_error_vs_oracle_field0": oerr,
        "mixed_iterations_field0": mixed_iters,
        "mixed_reliable_updates_field0": mixed_ru,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
