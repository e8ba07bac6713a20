"""GPU solver parity: mixed precision with FP64 reliable updates, batched
multi-RHS solves, continuous batching (alone vs in the mix), failure
statuses, and the m_c search.  Every solution is judged by the oracle's FP64
true residual ||b - A x|| / ||b||, b = M^dag chi (several x are correct;
the residual is unique)."""
import numpy as np
import pytest

import synth
from oracle import critical, solvers

pytestmark = pytest.mark.gpu

lq = pytest.importorskip("paper_1312_3265_amd")
torch = pytest.importorskip("torch")

DIMS = (8, 8, 6, 8)          # V = 3072: 12 site blocks of 256
EPS = 0.436
MASS = {synth.WILSON: -0.30, synth.STAGGERED_WILSON: -0.35}

_G = {}


def _field(dims=DIMS, seed=5):
    key = (dims, seed)
    if key not in _G:
        U = synth.gauge_field(dims, "near_identity", seed, EPS)
        lat = lq.Lattice(dims)
        _G[key] = (U, lat, lq.Gauge(lat, U))
    return _G[key]


def _res(form, U, chi, x, m):
    rn, _ = solvers.true_residual(form, U, chi, x.cpu().numpy(), m)
    return rn


@pytest.mark.parametrize("formulation", [synth.WILSON, synth.STAGGERED_WILSON])
@pytest.mark.parametrize("precision,links", [(lq.F32, 18), (lq.F32, 12), (lq.Q16, 12),
                                             (lq.Q16, 18)])
def test_mixed_precision_reaches_fp64_tolerance(formulation, precision, links):
    U, lat, g = _field()
    chi = synth.point_source(DIMS, formulation, 1)
    m, tol = MASS[formulation], 1e-8
    opts = lq.solve_opts(precision=precision, links=links, reliable_interval=50)
    x, info = lq.cg_solve(g, formulation, m, chi, tol, opts=opts)
    assert info["status"] == lq.OK, info
    assert info["reliable_updates"] >= 1
    rn = _res(formulation, U, chi, x, m)
    assert rn <= tol, (rn, info)
    x64, i64 = lq.cg_solve(g, formulation, m, chi, tol)
    err = (torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64)).item()
    print(f"prec={precision} links={links} iters={info['iterations']} "
          f"(fp64 {i64['iterations']}) ru={info['reliable_updates']} err_vs_fp64={err:.2e}")


def test_otf_gamma55_solve():
    U, lat, g = _field()
    chi = synth.point_source(DIMS, synth.STAGGERED_WILSON, 0)
    m, tol = MASS[synth.STAGGERED_WILSON], 1e-9
    xa, ia = lq.cg_solve(g, synth.STAGGERED_WILSON, m, chi, tol, g55=lq.G55_ONTHEFLY)
    xb, ib = lq.cg_solve(g, synth.STAGGERED_WILSON, m, chi, tol, g55=lq.G55_CORNERS)
    assert ia["status"] == lq.OK and ib["status"] == lq.OK
    assert _res(synth.STAGGERED_WILSON, U, chi, xa, m) <= tol
    assert abs(ia["iterations"] - ib["iterations"]) <= 2


@pytest.mark.parametrize("precision", [lq.F32, lq.Q16])
def test_otf_batched_low_precision_every_schedule(precision, monkeypatch):
    """Staggered Wilson batches with Gamma_55 on the fly (level launches per
    system, the last level shared by K systems per thread): every systems-per-
    thread choice gives bitwise the same solutions, each meeting eq. (2) by the
    oracle's FP64 residual."""
    U, lat, g = _field()
    form = synth.STAGGERED_WILSON
    chis = np.stack([synth.point_source(DIMS, form, a) for a in range(3)] +
                    [synth.z2_source(DIMS, form, 71)])
    ms = [MASS[form] + 0.03 * k for k in range(4)]
    opts = lq.solve_opts(precision=precision, links=12, poll_interval=8)
    ref = None
    for K in (1, 2, 4):
        monkeypatch.setenv("LQ_LAUNCH", f"{K},1")
        x, infos = lq.cg_solve_batch(g, form, ms, chis, [1e-8] * 4, opts=opts,
                                     g55=lq.G55_ONTHEFLY)
        assert all(i["status"] == lq.OK for i in infos), infos
        if ref is None:
            ref = x
            for k in range(4):
                assert _res(form, U, chis[k], x[k], ms[k]) <= 1e-8
        else:
            assert torch.equal(x, ref), K


def test_batched_multi_rhs_all_sources_and_masses():
    U, lat, g = _field()
    form = synth.WILSON
    chis, masses = [], []
    for alpha in (0, 4, 11):
        for dm in (0.0, 0.05):
            chis.append(synth.point_source(DIMS, form, alpha))
            masses.append(MASS[form] + dm)
    tol = 1e-8
    for opts in (lq.solve_opts(), lq.solve_opts(precision=lq.Q16, links=12)):
        x, infos = lq.cg_solve_batch(g, form, masses, np.stack(chis), [tol] * len(chis),
                                     opts=opts)
        for k in range(len(chis)):
            assert infos[k]["status"] == lq.OK
            assert _res(form, U, chis[k], x[k], masses[k]) <= tol


def test_batch_result_is_bitwise_the_single_result():
    """Each system's trajectory depends on its own state only (per-slot
    reliable updates, fixed-order reductions), so batching changes nothing."""
    U, lat, g = _field()
    form = synth.STAGGERED_WILSON
    chis = np.stack([synth.point_source(DIMS, form, a) for a in range(3)]
                    + [synth.z2_source(DIMS, form, 9)])
    masses = [MASS[form], MASS[form] + 0.1, MASS[form] + 0.02, MASS[form] + 0.05]
    tols = [1e-8, 1e-9, 1e-7, 1e-8]
    opts = lq.solve_opts(precision=lq.F32, links=12, reliable_interval=40)
    xb, ib = lq.cg_solve_batch(g, form, masses, chis, tols, opts=opts)
    for k in range(4):
        xs, is_ = lq.cg_solve(g, form, masses[k], chis[k], tols[k], opts=opts)
        assert is_["iterations"] == ib[k]["iterations"]
        assert torch.equal(xs, xb[k])


def test_continuous_batching_alone_vs_in_the_mix():
    """Requests admitted while others iterate give the same result as alone."""
    U, lat, g = _field()
    form = synth.WILSON
    opts = lq.solve_opts(precision=lq.Q16, links=12, reliable_interval=48, poll_interval=8)
    reqs = [(synth.point_source(DIMS, form, a), MASS[form] + d, t)
            for a, d, t in ((0, 0.0, 1e-8), (5, 0.05, 1e-7), (7, 0.1, 1e-9), (2, 0.02, 1e-8),
                            (9, 0.05, 1e-6))]
    alone = [lq.cg_solve(g, form, m, c, t, opts=opts) for c, m, t in reqs]
    b = lq.Batch(g, form, nslots=3, opts=opts)
    pending = list(range(len(reqs)))
    slot_of, results = {}, {}
    free = [0, 1, 2]
    guard = 0
    while pending or slot_of:
        while pending and free:
            k = pending.pop(0)
            s = free.pop(0)
            c, m, t = reqs[k]
            b.load(s, c, m, t)
            slot_of[s] = k
        states = b.step(16)
        for s, st in enumerate(states):
            if s in slot_of and st in (lq.SLOT_DONE, lq.SLOT_FAILED):
                results[slot_of.pop(s)] = b.fetch(s)
                free.append(s)
        guard += 1
        assert guard < 10000
    for k, (c, m, t) in enumerate(reqs):
        xm, im = results[k]
        xa, ia = alone[k]
        assert im["status"] == lq.OK
        assert im["iterations"] == ia["iterations"]
        assert torch.equal(xm, xa)
        assert _res(form, U, c, xm, m) <= t


def test_failure_statuses():
    U, lat, g = _field()
    form = synth.STAGGERED_WILSON
    chi = synth.point_source(DIMS, form, 0)
    x, info = lq.cg_solve(g, form, MASS[form], chi, 1e-12, maxiter=5)
    assert info["status"] == lq.NOT_CONVERGED and info["iterations"] == 5
    bad = chi.copy()
    bad[0, 0, 0, 1, 1] = np.nan
    with pytest.raises(lq.LQError) as e:
        lq.cg_solve(g, form, MASS[form], bad, 1e-8)
    assert e.value.code == lq.ERR_ARG


@pytest.mark.parametrize("formulation", [synth.WILSON, synth.STAGGERED_WILSON])
def test_critical_mass_matches_oracle_search(formulation):
    dims = (6, 6, 6, 6)
    U = synth.gauge_field(dims, "near_identity", 77, EPS)
    lat = lq.Lattice(dims)
    g = lq.Gauge(lat, U)
    v0 = synth.gaussian_field(dims, formulation, 7)
    mc, th = lq.critical_mass(g, formulation, v0, -0.8, -0.2, steps=80, ngrid=5, ngolden=4)
    mco, tho, _ = critical.critical_mass(formulation, U, v0, -0.8, -0.2, steps=80, ngrid=5,
                                         ngolden=4)
    assert abs(mc - mco) <= 1e-9
    assert abs(th - tho) <= 1e-6 * abs(tho) + 1e-12


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (16, 16, 4, 8)])
@pytest.mark.parametrize("precision", [lq.F32, lq.Q16])
@pytest.mark.parametrize("formulation", [synth.WILSON, synth.STAGGERED_WILSON])
def test_every_launch_schedule_gives_the_same_solution(formulation, precision, dims, monkeypatch):
    """Every block order and systems-per-thread choice covers each (site block,
    system) pair exactly once, so the batch's results are bitwise those of the
    plain order; 5 systems leave partial groups for K = 2 and 4.  8^4 has 16
    site blocks (windows of 1, 2, 4 differ); 16x16x4x8 has whole x-y planes of
    blocks, where the tiled orders -3 and -4 apply."""
    U, lat, g = _field(dims, 9)
    chis = np.stack([synth.point_source(dims, formulation, a) for a in range(3)] +
                    [synth.z2_source(dims, formulation, 70 + s) for s in range(2)])
    ms = [MASS[formulation] + 0.02 * k for k in range(5)]
    opts = lq.solve_opts(precision=precision, links=12, poll_interval=8)
    ref = None
    for K in (1, 2, 4):
        for w in (1, 2, 4, 0, -1, -2, -3, -4):
            monkeypatch.setenv("LQ_LAUNCH", f"{K},{w}")
            x, infos = lq.cg_solve_batch(g, formulation, ms, chis, [1e-8] * 5, opts=opts)
            assert all(i["status"] == lq.OK for i in infos)
            its = [i["iterations"] for i in infos]
            if ref is None:
                ref = (x, its)
                for k in range(5):
                    assert _res(formulation, U, chis[k], x[k], ms[k]) <= 1e-8
            else:
                assert its == ref[1], (K, w)
                assert torch.equal(x, ref[0]), (K, w)


@pytest.mark.parametrize("dims", [(16, 16, 4, 64), (32, 16, 4, 16)])
@pytest.mark.parametrize("links", [12, 18])
@pytest.mark.parametrize("precision", [lq.F32, lq.Q16])
def test_t_sweep_orders_give_the_same_solution(precision, links, dims, monkeypatch):
    """The t-sweeping Wilson CG stencils (block orders -11 ... -16: T = 2, 4, 8
    slices per block, x and y neighbours from LDS or fetched; 16-bit storage)
    do each site's arithmetic as the one-system stencil does, so every solution
    and iteration count is bitwise that of block order -3.  16x16x4x64 has
    256-site x-y planes (all six orders apply); on 32x16x4x16 (512-site planes)
    the LDS-neighbour orders fall back to the plain stencil and only T = 2 of
    the others fits, the rest falling back as well.  FP32 storage always falls
    back to the plain stencil."""
    U, lat, g = _field(dims, 9)
    form = synth.WILSON
    chis = np.stack([synth.point_source(dims, form, a) for a in range(3)] +
                    [synth.z2_source(dims, form, 70 + s) for s in range(2)])
    ms = [MASS[form] + 0.02 * k for k in range(5)]
    opts = lq.solve_opts(precision=precision, links=links, poll_interval=8)
    ref = None
    for w in (-3, -11, -12, -13, -14, -15, -16):
        monkeypatch.setenv("LQ_LAUNCH", f"1,{w}")
        x, infos = lq.cg_solve_batch(g, form, ms, chis, [1e-8] * 5, opts=opts)
        assert all(i["status"] == lq.OK for i in infos), (w, infos)
        its = [i["iterations"] for i in infos]
        if ref is None:
            ref = (x, its)
            for k in range(5):
                assert _res(form, U, chis[k], x[k], ms[k]) <= 1e-8
        else:
            assert its == ref[1], (w, its, ref[1])
            assert torch.equal(x, ref[0]), w


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (16, 16, 4, 8), (6, 4, 6, 8)])
@pytest.mark.parametrize("precision", [lq.F32, lq.Q16])
def test_lanes_stencil_is_bitwise_the_one_system_stencil(precision, dims, monkeypatch):
    """The Wilson stencils with four systems across the lanes of each site and
    the link products on the matrix cores (systems-per-thread code 8, 18-real
    links) reproduce the one-system-per-thread kernels bit for bit: the same
    FMA sequence for every link product (one MFMA step rounds like one FMA),
    the block partial sums in the same order.  5 systems leave a partial group
    of four; 6x4x6x8 has a ragged last site block."""
    U, lat, g = _field(dims, 9)
    form = synth.WILSON
    chis = np.stack([synth.point_source(dims, form, a) for a in range(3)] +
                    [synth.z2_source(dims, form, 70 + s) for s in range(2)])
    ms = [MASS[form] + 0.02 * k for k in range(5)]
    opts = lq.solve_opts(precision=precision, links=18, poll_interval=8)
    ref = None
    for K, w in ((1, 1), (8, 1), (8, 0), (8, -3), (8, -4), (8, 2)):
        monkeypatch.setenv("LQ_LAUNCH", f"{K},{w}")
        x, infos = lq.cg_solve_batch(g, form, ms, chis, [1e-8] * 5, opts=opts)
        assert all(i["status"] == lq.OK for i in infos), (K, w, infos)
        its = [i["iterations"] for i in infos]
        if ref is None:
            ref = (x, its)
            for k in range(5):
                assert _res(form, U, chis[k], x[k], ms[k]) <= 1e-8
        else:
            assert its == ref[1], (K, w, its, ref[1])
            assert torch.equal(x, ref[0]), (K, w)
    # a single system through the lanes stencil (three idle lanes per site)
    monkeypatch.setenv("LQ_LAUNCH", "8,1")
    x1, i1 = lq.cg_solve_batch(g, form, ms[:1], chis[:1], [1e-8], opts=opts)
    assert i1[0]["iterations"] == ref[1][0] and torch.equal(x1[0], ref[0][0])


def test_tuned_launch_and_stencil_timing():
    """The autotuner's choice is reported for the batch shape it tuned, and the
    three stencil timing modes run the solver's kernels."""
    import os
    if os.environ.get("LQ_LAUNCH"):
        pytest.skip("launch configuration forced from the environment")
    dims = (8, 8, 8, 8)
    U, lat, g = _field(dims, 9)
    chis = np.stack([synth.point_source(dims, synth.WILSON, a) for a in range(6)])
    opts = lq.solve_opts(precision=lq.Q16, links=12, poll_interval=8)
    x, infos = lq.cg_solve_batch(g, synth.WILSON, [-0.2] * 6, chis, [1e-8] * 6, opts=opts)
    assert all(i["status"] == lq.OK for i in infos)
    cfg = lq.tuned_launch(g, synth.WILSON, lq.Q16, 12, 6)
    assert cfg is not None and cfg[0] in (1, 2, 4) and (cfg[1] >= -4 or -16 <= cfg[1] <= -11)
    assert lq.tuned_launch(g, synth.WILSON, lq.F64, 0, 6) == (1, -3)
    for kern in (0, 1, 2):
        ms = lq.time_dslash(g, synth.WILSON, -0.2, precision=lq.Q16, links=12, nrhs=6, reps=3,
                            rhs_per_thread=cfg[0], window=cfg[1], kernel=kern)
        assert 0.0 < ms < 100.0


def test_critical_mass_of_the_frozen_workload():
    """The GPU search on the 16^3 x 32 workload field reproduces the m_c the
    oracle froze into tests/golden/workloads.json (same grid, same golden
    section, same start vector)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "workloads.json")) as f:
        w = json.load(f)
    dims = tuple(w["dims"])
    U = synth.gauge_field(dims, "near_identity", w["seed"], w["eps"])
    lat = lq.Lattice(dims)
    g = lq.Gauge(lat, U)
    assert abs(g.plaquette() - w["plaquette"]) < 1e-12
    for form, name in ((synth.WILSON, "wilson"), (synth.STAGGERED_WILSON, "staggered_wilson")):
        v0 = synth.gaussian_field(dims, form, w["v0_seed"])
        mc, th = lq.critical_mass(g, form, v0, -0.8, -0.2, steps=w["lanczos_steps"], ngrid=7,
                                  ngolden=6)
        assert abs(mc - w["m_c"][name]) <= 1e-9, (name, mc, w["m_c"][name])
        assert abs(th - w["theta_min_at_m_c"][name]) <= 1e-5 * abs(w["theta_min_at_m_c"][name])


def test_full_size_workload_batches_meet_eq2():
    """Field 0 of the 16^3 x 32 workload in the benchmark's launch
    configuration: the 36-system Wilson batch (12 point sources x 3 masses) and
    the 9-system staggered Wilson batch, 16-bit vectors and 12-real links.
    Every system converges; for one source per mass the oracle recomputes
    eq. (2)'s residual in FP64 and it meets tol and agrees with the library's."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "workloads.json")) as f:
        w = json.load(f)
    dims = tuple(w["dims"])
    U = synth.gauge_field(dims, "near_identity", w["seed"], w["eps"])
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_CORNERS | lq.FEAT_Q16)
    opts = lq.solve_opts(precision=lq.Q16, links=12, poll_interval=16)
    tol = 1e-8
    for form, name, nsrc in ((synth.WILSON, "wilson", 12),
                             (synth.STAGGERED_WILSON, "staggered_wilson", 3)):
        masses, chis = [], []
        for d in w["deltas"]:
            for a in range(nsrc):
                masses.append(w["m_c"][name] + d)
                chis.append(synth.point_source(dims, form, a))
        x, infos = lq.cg_solve_batch(g, form, masses, np.stack(chis), [tol] * len(chis),
                                     opts=opts)
        assert all(i["status"] == lq.OK and i["true_residual"] <= tol for i in infos)
        for j in range(len(w["deltas"])):
            k = j * nsrc + (j % nsrc)
            rn, _ = solvers.true_residual(form, U, chis[k], x[k].cpu().numpy(), masses[k])
            assert rn <= tol, (name, k, rn)
            assert abs(infos[k]["true_residual"] - rn) <= 1e-3 * tol


@pytest.mark.parametrize("formulation", [synth.WILSON, synth.STAGGERED_WILSON])
def test_grouped_x_update_keeps_every_step(formulation):
    """FP32 and 16-bit solves advance x once per group of four iterations,
    FP64 solves once per pair.  A solve cut off after n = 40..43 iterations
    stops at every position of a group, and its x must still hold all n
    steps: the FP32 result equals the FP64 iterate after n iterations to FP32
    roundoff.  With 16-bit storage, reliable updates land mid-group, and a
    step lost there would cost iterations: the count stays near FP64's."""
    U, lat, g = _field()
    chi = synth.point_source(DIMS, formulation, 2)
    m = MASS[formulation]
    o32 = lq.solve_opts(precision=lq.F32, links=18)
    x64 = {}
    for n in range(39, 44):
        x64[n], i64 = lq.cg_solve(g, formulation, m, chi, 1e-14, maxiter=n)
        assert i64["status"] == lq.NOT_CONVERGED and i64["iterations"] == n, i64
    norm = torch.linalg.vector_norm
    # a lost step would leave an error the size of one step
    step = min(norm(x64[n] - x64[n - 1]).item() for n in range(40, 44))
    for n in range(40, 44):
        x32, i32 = lq.cg_solve(g, formulation, m, chi, 1e-14, maxiter=n, opts=o32)
        assert i32["status"] == lq.NOT_CONVERGED and i32["iterations"] == n, i32
        err = norm(x32 - x64[n]).item()
        print(f"n={n} |x32 - x64|={err:.3e} smallest step={step:.3e}")
        assert err <= 0.02 * step, (n, err, step)
    tol = 1e-8
    x16, i16 = lq.cg_solve(g, formulation, m, chi, tol, opts=lq.solve_opts(precision=lq.Q16))
    _, i64 = lq.cg_solve(g, formulation, m, chi, tol)
    print(f"16-bit {i16['iterations']} iterations, {i16['reliable_updates']} reliable updates; "
          f"FP64 {i64['iterations']}")
    assert i16["status"] == lq.OK and i16["reliable_updates"] >= 2
    assert i16["iterations"] <= 1.1 * i64["iterations"] + 8, (i16, i64["iterations"])
    assert _res(formulation, U, chi, x16, m) <= tol


def test_full_size_fp64_iterations_and_kappa_match_oracle_golden():
    """The 16^3 x 32 workload field 0 (Sec. 3's lattice): plain FP64 CG on
    eq. (2) from the point source alpha = 0 at m_c + {0.02, 0.05, 0.1} takes the
    oracle's iteration counts (tests/golden/fullsize.json, written by the
    oracle alone) to within 2%, and the 200-step Lanczos estimates of
    theta_min, theta_max and kappa of (D+m)^dag (D+m) from the same start
    vector agree with the oracle's."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(here, "workloads.json")) as f:
        w = json.load(f)
    with open(os.path.join(here, "fullsize.json")) as f:
        gold = json.load(f)
    dims = tuple(w["dims"])
    U = synth.gauge_field(dims, "near_identity", w["seed"], w["eps"])
    g = lq.Gauge(lq.Lattice(dims), U)
    for form, name in ((synth.WILSON, "wilson"), (synth.STAGGERED_WILSON, "staggered_wilson")):
        chi = synth.point_source(dims, form, 0)
        v0 = synth.gaussian_field(dims, form, gold["v0_seed"])
        for d in w["deltas"]:
            m = w["m_c"][name] + d
            x, info = lq.cg_solve(g, form, m, chi, gold["tol"])
            it_o = gold["cg"][name][str(d)]["iterations"]
            print(f"{name} delta={d}: iterations {info['iterations']} (oracle {it_o})")
            assert info["status"] == lq.OK and info["true_residual"] <= gold["tol"]
            assert abs(info["iterations"] - it_o) <= max(2, 0.02 * it_o)
            k = lq.condition_number(g, form, m, v0, steps=gold["lanczos_steps"])
            lo = gold["lanczos"][name][str(d)]
            print(f"  kappa {k['kappa']:.6g} (oracle {lo['kappa']:.6g})")
            assert abs(k["lmax"] - lo["theta_max"]) <= 1e-9 * lo["theta_max"]
            assert abs(k["lmin"] - lo["theta_min"]) <= 1e-6 * lo["theta_min"]
            assert abs(k["kappa"] - lo["kappa"]) <= 1e-6 * lo["kappa"]


def _solution_errors(x, ref, form, dims):
    """(sampled error, projection error) of x against the oracle fingerprint ref,
    both relative to ||x*||: the components at ref's sites, and the projections
    on ref's seeded Gaussian fields."""
    V = int(np.prod(dims))
    xs = x.reshape(V, -1)
    sites = torch.as_tensor(ref["sites"], device=x.device)
    samp = torch.complex(torch.tensor(ref["samples_re"], dtype=torch.float64),
                         torch.tensor(ref["samples_im"], dtype=torch.float64)).to(x.device)
    nrm = float(np.sqrt(ref["norm2"]))
    e_samp = float(torch.linalg.vector_norm(xs[sites] - samp)) / nrm
    e_proj = 0.0
    for s, pr, pi in zip(ref["proj_seeds"], ref["proj_re"], ref["proj_im"]):
        v = torch.from_numpy(synth.gaussian_field(dims, form, s)).to(x.device)
        d = complex(torch.vdot(v.reshape(-1), x.reshape(-1))) - complex(pr, pi)
        e_proj = max(e_proj, abs(d) / (float(torch.linalg.vector_norm(v)) * nrm))
    return e_samp, e_proj


@pytest.mark.timeout(600)
def test_full_size_solutions_match_the_oracle_in_every_precision():
    """16^3 x 32 workload field 0, point source alpha = 0, both formulations at
    m_c + {0.02, 0.05, 0.1}: FP64, FP32 and 16-bit solves of eq. (2) at tol 1e-8
    against the oracle's own FP64 solution x* (its fingerprint in
    tests/golden/fullsize_solutions.json, written by the oracle alone).  Two
    solutions that both meet eq. (2) at tol differ by at most
    2 tol kappa (1 + tol kappa) ||x*|| (kappa of A = (D+m)^dag (D+m), the
    oracle's 200-step Lanczos value); the error on the 64 sampled sites and on
    the four seeded projections, each relative to ||x*||, must stay within it.
    The errors are printed per precision."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    with open(os.path.join(here, "workloads.json")) as f:
        w = json.load(f)
    with open(os.path.join(here, "fullsize.json")) as f:
        gold = json.load(f)
    with open(os.path.join(here, "fullsize_solutions.json")) as f:
        sols = json.load(f)
    dims = tuple(w["dims"])
    U = synth.gauge_field(dims, "near_identity", w["seed"], w["eps"])
    g = lq.Gauge(lq.Lattice(dims), U, lq.FEAT_CORNERS | lq.FEAT_F32 | lq.FEAT_Q16)
    tol = sols["tol"]
    for form, name in ((synth.WILSON, "wilson"), (synth.STAGGERED_WILSON, "staggered_wilson")):
        chi = synth.point_source(dims, form, 0)
        for d in w["deltas"]:
            m = w["m_c"][name] + d
            ref = dict(sols["solutions"][name][str(d)], proj_seeds=sols["proj_seeds"])
            kappa = gold["lanczos"][name][str(d)]["kappa"]
            bound = 2 * tol * kappa * (1 + tol * kappa)
            for prec in (lq.F64, lq.F32, lq.Q16):
                opts = lq.solve_opts(precision=prec, links=12)
                x, info = lq.cg_solve(g, form, m, chi, tol, opts=opts)
                assert info["status"] == lq.OK and info["true_residual"] <= tol
                es, ep = _solution_errors(x, ref, form, dims)
                print(f"{name} delta={d} precision={prec}: iterations {info['iterations']} "
                      f"(oracle {ref['iterations']}), error vs oracle: sampled {es:.2e}, "
                      f"projections {ep:.2e} (bound {bound:.1e})")
                assert es <= bound and ep <= bound, (name, d, prec, es, ep, bound)
