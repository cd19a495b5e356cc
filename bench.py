"""Benchmarks of the coupled porous cascaded LB step on one MI355X.

Default (the headline line): natural convection in a square porous cavity,
4096 x 4096 nodes, Ra = 1e6, Da = 1e-4, porosity 0.4, Pr = 1, J = sigma = 1,
Ergun F_phi, FP32 deviation storage with FP32 arithmetic (--storage f32 for
FP64 arithmetic, f16 / mixed for the narrow modes); FP64 is used only in the
reductions.  One "step" is one time step of the whole path for every domain:
pull streaming + macroscopic values + boundary reconstruction + D2Q9 and
D2Q5 collisions + store, with the FP64 residual, mass and Nusselt reductions
every 100 steps (their cost is inside the timed region).  Populations are
resident in HBM before timing starts.  Prints one JSON line with a
`roofline` object (the step kernel against HBM: algorithmic bytes per node
update are the 14 populations read and written, 112 B FP32, 56 B FP16, 76 B
mixed, plus 4 B for a porosity field) and a `cpu_baseline` (the FP64 CPU
oracle on a bounded sample of the same workload on the host cores).

Other workloads (--workload):
  batch          256 cavities of 64^2..512^2 with drawn parameters, one context
  channel        2048^2 mixed-convection channel with a porosity map
  batch-steady   the batch run to steady state with retirement
  cavity-sweep   step throughput over Ra x Da x porosity at 1024^2 and 4096^2
  table1         the 27 cavities of Table 1 run to steady state
  table1-grid    grid study of the Da = 1e-6 rows of Table 1 (256^2, 511^2, 1021^2)
  models         cascaded vs MRT vs BGK collisions: step time and stability
  paper-channel  the channel of Section 3.1 against its closed form: the N_y
                 study, the Re family and the low-viscosity runs of Fig. 4
  sigma          hot-wall Nusselt number against time for several sigma (Fig. 7)
  net            the warm-start network's kernels: training step and inference
  warmstart      time to steady state from rest vs from the trained network
  oracle-timing  the CPU oracle's own speed (1 thread, all threads)
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("coupled CLB MLUPS & %HBM BW; time-to-steady-state (Nu err≤1e-4) plain vs learned")
HBM_PEAK_GBS = 8000.0
REDUCE_EVERY = 100


def code_only(text):
    """C++ source with comments removed and whitespace runs collapsed."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash():
    """Hash of the step kernels' code (comments and layout ignored)."""
    h = hashlib.sha256()
    for f in ("paper_2110_05943_amd/csrc/clb_kernels.hip", "paper_2110_05943_amd/csrc/clb_internal.h"):
        h.update(code_only(open(os.path.join(ROOT, f)).read()).encode())
    return h.hexdigest()[:16]


def profile_record(key):
    """The committed rocprofv3 counter summary of a workload's dominant step
    kernel (HBM bytes per launch; for FP32 also VALU counts), or None when the
    kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
    try:
        data = json.load(open(path))
    except (OSError, ValueError):
        return None
    rec = data.get(key)
    if not rec or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec


def measured_traffic(key):
    """HBM bytes per launch of the dominant step kernel, or None."""
    rec = profile_record(key)
    return rec.get("bytes_per_launch") if rec else None


def build_workload(args):
    """(list of domain parameter dicts, workload description, short key)."""
    from paper_2110_05943_amd import workloads
    if args.workload == "cavity":
        n = args.n
        cases = [workloads.cavity(n, Ra=1e6, Da=1e-4, phi=0.4, Pr=1.0, storage=args.storage)]
        desc = ("porous cavity natural convection %dx%d, Ra=1e6, Da=1e-4, phi=0.4, Pr=1, "
                "%s deviation storage" % (n, n, args.storage))
        return cases, desc, "cavity%d_%s" % (n, args.storage)
    if args.workload == "batch":
        args.count = args.count or 256
        cases = workloads.batch(count=args.count, seed=3, storage=args.storage)
        desc = ("%d porous cavities in one context, N in {64,128,256,512}, Ra 1e3..1e7, "
                "Da 1e-5..1e-1, phi 0.3..0.95, Pr {0.71,1,7}, sigma 0.8..1.2 (seed 3), "
                "%s deviation storage" % (args.count, args.storage))
        return cases, desc, "batch%d_%s" % (args.count, args.storage)
    n = args.n if args.n != 4096 else 2048
    cases = [workloads.hetero_channel(n, n, ell=32, seed=4, storage=args.storage)]
    desc = ("porous mixed-convection channel %dx%d, inlet/outlet, random porosity map "
            "(l=32, eps 0.3..0.9, mean Da=1e-3), Re=100, Ri=1, Pr=1, %s deviation storage"
            % (n, n, args.storage))
    return cases, desc, "channel%d_%s" % (n, args.storage)


def initial_state(solver, cases):
    from paper_2110_05943_amd import inputs
    for k, c in enumerate(cases):
        if c["bc"][0] == "wall_T":  # cavity: T = 0.5 + seeded noise
            solver.set_state(k, inputs.cavity_initial_T(c["nx"], seed=1, ny=c["ny"]))


def cpu_baseline(cases, steps):
    """The FP64 oracle (test infrastructure) on a bounded sample of the
    workload: `steps` steps of its domains, in order, until about 3e8 node
    updates are reached."""
    import numpy as np
    from paper_2110_05943_amd import inputs
    from tests.cases import oracle_lattice
    lus, dt, used = 0, 0.0, 0
    for c in cases:
        lat = oracle_lattice(c)
        if c["bc"][0] == "wall_T":
            lat.init_equilibrium(inputs.cavity_initial_T(c["nx"], seed=1, ny=c["ny"]))
        else:
            lat.init_equilibrium(c.get("T_init", 0.5))
        t0 = time.perf_counter()
        lat.step(steps)
        dt += time.perf_counter() - t0
        assert np.isfinite(lat.f[:9]).all()
        lus += c["nx"] * c["ny"] * steps
        used += 1
        if lus >= 3e8:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return {"value": round(lus / dt / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": "%d steps of %d of the %d domains (%.3g node updates), FP64, OpenMP, %.1f s"
                      % (steps, used, len(cases), lus, dt)}


WEIGHTS = os.path.join(ROOT, "paper_2110_05943_amd", "data", "warmstart_unet.npz")


def warmstart_bench(args):
    """Held-out cavities (128^2, random porosity maps and groups, seed 1) run
    to steady state twice: from rest and from the trained network's
    prediction.  Reports the time to steady state (hot-wall Nusselt number
    within 1e-4 of the from-rest final value) of both."""
    import numpy as np
    from paper_2110_05943_amd import inputs
    from paper_2110_05943_amd import warmstart as W
    from paper_2110_05943_amd.train_warmstart import load_weights
    weights = args.weights or WEIGHTS
    if not os.path.exists(weights):
        print("no trained weights at %s (python -m paper_2110_05943_amd.train_warmstart)"
              % weights, file=sys.stderr)
        sys.exit(2)
    count = args.count or 500
    sur = W.Surrogate(n=128)
    meta = load_weights(weights, sur.net)
    draws = inputs.warmstart_draws(count, seed=1)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    max_steps = args.max_steps if args.max_steps != 10_000_000 else 3_000_000
    r = W.evaluate(sur, draws, tol=WS_TOL, check_every=5000, max_steps=max_steps, log=log)
    summ = warmstart_summary(r, draws, max_steps)
    out = {
        "metric": "time-to-steady-state (Nu err<=1e-4): plain vs learned warm start",
        "value": summ["speedup_steps"],
        "unit": "x fewer steps (sum over held-out cavities settled in both runs)",
        "higher_is_better": True,
        "n_gpus": 1, "data": "synthetic", "dtype": "f64 arithmetic, f32 storage; bf16 network",
        "config": {"workload": "%d held-out porous cavities 128x128, Ra 1e3..1e7, Da 1e-5..1e-1, "
                               "Pr {0.71,1,7}, sigma 0.8..1.2, random porosity maps (seed 1)"
                               % count, "tol": WS_TOL, "check_every": 5000},
        "training": {k: meta[k] for k in ("train", "epochs", "train_s", "datagen_s")
                     if k in meta},
    }
    out.update(summ)
    print(json.dumps(out), flush=True)


# Round residual at which the warm-start comparisons stop a run.  The
# reference steady Nusselt number is the final value of the run from rest; at
# 1e-9 a run whose slowest thermal mode decays slowly can stop with its
# Nusselt number still about 1e-4 from steady (the per-step change is then
# below the tolerance), so two runs of one cavity may disagree by more than
# the 1e-4 the comparison resolves.  At 1e-10 they agree within 6e-5.
WS_TOL = 1e-10


def warmstart_summary(r, draws, max_steps):
    """Time-to-steady-state comparison of a warmstart.evaluate result.

    Time to steady state: steps after which the hot-wall Nusselt number stays
    within 1e-4 of the final value of the run from rest.  Cavities whose run
    from rest reached the step cap are reported (count) rather than dropped:
    `speedup_steps` is over the cavities that settle in both runs,
    `speedup_steps_censored` over all cavities with every unsettled or capped
    time counted at the cap.  The cavities are the same size, so the step
    sums are the node-update work.  The batch wall clock of each run ends
    with its slowest cavity (those at the cap, in both runs)."""
    import numpy as np
    sp = np.array([x if x is not None else -1 for x in r["settle_plain"]], dtype=float)
    sw = np.array([x if x is not None else -1 for x in r["settle_warm"]], dtype=float)
    capped_p = np.array(r["status_plain"]) != 0
    capped_w = np.array(r["status_warm"]) != 0
    ok = (sp > 0) & (sw > 0)
    # censored at the cap: a cavity whose run from rest reached the cap has no
    # reference steady value, so both runs count max_steps for it; a learned
    # run that does not settle on a settled reference counts max_steps
    cp = np.where(capped_p, max_steps, np.where(sp > 0, sp, max_steps))
    cw = np.where(capped_p, max_steps, np.where(sw > 0, sw, max_steps))
    dnu = np.abs(np.array(r["nu_warm"]) - np.array(r["nu_plain"]))
    return {
        "cavities": len(draws), "settled_both": int(ok.sum()),
        "capped": {"plain": int(capped_p.sum()), "learned": int(capped_w.sum())},
        "steps_to_steady": {"plain": int(sp[ok].sum()), "learned": int(sw[ok].sum())},
        "speedup_steps": round(float(sp[ok].sum() / sw[ok].sum()), 3) if ok.any() else None,
        "speedup_steps_censored": round(float(cp.sum() / cw.sum()), 3),
        "median_per_case_speedup": round(float(np.median(sp[ok] / sw[ok])), 3) if ok.any() else None,
        "wall_s": {"plain": round(r["wall_plain"], 2),
                   "learned": round(r["wall_warm"] + r["inference_s"], 2),
                   "inference": round(r["inference_s"], 3)},
        "speedup_wall": round(r["wall_plain"] / (r["wall_warm"] + r["inference_s"]), 3),
        "nu_learned_vs_plain": {"max_abs": float(np.nanmax(dnu[ok])) if ok.any() else None,
                                "within_1e-4": int((dnu[ok] <= 1e-4).sum())},
        "fallback_to_rest": r["fallback"],
        "prediction_rel_l2_median": round(float(np.median(r["pred_rel_l2"])), 4),
        "max_steps": max_steps}


def warmstart_leg(count=24, max_steps=2_000_000):
    """The bounded time-to-steady-state leg of the default line: the first
    `count` held-out cavities (128^2, seed 1, the batched sweep's parameter
    ranges) run to a round residual of 1e-10 (WS_TOL) from rest and from the trained
    network's prediction."""
    from paper_2110_05943_amd import inputs
    from paper_2110_05943_amd import warmstart as W
    from paper_2110_05943_amd.train_warmstart import load_weights
    if not os.path.exists(WEIGHTS):
        return None
    sur = W.Surrogate(n=128)
    meta = load_weights(WEIGHTS, sur.net)
    draws = inputs.warmstart_draws(count, seed=1)

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    r = W.evaluate(sur, draws, tol=WS_TOL, check_every=5000, max_steps=max_steps, log=log)
    out = {"metric": "time-to-steady-state (Nu err<=1e-4) plain vs learned",
           "workload": "%d held-out porous cavities 128x128, Ra 1e3..1e7, Da 1e-5..1e-1, "
                       "Pr {0.71,1,7}, sigma 0.8..1.2, random porosity maps (seed 1)" % count}
    out.update(warmstart_summary(r, draws, max_steps))
    out["network"] = {k: meta[k] for k in ("train", "epochs") if k in meta}
    return out


def table1_bench(args):
    """Table 1 of the paper: steady hot-wall Nusselt numbers of the porous
    cavity for Da = 1e-2, 1e-4, 1e-6 (grids 128^2, 192^2, 256^2 as in Section
    3.2), three Ra each and porosity 0.4, 0.6, 0.9, Pr = 1: 27 cavities in
    one context, run from rest until the change per step over 5000-step
    rounds is <= 1e-9 (or 1e7 steps)."""
    import numpy as np
    from paper_2110_05943_amd import WEST, Solver, inputs, workloads
    from paper_2110_05943_amd._binding import NOT_CONVERGED, OK
    grid = {1e-2: 128, 1e-4: 192, 1e-6: 256}
    ref = []
    for line in open(os.path.join(ROOT, "tests", "golden", "table1_present.txt")):
        if line.strip() and not line.startswith("#"):
            v = [float(x) for x in line.split()]
            for phi, nu in zip((0.4, 0.6, 0.9), v[2:]):
                ref.append((v[0], v[1], phi, nu))
    if args.da is not None:
        ref = [r for r in ref if abs(r[0] / args.da - 1) < 1e-9]
    cases = [workloads.cavity(grid[Da], Ra=Ra, Da=Da, phi=phi, Pr=1.0, storage=args.storage)
             for Da, Ra, phi, _ in ref]
    s = Solver(cases)
    for k, c in enumerate(cases):
        T = inputs.cavity_initial_T(c["nx"], seed=1)
        if args.init == "conduction":  # linear profile between the hot and cold walls
            T = T - 0.5 + (1.0 - np.arange(c["nx"]) / (c["nx"] - 1))[None, :]
        s.set_state(k, T)
    every, chunk, cap, tol = 5000, 500_000, args.max_steps, 1e-9
    steps = np.zeros(len(cases), dtype=np.int64)
    status = np.full(len(cases), NOT_CONVERGED)
    nu_last = np.full(len(cases), np.nan)
    done = 0
    t0 = time.perf_counter()
    while done < cap and np.any(status == NOT_CONVERGED):
        r = s.run(chunk, check_every=every, tol=tol, nu_side=WEST, max_records=chunk // every)
        live = status == NOT_CONVERGED
        steps[live] += r["steps"][live]
        fin = live & (r["status"] != NOT_CONVERGED)
        status[fin] = r["status"][fin]
        for k in np.nonzero(live)[0]:
            rec = r["nu"][k][np.isfinite(r["nu"][k])]
            if rec.size:
                nu_last[k] = rec[-1]
        done += chunk
        print("  %d steps, %d of %d steady, %.1f s" % (done, int((status == OK).sum()), len(cases),
                                                      time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    rows = []
    for k, (Da, Ra, phi, nu_p) in enumerate(ref):
        rows.append({"Da": Da, "Ra": Ra, "phi": phi, "grid": grid[Da], "nu": round(float(nu_last[k]), 5),
                     "nu_paper": nu_p, "dev_pct": round(100 * (nu_last[k] - nu_p) / nu_p, 3),
                     "steps": int(steps[k]), "status": {0: "steady", 4: "diverged",
                                                        6: "not steady"}.get(int(status[k]), "?")})
    dev = np.array([abs(r["dev_pct"]) for r in rows if r["status"] == "steady"])
    out = {"metric": "Table 1 steady mean Nusselt number, deviation from the paper's values",
           "value": round(float(np.median(dev)), 3) if dev.size else None,
           "unit": "% (median |deviation| over steady cases)", "higher_is_better": False,
           "n_gpus": 1, "data": "synthetic", "dtype": DTYPE[args.storage],
           "config": {"workload": "%d porous cavities of Table 1 in one context" % len(cases),
                      "tol": tol, "check_every": every, "max_steps": cap, "init": args.init},
           "wall_s": round(wall, 1), "steady": int((status == OK).sum()),
           "max_abs_dev_pct": round(float(dev.max()), 3) if dev.size else None, "rows": rows}
    print(json.dumps(out), flush=True)


def _prolong(a):
    """Field on n x n nodes (L = n - 1) onto 2n - 1 nodes (L doubled): even
    nodes copy, odd ones average their neighbours (bilinear)."""
    import numpy as np
    n = a.shape[0]
    b = np.empty((2 * n - 1, 2 * n - 1))
    b[::2, ::2] = a
    b[1::2, ::2] = 0.5 * (a[:-1] + a[1:])
    b[:, 1::2] = 0.5 * (b[:, :-2:2] + b[:, 2::2])
    return b


def table1_grid_bench(args):
    """Grid study of the Da = 1e-6 rows of Table 1 (phi = 0.6, Ra = 1e7,
    1e8, 1e9): the paper's 256^2 grid (L = 255), then L = 510 and L = 1020
    (511^2 and 1021^2 nodes), each finer run started from the coarser steady
    fields (bilinear prolongation; lattice velocities do not change with the
    grid under the scaling of Eq. 46) and run until the hot-wall Nusselt
    number changes by less than 2e-5 relative over `every` steps."""
    import numpy as np
    from paper_2110_05943_amd import WEST, Solver, inputs, workloads
    Ras, phi, Da = (1e7, 1e8, 1e9), 0.6, 1e-6
    paper = {1e7: 1.0786, 1e8: 3.0156, 1e9: 12.020}
    every = 100_000

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    fields, out_rows = None, []
    t0 = time.perf_counter()
    for n in (256, 511, 1021):
        cases = [workloads.cavity(n, Ra=Ra, Da=Da, phi=phi, Pr=1.0) for Ra in Ras]
        s = Solver(cases)
        for k in range(len(cases)):
            if fields is None:  # conduction profile
                T = inputs.cavity_initial_T(n, seed=1) - 0.5 + (1.0 - np.arange(n) / (n - 1))[None, :]
                s.set_state(k, T)
            else:
                u, v, T = (_prolong(f) for f in fields[k])
                s.set_state(k, T, u, v)
        nu_prev = np.full(len(cases), np.nan)
        steps = 0
        while steps < args.max_steps:
            s.step(every)
            steps += every
            nu = np.array(s.nusselt_all(WEST))
            rel = np.abs(nu - nu_prev) / nu
            log("L=%d %d steps Nu %s rel change %s (%.0f s)" % (n - 1, steps, np.array2string(nu, precision=5),
                np.array2string(rel, precision=2), time.perf_counter() - t0))
            nu_prev = nu
            if np.all(rel <= 2e-5):
                break
        fields = []
        for k in range(len(cases)):
            m = s.macros(k)
            fields.append((m["ux"], m["uy"], m["T"]))
        for k, Ra in enumerate(Ras):
            out_rows.append({"L": n - 1, "Ra": Ra, "nu": round(float(nu[k]), 5),
                             "dev_pct": round(100 * (nu[k] - paper[Ra]) / paper[Ra], 3),
                             "steps": steps, "last_rel_change": float(rel[k])})
        s.close()
    res = {}
    for Ra in Ras:
        v = [r["nu"] for r in out_rows if r["Ra"] == Ra]
        # observed order and Richardson extrapolation from the three grids
        p = float(np.log2(abs(v[0] - v[1]) / abs(v[1] - v[2]))) if v[1] != v[2] else None
        ext = v[2] + (v[2] - v[1]) / (2 ** p - 1) if p and p > 0 else None
        res["%g" % Ra] = {"nu_by_L": v, "paper": paper[Ra], "observed_order": p,
                         "extrapolated": ext}
    print(json.dumps({"metric": "Table 1 Da = 1e-6 grid study (phi = 0.6)", "rows": out_rows,
                      "by_Ra": res, "wall_s": round(time.perf_counter() - t0, 1)}), flush=True)


def batch_steady_bench(args):
    """The 256-cavity batch run from rest to steady state with retirement
    (clb_run): per-cavity steps to steady state, the aggregate update rate
    over the whole run, and the final hot-wall Nusselt numbers."""
    import numpy as np
    from paper_2110_05943_amd import WEST, Solver, inputs, workloads
    from paper_2110_05943_amd._binding import ERR_DIVERGED, NOT_CONVERGED, OK
    cases = workloads.batch(count=args.count or 256, seed=3, storage=args.storage)
    s = Solver(cases)
    for k, c in enumerate(cases):
        s.set_state(k, inputs.cavity_initial_T(c["nx"], seed=1))
    sizes = np.array([c["nx"] * c["ny"] for c in cases])
    every, chunk, cap = 5000, 100_000, 2_000_000
    steps = np.zeros(len(cases), dtype=np.int64)
    status = np.full(len(cases), NOT_CONVERGED)
    t0 = time.perf_counter()
    done = 0
    while done < cap and np.any(status == NOT_CONVERGED):
        r = s.run(chunk, check_every=every, tol=args.tol)
        live = status == NOT_CONVERGED
        steps[live] += r["steps"][live]
        fin = live & (r["status"] != NOT_CONVERGED)
        status[fin] = r["status"][fin]
        done += chunk
        print("  %d steps, %d steady, %d diverged, %.1f s" % (done, int((status == OK).sum()),
              int((status == ERR_DIVERGED).sum()), time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    s.synchronize()
    wall = time.perf_counter() - t0
    s.set_active(np.ones(len(cases), dtype=np.uint8))
    nu = s.nusselt_all(WEST)
    ok = status == OK
    lu = float((steps * sizes).sum())
    by_n = {}
    for n in sorted(set(c["nx"] for c in cases)):
        m = ok & (np.array([c["nx"] for c in cases]) == n)
        if m.any():
            by_n[str(n)] = {"steady": int(m.sum()), "median_steps": float(np.median(steps[m])),
                            "max_steps": int(steps[m].max())}
    out = {"metric": "batched run to steady state with retirement",
           "value": round(lu / wall / 1e6, 1), "unit": "MLUPS (aggregate over the run)",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic",
           "dtype": DTYPE[args.storage],
           "config": {"workload": "256 porous cavities (seed 3), from rest", "tol": args.tol,
                      "check_every": every, "max_steps": cap},
           "wall_s": round(wall, 1), "node_updates": lu, "steady": int(ok.sum()),
           "diverged": int((status == ERR_DIVERGED).sum()),
           "not_steady": int((status == NOT_CONVERGED).sum()), "by_size": by_n,
           "steps": steps.tolist(), "status": status.tolist(),
           "nu_hot": [round(float(v), 6) for v in nu]}
    print(json.dumps(out), flush=True)


def cavity_sweep_bench(args):
    """Throughput of the single-cavity step over the parameter sets Ra in
    {1e4, 1e6} x Da in {1e-2, 1e-4} x porosity in {0.4, 0.9} at 1024^2 and
    4096^2 (Pr = J = sigma = 1)."""
    import torch
    from paper_2110_05943_amd import Solver, inputs, workloads
    from paper_2110_05943_amd._binding import BYTES_PER_UPDATE
    rows = []
    for n in (1024, 4096):
        for Ra in (1e4, 1e6):
            for Da in (1e-2, 1e-4):
                for phi in (0.4, 0.9):
                    c = workloads.cavity(n, Ra=Ra, Da=Da, phi=phi, storage=args.storage)
                    s = Solver(c)
                    s.set_state(0, inputs.cavity_initial_T(n, seed=1))
                    s.step(50)
                    s.synchronize()
                    K = 400 if n == 4096 else 2000
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(s.stream)
                    s.step(K)
                    e1.record(s.stream)
                    e1.synchronize()
                    us = e0.elapsed_time(e1) * 1e3 / K
                    rows.append({"n": n, "Ra": Ra, "Da": Da, "phi": phi, "us_per_step": round(us, 2),
                                 "MLUPS": round(n * n / us, 1),
                                 "GBps": round(BYTES_PER_UPDATE[args.storage] * n * n / us / 1e3, 1)})
                    s.close()
                    print(rows[-1], file=sys.stderr, flush=True)
    print(json.dumps({"metric": "step throughput over parameter sets", "storage": args.storage,
                      "rows": rows}), flush=True)


def models_bench(args):
    """The cascaded method against its MRT (N = N_T = I) and single-rate
    (BGK) variants on the GPU: step time on the Table 2 case (Ra = 1e7,
    Da = 1e-4, phi = 0.6, 192^2) and on a 4096^2 grid, and how long each
    stays finite on cavities with relaxation times close to 1/2."""
    import numpy as np
    import torch
    from paper_2110_05943_amd import Solver, inputs, workloads
    from paper_2110_05943_amd._binding import ERR_DIVERGED
    out = {"metric": "collision models: step time and stability", "storage": args.storage,
           "cost": [], "stability": []}
    for n, K in ((192, 20000), (4096, 400)):
        base = None
        for model in ("bgk", "mrt", "clb"):
            c = workloads.cavity(n, Ra=1e7, Da=1e-4, phi=0.6, model=model, storage=args.storage)
            s = Solver(c)
            s.set_state(0, inputs.cavity_initial_T(n, seed=1))
            s.step(100)
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.step(K)
            e1.record(s.stream)
            e1.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / K
            base = base or us
            out["cost"].append({"n": n, "model": model, "us_per_step": round(us, 3),
                                "ratio_to_bgk": round(us / base, 3)})
            print(out["cost"][-1], file=sys.stderr, flush=True)
            s.close()
    configs = [(256, 1e9, 1e-6, 0.6), (256, 1e8, 1e-6, 0.6), (192, 1e7, 1e-4, 0.6),
               (128, 1e8, 1e-2, 0.9), (128, 1e9, 1e-4, 0.9)]
    steps, every = 1_000_000, 5000
    for model in ("clb", "mrt", "bgk"):
        cases = [workloads.cavity(n, Ra=Ra, Da=Da, phi=phi, model=model, storage=args.storage)
                 for n, Ra, Da, phi in configs]
        s = Solver(cases)
        for k, c in enumerate(cases):
            s.set_state(k, inputs.cavity_initial_T(c["nx"], seed=1))
        r = s.run(steps, check_every=every, tol=0.0)
        for k, (n, Ra, Da, phi) in enumerate(configs):
            tau = 1.0 / s_v_of(cases[k])
            out["stability"].append({"model": model, "n": n, "Ra": Ra, "Da": Da, "phi": phi,
                                     "tau_v": round(tau, 6),
                                     "diverged_after": int(r["steps"][k])
                                     if r["status"][k] == ERR_DIVERGED else None,
                                     "steps": int(r["steps"][k])})
            print(out["stability"][-1], file=sys.stderr, flush=True)
        s.close()
    print(json.dumps(out), flush=True)


def _channel_start(s, k, c):
    import numpy as np
    ny, nx, u1 = c["ny"], c["nx"], c["bc_v"][2]
    s.set_state(k, np.full((ny, nx), 0.5), np.zeros((ny, nx)), np.full((ny, nx), u1))


def _channel_errors(m, c):
    """Global relative errors of Eq. 45 against Eqs. 43-44 (u as a vector)."""
    import numpy as np
    from paper_2110_05943_amd import workloads
    from tests.closed_forms import paper_channel_exact
    ux_a, uy_a, T_a = paper_channel_exact(c)
    ux, uy, T = m["ux"][:, 0], m["uy"][:, 0], m["T"][:, 0]
    eu = np.sqrt(np.sum((ux - ux_a) ** 2 + (uy - uy_a) ** 2) / np.sum(ux_a ** 2 + uy_a ** 2))
    eT = np.sqrt(np.sum((T - T_a) ** 2) / np.sum(T_a ** 2))
    return float(eu), float(eT)


def paper_channel_bench(args):
    """The mixed-convection channel of Section 3.1 (periodic in x, injection
    through both plates, the y-acceleration of Eq. 42 per row) against its
    closed form, Eqs. 43-44:
      - the N_y study (s_v = 1, Re = 5, N_y = 17 .. 97 in one context);
      - the Re family on 32 x 32 with u0 = u1 = 0.01 (Fig. 2);
      - the low-viscosity runs of Fig. 4 (nu = 5e-4 and 1e-4, Re = 5,
        32 x 32) with the cascaded, MRT and BGK collisions, run until the
        change per step is <= 1e-10 or --max-steps."""
    import numpy as np
    from paper_2110_05943_amd import Solver, workloads
    from paper_2110_05943_amd._binding import ERR_DIVERGED, NOT_CONVERGED, OK
    out = {"metric": "Section 3.1 channel: global errors against Eqs. 43-44",
           "storage": args.storage, "ny_study": [], "re_family": [], "low_viscosity": []}

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    ns = (17, 25, 33, 49, 65, 97)
    cases = [workloads.paper_channel(n, s_v=1.0, Re=5.0, storage=args.storage) for n in ns]
    s = Solver(cases)
    for k, c in enumerate(cases):
        _channel_start(s, k, c)
    t0 = time.perf_counter()
    s.step(150_000)
    s.synchronize()
    log("N_y study: 150000 steps, %.1f s" % (time.perf_counter() - t0))
    for k, c in enumerate(cases):
        eu, eT = _channel_errors(s.macros(k), c)
        out["ny_study"].append({"ny": c["ny"], "E_u": eu, "E_T": eT})
        log(out["ny_study"][-1])
    s.close()
    fit = lambda key: float(-np.polyfit(np.log(ns), np.log([r[key] for r in out["ny_study"]]), 1)[0])
    out["slope_u"], out["slope_T"] = round(fit("E_u"), 3), round(fit("E_T"), 3)
    out["slope_paper"] = {"u": 2.032, "T": 1.996}

    res = (1.0, 5.0, 10.0, 20.0)
    cases = [workloads.paper_channel(32, nx=32, Re=Re, storage=args.storage) for Re in res]
    s = Solver(cases)
    for k, c in enumerate(cases):
        _channel_start(s, k, c)
    s.step(300_000)
    for k, c in enumerate(cases):
        eu, eT = _channel_errors(s.macros(k), c)
        out["re_family"].append({"Re": c["Re"], "tau_v": round(1.0 / s_v_of(c), 5), "E_u": eu,
                                 "E_T": eT})
        log(out["re_family"][-1])
    s.close()

    taus = (0.5015, 0.5003)  # nu = 5e-4, 1e-4
    chunk = 2_000_000
    for model in ("clb", "mrt", "bgk"):
        cases = [workloads.paper_channel(32, nx=32, s_v=1.0 / t, Re=5.0, model=model,
                                         storage=args.storage) for t in taus]
        s = Solver(cases)
        for k, c in enumerate(cases):
            _channel_start(s, k, c)
        status = np.full(len(cases), NOT_CONVERGED)
        steps = np.zeros(len(cases), dtype=np.int64)
        done, t0 = 0, time.perf_counter()
        while done < args.max_steps and np.any(status == NOT_CONVERGED):
            r = s.run(min(chunk, args.max_steps - done), check_every=20_000, tol=1e-10)
            live = status == NOT_CONVERGED
            steps[live] += r["steps"][live]
            fin = live & (r["status"] != NOT_CONVERGED)
            status[fin] = r["status"][fin]
            done += chunk
            log("  %s: %d steps, %.1f s" % (model, done, time.perf_counter() - t0))
        for k, c in enumerate(cases):
            row = {"model": model, "tau_v": taus[k], "nu": round((taus[k] - 0.5) / 3, 7),
                   "status": {OK: "steady", ERR_DIVERGED: "diverged",
                              NOT_CONVERGED: "not steady"}.get(int(status[k]), "?"),
                   "steps": int(steps[k])}
            if status[k] != ERR_DIVERGED:
                row["E_u"], row["E_T"] = _channel_errors(s.macros(k), c)
            out["low_viscosity"].append(row)
            log(row)
        s.close()
    print(json.dumps(out), flush=True)


def sigma_bench(args):
    """Fig. 7: the hot-wall mean Nusselt number against time for several
    heat-capacity ratios sigma; Ra = 1e5, Da = 1e-2, phi = 0.6, Pr = 1 on the
    128^2 grid that Section 3.2 uses for Da = 1e-2, from rest, one context,
    2e6 steps (over 4 times the longest settling time), Nu recorded every 1000
    steps.  At steady state sigma drops out of the energy equation, so the
    final Nusselt numbers should agree; a smaller sigma should settle sooner."""
    import numpy as np
    from paper_2110_05943_amd import WEST, Solver, inputs, workloads
    sigmas = (0.5, 1.0, 2.0, 4.0)
    every, cap = 1000, 2_000_000
    cases = [workloads.cavity(128, Ra=1e5, Da=1e-2, phi=0.6, Pr=1.0, sigma=sg,
                              storage=args.storage) for sg in sigmas]
    s = Solver(cases)
    for k in range(len(cases)):
        s.set_state(k, inputs.cavity_initial_T(128, seed=1))
    t0 = time.perf_counter()
    r = s.run(cap, check_every=every, tol=0.0, nu_side=WEST, max_records=cap // every)
    wall = time.perf_counter() - t0
    ru, rT, _, _ = s.residual_all()
    rows = []
    for k, sg in enumerate(sigmas):
        rec = r["nu"][k]
        rec = rec[np.isfinite(rec)]
        nu_inf = float(rec[-1])
        off = np.abs(rec - nu_inf)
        bad = np.nonzero(off > 1e-4)[0]
        settle = int((bad[-1] + 2) * every) if bad.size else every
        bad3 = np.nonzero(off > 1e-3 * nu_inf)[0]
        resp = int((bad3[-1] + 2) * every) if bad3.size else every
        rows.append({"sigma": sg, "nu_final": round(nu_inf, 7), "steps": int(r["steps"][k]),
                     "final_change_per_step": {"u": float(ru[k]), "T": float(rT[k])},
                     "steps_to_nu_within_1e-4": settle, "steps_to_nu_within_0.1pct": resp,
                     "nu_history": [round(float(v), 5) for v in rec[: 400: 10]]})
        print({k2: v for k2, v in rows[-1].items() if k2 != "nu_history"}, file=sys.stderr,
              flush=True)
    nus = [r_["nu_final"] for r_ in rows]
    print(json.dumps({"metric": "Fig. 7: hot-wall Nusselt number history against sigma",
                      "paper_steady_nu": 3.4429, "spread_final_nu": round(max(nus) - min(nus), 7),
                      "wall_s": round(wall, 1), "history_every_steps": every * 10,
                      "rows": rows}), flush=True)


def net_bench(args):
    """The warm-start network (nn.UNet, 1.97 M parameters) on its own: a
    training step (forward, MSE, backward, AdamW) on a batch of 32 inputs of
    128 x 128 x 16 channels, and inference of 500 inputs, timed with HIP
    events on the network's stream.  Algorithmic work: 2 * 9 * cin * cout
    flops per pixel and 3x3 convolution; the backward pass repeats it for the
    weight gradient and (except the first layer) the input gradient.  Inputs
    and targets are seeded random tensors of the warm-start shapes."""
    import numpy as np
    import torch
    from paper_2110_05943_amd import nn
    dev = torch.device("cuda:0")
    net = nn.UNet(device=dev, stream=torch.cuda.Stream(device=dev))
    r = np.random.Generator(np.random.PCG64(5))
    n = 128

    def conv_flops(B):
        fwd = dgrad = 0
        for st in net.steps:
            if st["op"] == "conv":
                a = st["ins"][0]
                f = 2 * 9 * net.ch[a] * st["out"] * B * (n >> net.lv[a]) ** 2
                fwd += f
                dgrad += f if a > 0 else 0
        return fwd, dgrad

    def timed(fn, reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(net.stream)
        for _ in range(reps):
            fn()
        e1.record(net.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    B = 32
    x = torch.tensor(r.standard_normal((B, n, n, 16)), dtype=torch.bfloat16, device=dev)
    tgt = torch.tensor(0.1 * r.standard_normal((B, n, n, 3)), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    def train_step():
        net.forward(x, B, n, n)
        net.backward(tgt, 3, B, n, n)
        net.adamw(1e-4)

    for _ in range(3):
        train_step()
    reps = max(args.steps // 40, 10)
    ms = timed(train_step, reps)
    fwd, dgrad = conv_flops(B)
    train_tf = (2 * fwd + dgrad) / ms / 1e9
    print("train: %.2f ms per step of %d, %.1f TFLOP/s" % (ms, B, train_tf), file=sys.stderr,
          flush=True)
    S = 500
    xi = torch.tensor(r.standard_normal((S, n, n, 16)), dtype=torch.bfloat16, device=dev)
    net.forward(xi, S, n, n)
    ms_inf = timed(lambda: net.forward(xi, S, n, n), 5)
    inf_tf = conv_flops(S)[0] / ms_inf / 1e9
    print("inference: %.2f ms for %d, %.1f TFLOP/s" % (ms_inf, S, inf_tf), file=sys.stderr,
          flush=True)
    print(json.dumps({
        "metric": "warm-start network: training samples/s and MFMA rate",
        "value": round(B / ms * 1e3, 1), "unit": "samples/s (training, batch 32, 128x128)",
        "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "dtype": "bf16 MFMA, fp32 accumulate",
        "config": {"workload": "U-Net 5 levels, widths 16..256, 1.97M parameters",
                   "batch": B, "grid": [n, n], "params": net.nparams},
        "ms_per_train_step": round(ms, 3), "inference_ms_500": round(ms_inf, 2),
        "roofline": {"bound": "mfma", "achieved": round(train_tf, 2), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(train_tf / 2500.0, 5),
                     "inference_achieved": round(inf_tf, 2),
                     "flops_per_train_step": 2 * fwd + dgrad}}), flush=True)


def s_v_of(case):
    from paper_2110_05943_amd import derive
    kw = {k: v for k, v in case.items() if k != "storage"}
    return derive(**kw)["s_v"]


def oracle_timing():
    """The FP64 CPU oracle's own speed on this host: one thread and all
    threads, 64^2 / 256^2 / 1024^2 cavities at fixed step counts."""
    import numpy as np
    from paper_2110_05943_amd import inputs, workloads
    from tests.cases import oracle_lattice
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    rows = []
    for n, steps in ((64, 5000), (256, 2000), (1024, 200)):
        c = workloads.cavity(n, Ra=1e5, Da=1e-2, phi=0.6)
        for threads in (1, cores):
            k = steps if threads > 1 or n == 64 else steps // 5
            lat = oracle_lattice(c, nthreads=threads)
            lat.init_equilibrium(inputs.cavity_initial_T(n, seed=1))
            t0 = time.perf_counter()
            lat.step(k)
            dt = time.perf_counter() - t0
            assert np.isfinite(lat.f[:9]).all()
            rows.append({"n": n, "steps": k, "threads": threads, "s": round(dt, 2),
                         "MLUPS": round(n * n * k / dt / 1e6, 3)})
            print(rows[-1], file=sys.stderr, flush=True)
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    print(json.dumps({"metric": "FP64 CPU oracle speed", "cpu": cpu, "cores": cores,
                      "rows": rows, "paper_clb_mlups_context": 3.5}), flush=True)


DTYPE = {"f32": "f64 arithmetic, f32 storage", "f32c": "f32 arithmetic, f32 storage",
         "f16": "f32 arithmetic, f16 storage",
         "mixed": "f32 arithmetic, f16 flow / f32 temperature storage"}
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9  # lane instructions per second (one wave64 op / 4 cycles / SIMD)
FP64_PEAK_TFLOPS = 78.6


def two_step_roofline(key, storage, nodes, step_ms, bytes_per_lu):
    """Roofline of the two-steps-per-launch kernel against HBM.

    Algorithmic bytes per node update are the 14 populations read and
    written once (bytes_per_lu: 112 B FP32, 56 B FP16, 76 B mixed); one
    launch updates every node twice, so it owes bytes_per_lu x 2 x nodes.
    `achieved` is that over the launch time measured here (HIP events on the
    solver stream), `frac` = achieved / 8 TB/s, which equals MLUPS x
    bytes_per_lu / 8e12.  Beside it:
    - traffic: HBM bytes per launch measured by rocprofv3 (FETCH_SIZE and
      WRITE_SIZE scaled by a plain copy), and traffic_frac, the same over the
      launch time against 8 TB/s;
    - valu: instruction issue, peak one wave64 VALU instruction per four
      cycles on each of the 1024 SIMDs at 2.4 GHz; the algorithmic count per
      node update is the one-step kernel's (which recomputes nothing);
    - fp64: FP64 flops per node update against the FP64 vector peak."""
    launch_s = 2 * step_ms * 1e-3
    single = profile_record("cavity4096_%s_single" % storage) or {}
    rec = profile_record(key) or {}
    gbps = bytes_per_lu * 2 * nodes / launch_s / 1e9
    out = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbps / HBM_PEAK_GBS, 4), "traffic": rec.get("bytes_per_launch"),
           "kernel": "step2_kernel", "kernel_us": round(launch_s * 1e6, 2),
           "steps_per_launch": 2, "bytes_per_node_update": bytes_per_lu,
           "node_updates_per_launch": 2 * nodes}
    if rec.get("bytes_per_launch"):
        out["traffic_frac"] = round(rec["bytes_per_launch"] / launch_s / 1e9 / HBM_PEAK_GBS, 4)
    if single.get("valu_instr_per_launch"):
        ops_lu = single["valu_instr_per_launch"] * 64 / single["nodes"]
        achieved = ops_lu * 2 * nodes / launch_s
        out["valu"] = {"achieved_TOPs": round(achieved / 1e12, 2),
                       "peak_TOPs": round(VALU_LANE_PEAK / 1e12, 2),
                       "frac": round(achieved / VALU_LANE_PEAK, 4),
                       "ops_per_node_update": round(ops_lu, 1)}
        if rec.get("valu_instr_per_launch"):
            out["valu"]["issued_frac"] = round(rec["valu_instr_per_launch"] * 64 / launch_s
                                               / VALU_LANE_PEAK, 4)
    if single.get("fp64_flops_per_launch"):
        flops_lu = single["fp64_flops_per_launch"] / single["nodes"]
        fp64 = flops_lu * 2 * nodes / launch_s / 1e12
        out["fp64"] = {"TFLOPs": round(fp64, 2), "frac": round(fp64 / FP64_PEAK_TFLOPS, 4),
                       "flops_per_node_update": round(flops_lu, 1)}
    return out


def preheat(s, min_s=0.15):
    """Untimed stepping between the warm-up and the timed region: captures
    the step graphs of both buffer parities and steps for at least min_s
    seconds, so that neither graph capture nor the clock ramp falls into the
    timed region.  Returns the steps taken (an even number: the parity of
    the state is unchanged)."""
    steps = 0
    for _ in range(2):  # one graph per parity
        s.step(66)
        s.step(1)
        steps += 67
    s.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_s:
        s.step(64)
        s.synchronize()
        steps += 64
    return steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", choices=("cavity", "batch", "channel", "warmstart", "table1",
                                           "table1-grid",
                                           "batch-steady", "cavity-sweep", "oracle-timing",
                                           "models", "paper-channel", "sigma", "net"),
                    default="cavity")
    ap.add_argument("--tol", type=float, default=1e-9,
                    help="batch-steady: change per step over 5000-step rounds")
    ap.add_argument("--da", type=float, default=None, help="table1: only the rows of this Da")
    ap.add_argument("--init", choices=("rest", "conduction"), default="rest",
                    help="table1: start from rest or from the conduction profile")
    ap.add_argument("--max-steps", type=int, default=10_000_000,
                    help="table1, paper-channel (low viscosity): step limit")
    ap.add_argument("--n", type=int, default=4096, help="grid size (cavity; channel: 2048)")
    ap.add_argument("--count", type=int, default=None,
                    help="domains of the batch (256) or warmstart (500) workload")
    ap.add_argument("--storage", choices=("f32", "f32c", "f16", "mixed"), default=None,
                    help="f32c: FP32 planes, FP32 arithmetic (default of the cavity, batch and "
                         "channel workloads); f32: FP32 planes, FP64 arithmetic (default of the "
                         "others)")
    ap.add_argument("--weights", default=None, help="warmstart: network weights (.npz)")
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warmstart", action="store_true",
                    help="leave out the time-to-steady-state leg of the default line")
    ap.add_argument("--autotune", action="store_true", help="time launch shapes first")
    ap.add_argument("--launch", type=str, default=None, help="tile_x,tile_y,blocks")
    ap.add_argument("--steps-per-launch", type=int, default=None, choices=(1, 2),
                    help="time steps per launch (default: the library's, 2 unless f16 storage "
                         "has a domain narrower than 128)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 10 times (counter calibration)")
    args = ap.parse_args()
    if args.storage is None:
        args.storage = "f32c" if args.workload in ("cavity", "batch", "channel") else "f32"
    if args.workload == "oracle-timing":
        return oracle_timing()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        x = torch.ones(2 ** 28, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        y.copy_(x)
        e0.record()
        for _ in range(10):
            y.copy_(x)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"copy_bytes_per_launch": 2 * x.numel() * 4,
                          "copy_GBps": round(2 * x.numel() * 4 / ms / 1e6, 1)}), flush=True)
        return
    if args.workload == "warmstart":
        return warmstart_bench(args)
    if args.workload == "table1":
        return table1_bench(args)
    if args.workload == "table1-grid":
        return table1_grid_bench(args)
    if args.workload == "batch-steady":
        return batch_steady_bench(args)
    if args.workload == "cavity-sweep":
        return cavity_sweep_bench(args)
    if args.workload == "paper-channel":
        return paper_channel_bench(args)
    if args.workload == "sigma":
        return sigma_bench(args)
    if args.workload == "net":
        return net_bench(args)
    if args.workload == "models":
        return models_bench(args)
    from paper_2110_05943_amd import WEST, Solver
    from paper_2110_05943_amd._binding import BYTES_PER_UPDATE

    cases, desc, key = build_workload(args)
    s = Solver(cases, device="cuda:0")
    initial_state(s, cases)
    if args.launch:
        s.set_launch(*[int(v) for v in args.launch.split(",")])
    if args.steps_per_launch is None:  # the library's default for this context
        args.steps_per_launch = s.get_steps_per_launch()[0]
    s.set_steps_per_launch(args.steps_per_launch)
    if args.autotune:
        s.autotune()
    shape = s.get_launch()
    s.step(args.warmup)
    pre = preheat(s)
    s.synchronize()
    torch.cuda.synchronize()

    K = args.steps
    events = []
    t0 = time.perf_counter()
    done = 0
    while done < K:
        chunk = min(REDUCE_EVERY, K - done)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.step(chunk)
        e1.record(s.stream)
        events.append((e0, e1, chunk))
        done += chunk
        ru, rT, mass, status = s.residual_all()
        nu = s.nusselt_all(WEST) if args.workload != "channel" else s.nusselt_all(2)
    s.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    kernel_ms = sum(a.elapsed_time(b) for a, b, _ in events) / K  # per time step
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    bytes_per_lu = BYTES_PER_UPDATE[args.storage] + (4 if cases[0].get("eps") is not None else 0)
    mlups = nodes * K / wall / 1e6
    if args.steps_per_launch == 2:
        roofline = two_step_roofline(key, args.storage, nodes, kernel_ms, bytes_per_lu)
    else:
        achieved = bytes_per_lu * nodes / (kernel_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic(key + "_single"),
                    "kernel": "step_kernel", "kernel_us": round(kernel_ms * 1e3, 2),
                    "bytes_per_node_update": bytes_per_lu}
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic",
        "config": {"workload": desc, "domains": len(cases), "nodes": nodes,
                   "storage": args.storage, "launch_shape": list(shape),
                   "steps_per_launch": args.steps_per_launch,
                   "two_step_tile_x": s.get_steps_per_launch()[1],
                   "reductions_every": REDUCE_EVERY, "preheat_steps": pre},
        "roofline": roofline,
        "state_check": {"res_u_max": float(max(ru)), "res_T_max": float(max(rT)),
                        "diverged": int((status != 0).sum()), "mass": float(sum(mass)),
                        "nu_first": float(nu[0])},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cases, args.cpu_steps)
    else:
        out["cpu_baseline"] = None
    s.close()
    if args.workload == "cavity" and not args.no_warmstart:
        # the metric's second half, on the learned warm start's own workload
        out["time_to_steady"] = warmstart_leg()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
