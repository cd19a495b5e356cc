"""GPU: batched stepping with retirement (clb_run) against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

from paper_2110_05943_amd import inputs
from tests.cases import cavity, node_errors, node_tol, oracle_lattice, rel_l2, vel_rel_l2

pytestmark = pytest.mark.gpu

TOL32 = 1e-6


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "needs the MI355X"
    import paper_2110_05943_amd._binding as b
    return b


def check_state(g, o, tol, what):
    """Eq. 45 over the domain, and the worst single node against
    node_tol(tol)."""
    eu, eT = vel_rel_l2(g, o), rel_l2(g["T"], o["T"])
    nu_, nT = node_errors(g, o)
    log("%s rel-L2 u=%.3e T=%.3e  worst node u=%.3e T=%.3e" % (what, eu, eT, nu_, nT))
    assert eu <= tol and eT <= tol, (what, eu, eT)
    assert nu_ <= node_tol(tol) and nT <= node_tol(tol), (what, nu_, nT)


def test_run_retires_steady_and_diverged_domains(B):
    """Three domains in one context: a small cavity that becomes steady, a
    larger one that does not within the step limit, and one whose initial
    temperature holds a NaN.  Each retires with the right status after the
    right number of steps, and the states match the oracle run for exactly
    those steps."""
    small = cavity(17, Ra=1e3, Da=1e-2, phi=0.6)
    large = cavity(64, ny=48, Ra=1e5, Da=1e-3, phi=0.4, sigma=1.2)
    bad = cavity(20, Ra=1e4)
    T_small = inputs.cavity_initial_T(17, seed=1)
    T_large = inputs.cavity_initial_T(64, seed=2, ny=48)
    T_bad = inputs.cavity_initial_T(20, seed=3)
    T_bad[5, 5] = float("nan")
    s = B.Solver([small, large, bad])
    for k, T in enumerate((T_small, T_large, T_bad)):
        s.set_state(k, T)
    max_steps, every, tol = 8000, 100, 1e-5
    r = s.run(max_steps, check_every=every, tol=tol, nu_side=B.WEST, max_records=100)
    log("steps", r["steps"], "status", r["status"])
    assert r["status"][0] == B.OK and 0 < r["steps"][0] < max_steps
    assert r["steps"][0] % every == 0
    assert r["status"][1] == B.NOT_CONVERGED and r["steps"][1] == max_steps
    assert r["status"][2] == B.ERR_DIVERGED and r["steps"][2] == every
    nu = r["nu"]
    rounds0 = r["steps"][0] // every
    assert np.all(np.isfinite(nu[0, :rounds0])) and np.all(np.isnan(nu[0, rounds0:]))
    assert np.all(np.isfinite(nu[1, :80])) and np.all(np.isnan(nu[1, 80:]))
    # the last record of each running domain is the Nusselt number of its state
    assert nu[0, rounds0 - 1] == s.nusselt(0, B.WEST)
    assert nu[1, 79] == s.nusselt(1, B.WEST)

    lat0 = oracle_lattice(small)
    lat0.init_equilibrium(T_small)
    lat0.step(int(r["steps"][0]) - 1)
    prev = lat0.macros()
    lat0.step(1)
    o0 = lat0.macros()
    check_state(s.macros(0), o0, TOL32, "retired small cavity")
    # the oracle agrees that the small cavity is steady at this tolerance
    ro_T = rel_l2(o0["T"], prev["T"])
    log("oracle residual at retirement: T %.3e" % ro_T)
    assert ro_T <= 2 * tol
    assert abs(nu[0, rounds0 - 1] - lat0.nusselt(0, 1.0)) <= 1e-6

    lat1 = oracle_lattice(large)
    lat1.init_equilibrium(T_large)
    lat1.step(max_steps)
    check_state(s.macros(1), lat1.macros(), TOL32, "running large cavity")

    # retired domains stay frozen; the running one continues
    g0 = s.macros(0)
    s.step(200)
    assert np.array_equal(s.macros(0)["T"], g0["T"])
    lat1.step(200)
    check_state(s.macros(1), lat1.macros(), TOL32, "large cavity after 200 more steps")
    # set_active resumes a retired domain
    s.set_active([1, 0, 0])
    s.step(100)
    lat0.step(100)
    check_state(s.macros(0), lat0.macros(), TOL32, "resumed small cavity")
    s.close()


def test_retired_domain_keeps_its_state_under_odd_rounds(B):
    """Rounds of an odd number of steps flip the buffer parity each round.  A
    domain that retired still reads, and resumes from, the state it retired
    with: compared bit for bit with the same cavity run alone for the same
    steps (index 0 in both contexts, hence the same rounding words; FP32
    storage with FP64 arithmetic, where launch modes give identical bits)."""
    small = cavity(17, Ra=1e3, Da=1e-2, phi=0.6)
    large = cavity(48, Ra=1e5, Da=1e-3, phi=0.4)
    T_small = inputs.cavity_initial_T(17, seed=1)
    T_large = inputs.cavity_initial_T(48, seed=2)
    s = B.Solver([small, large])
    s.set_state(0, T_small)
    s.set_state(1, T_large)
    every, tol, cap = 333, 1e-5, 20 * 333
    r = s.run(cap, check_every=every, tol=tol)
    n0 = int(r["steps"][0])
    log("steps", r["steps"], "status", r["status"])
    assert r["status"][0] == B.OK and n0 < cap and r["status"][1] == B.NOT_CONVERGED
    if ((cap - n0) // every) % 2 == 0:  # make the parity flips after retirement odd
        s.run(every, check_every=every, tol=tol)
    alone = B.Solver(small)
    alone.set_state(0, T_small)
    alone.step(n0)
    a, b = s.macros(0), alone.macros()
    assert all(np.array_equal(a[k], b[k]) for k in a)
    # resumed, it continues from that state (the rounding words now follow
    # the context's later step index, so the two agree to the FP32 tolerance)
    s.set_active([1, 1])
    s.step(51)
    alone.step(51)
    a, b = s.macros(0), alone.macros()
    assert vel_rel_l2(a, b) <= TOL32 and rel_l2(a["T"], b["T"]) <= TOL32
    s.close()


def test_state_written_to_an_inactive_domain_survives_odd_steps(B):
    """clb_set_state on a stopped domain, then an odd number of steps of the
    other: the stopped domain still holds what was written."""
    s = B.Solver([cavity(24, Ra=1e3), cavity(32, Ra=1e4)])
    s.set_active([0, 1])
    s.set_state(0, inputs.cavity_initial_T(24, seed=5, amp=0.1))
    m0 = s.macros(0)
    s.step(7)
    m1 = s.macros(0)
    assert all(np.array_equal(m0[k], m1[k]) for k in m0)
    # likewise a checkpoint restored while the domain is stopped
    blob = s.get_state()
    s.set_active([1, 1])
    s.step(3)
    s.set_active([0, 1])
    s.put_state(blob)
    s.step(5)
    m2 = s.macros(0)
    assert all(np.array_equal(m0[k], m2[k]) for k in m0)
    s.close()


def test_run_argument_errors(B):
    s = B.Solver(cavity(16, Ra=1e3))
    for kw in (dict(check_every=0), dict(tol=-1.0), dict(tol=float("nan")),
               dict(nu_side=7, max_records=4)):
        with pytest.raises(B.CLBError) as e:
            s.run(100, **kw)
        assert e.value.status == B.ERR_ARG
    r = s.run(0)
    assert r["status"][0] == B.NOT_CONVERGED and r["steps"][0] == 0
    s.close()


def table1_present():
    """Table 1 "Present" column: {(Da, Ra): (Nu at phi 0.4, 0.6, 0.9)}."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "table1_present.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            v = [float(x) for x in line.split()]
            out[(v[0], v[1])] = tuple(v[2:])
    return out


def test_table1_steady_nusselt_128(B):
    """Steady mean Nusselt numbers of the porous cavity, 128^2, Da = 1e-2,
    phi = 0.6, Ra = 1e3, 1e4, 1e5 (Table 1), each with sigma = 0.8, 1, 1.2:
    nine cavities in one context.  The steady Nusselt number lies within 1% of
    the paper's values and does not depend on sigma (Section 3.2: sigma only
    changes the transient); a smaller sigma settles sooner (Fig. 7)."""
    ref = table1_present()
    Ras, sigmas = (1e3, 1e4, 1e5), (0.8, 1.0, 1.2)
    cases = [cavity(128, Ra=Ra, Da=1e-2, phi=0.6, sigma=sg) for Ra in Ras for sg in sigmas]
    s = B.Solver(cases)
    for k in range(len(cases)):
        s.set_state(k, inputs.cavity_initial_T(128, seed=1))
    every, steps = 1000, 300000
    r = s.run(steps, check_every=every, tol=0.0, nu_side=B.WEST, max_records=steps // every)
    assert np.all(r["status"] == B.NOT_CONVERGED)
    nu = r["nu"]
    final = nu[:, -1]
    ru, rT, _, st = s.residual_all()
    assert np.all(st == B.OK)
    for i, Ra in enumerate(Ras):
        paper = ref[(1e-2, Ra)][1]
        block = final[3 * i:3 * i + 3]
        # steps after which Nu stays within 1e-4 of its final value
        settle = []
        for k in range(3 * i, 3 * i + 3):
            off = np.nonzero(np.abs(nu[k] - final[k]) > 1e-4)[0]
            settle.append((off[-1] + 1 if off.size else 0) * every)
        log("Ra=%g Nu=%s paper=%.4f dev=%.3f%% sigma spread=%.2e settle(1e-4)=%s "
            "r_u=%s r_T=%s" % (Ra, np.array2string(block, precision=6), paper,
                               100 * (block.mean() - paper) / paper, np.ptp(block), settle,
                               np.array2string(ru[3 * i:3 * i + 3], precision=2),
                               np.array2string(rT[3 * i:3 * i + 3], precision=2)))
        assert np.all(np.abs(block - paper) <= 0.01 * paper)
        assert np.ptp(block) <= 1e-4
        assert settle[0] <= settle[1] <= settle[2]
        # steady: Nu stayed within 1e-4 of its final value over the last 50 000 steps
        tail = nu[3 * i:3 * i + 3, -50:]
        assert np.all(np.abs(tail - final[3 * i:3 * i + 3, None]) <= 1e-4)
    s.close()


def test_set_state_device_matches_host_warm_start(B):
    """clb_set_state_device (fields in device memory with a row stride, as a
    network writes them) gives the same populations as clb_set_state."""
    import torch
    from paper_2110_05943_amd import nn
    case = cavity(40, ny=24, Ra=1e4, sigma=1.1, T_init=0.25)
    u, v, T = inputs.random_fields(40, 24, seed=5, u_amp=0.02, T_amp=0.3)
    # values representable in FP32, so both paths see the same numbers
    u, v, T = (a.astype(np.float32).astype(np.float64) for a in (u, v, T))
    uc, T_off = 0.0625, 0.0  # scalings that keep every value exact in FP32
    a = B.Solver([cavity(8, Ra=1e3), case])
    a.set_state(1, T, u, v)
    fields = np.zeros((24 * 40, 16), dtype=np.float32)
    fields[:, 0] = (u / uc).ravel()
    fields[:, 1] = (v / uc).ravel()
    fields[:, 2] = (T - T_off).ravel()
    d = torch.tensor(fields).cuda()
    torch.cuda.synchronize()  # the copy ran on torch's stream, the solver has its own
    b = B.Solver([cavity(8, Ra=1e3), case])
    nn.call("clb_set_state_device", b._ctx, 1, nn.ptr(d), 16, uc, T_off)
    b.synchronize()
    assert np.array_equal(a.get_state(), b.get_state())
    a.step(50)
    b.step(50)
    assert np.array_equal(a.get_state(), b.get_state())


@pytest.fixture(scope="module")
def batch256_oracle():
    """The batched bench workload and the oracle's state of eight of its
    cavities (the largest, the smallest and six drawn ones) after 300 steps
    from the seeded initial state, each run by itself."""
    from paper_2110_05943_amd import workloads
    cases = workloads.batch(256, seed=3)
    sizes = np.array([c["nx"] for c in cases])
    pick = [int(np.argmax(sizes)), int(np.argmin(sizes))]
    pick += [int(k) for k in inputs.rng(77).choice(256, 6, replace=False) if k not in pick][:6]
    out = {}
    for k in pick:
        lat = oracle_lattice(cases[k])
        lat.init_equilibrium(inputs.cavity_initial_T(cases[k]["nx"], seed=1))
        lat.step(300)
        out[k] = lat.macros()
    return out


@pytest.mark.parametrize("storage", ["f32", "f32c"])
def test_batch256_workload_sampled_cavities(B, batch256_oracle, storage):
    """The batched bench workload (256 cavities, 64^2..512^2, drawn
    parameters) in its launch configuration, FP32 storage with FP64 or FP32
    arithmetic: 300 steps from the seeded initial state; eight cavities, the
    largest and smallest among them, against the oracle run by themselves."""
    from paper_2110_05943_amd import workloads
    cases = workloads.batch(256, seed=3, storage=storage)
    s = B.Solver(cases)
    for k, c in enumerate(cases):
        s.set_state(k, inputs.cavity_initial_T(c["nx"], seed=1))
    s.step(300)
    ru, rT, mass, st = s.residual_all()
    compared = diverged = 0
    for k, o in batch256_oracle.items():
        c = cases[k]
        if st[k] != B.OK:
            # a drawn cavity at the stability edge may diverge: then the
            # oracle must diverge too
            log("cavity %d (N=%d, Ra=%.3g) diverged on the GPU" % (k, c["nx"], c["Ra"]))
            assert not all(np.all(np.isfinite(v)) for v in o.values()), \
                "cavity %d diverged on the GPU only" % k
            diverged += 1
            continue
        check_state(s.macros(k), o, TOL32,
                    "batch %s [%d] N=%d Ra=%.3g Da=%.3g" % (storage, k, c["nx"], c["Ra"], c["Da"]))
        compared += 1
    log("batch %s: %d cavities compared, %d diverged on both sides" % (storage, compared, diverged))
    assert compared >= 6
    s.close()


@pytest.fixture(scope="module")
def cavity1024_oracle():
    case = cavity(1024, Ra=1e6, Da=1e-4, phi=0.4)
    lat = oracle_lattice(case)
    lat.init_equilibrium(inputs.cavity_initial_T(1024, seed=1))
    lat.step(2000)
    return lat.macros(), lat.nusselt(0, 1.0)


@pytest.mark.parametrize("storage", ["f32", "f32c"])
def test_cavity_1024_full_field(B, cavity1024_oracle, storage):
    """1024^2 cavity (Ra = 1e6, Da = 1e-4, phi = 0.4), 2000 steps from the
    seeded initial state (the parity window of the 1024^2 configuration),
    FP32 storage with FP64 or FP32 arithmetic: the whole field against the
    oracle."""
    case = cavity(1024, Ra=1e6, Da=1e-4, phi=0.4, storage=storage)
    s = B.Solver(case)
    s.set_state(0, inputs.cavity_initial_T(1024, seed=1))
    s.step(2000)
    o, nu_o = cavity1024_oracle
    check_state(s.macros(), o, TOL32, "cavity 1024 %s 2000 steps" % storage)
    assert abs(s.nusselt(0, B.WEST) - nu_o) <= 1e-4
    s.close()
