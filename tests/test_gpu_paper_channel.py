"""GPU runs of the mixed-convection channel of Section 3.1 (periodic in x,
moving hot top plate, injection through both plates, the y-acceleration of
Eq. 42 added per row by the library).

- parity with the FP64 oracle during the transient, alone and batched with a
  domain that has no per-row acceleration;
- second-order convergence to the closed form of Eqs. 43-44 (the N_y study of
  Section 3.1) and agreement with the oracle's steady state;
- the low-viscosity case of Fig. 4 (tau_v = 0.5015) stays bounded.
"""
import math
import sys

import numpy as np
import pytest

from paper_2110_05943_amd import inputs, workloads
from tests.cases import cavity, node_errors, node_tol, oracle_lattice, rel_l2, vel_rel_l2
from tests.closed_forms import paper_channel_exact

pytestmark = pytest.mark.gpu

TOL32 = 1e-6


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Solver():
    import torch
    assert torch.cuda.is_available(), "needs the MI355X"
    from paper_2110_05943_amd import Solver as S
    return S


def start(s, k, case):
    """T = 1/2, u = (0, u1) everywhere (as the oracle's init_equilibrium)."""
    ny, nx = case["ny"], case["nx"]
    u1 = case["bc_v"][2]
    s.set_state(k, np.full((ny, nx), 0.5), np.zeros((ny, nx)), np.full((ny, nx), u1))


def slope(ns, errs):
    return -np.polyfit(np.log(ns), np.log(errs), 1)[0]


def errors(m, case):
    ux_a, uy_a, T_a = paper_channel_exact(case)
    ux, uy, T = m["ux"][:, 0], m["uy"][:, 0], m["T"][:, 0]
    eu = math.sqrt(np.sum((ux - ux_a) ** 2 + (uy - uy_a) ** 2) / np.sum(ux_a ** 2 + uy_a ** 2))
    return eu, rel_l2(T, T_a)


@pytest.mark.parametrize("storage,tol", [("f32", TOL32), ("mixed", 1e-3)])
def test_paper_channel_transient_matches_oracle(Solver, storage, tol):
    """Re = 5, u0 = u1 = 0.01, 8 x 33 nodes, 3000 steps from T = 1/2."""
    case = workloads.paper_channel(33, nx=8, Re=5.0, storage=storage)
    log("paper channel 8x33 %s, 3000 steps" % storage)
    s = Solver(case)
    start(s, 0, case)
    lat = oracle_lattice(case)
    lat.init_equilibrium(0.5, ux=0.0, uy=case["bc_v"][2])
    s.step(3000)
    lat.step(3000)
    g, o = s.macros(), lat.macros()
    eu, eT = vel_rel_l2(g, o), rel_l2(g["T"], o["T"])
    nu_, nT = node_errors(g, o)
    log("rel-L2 u=%.3e T=%.3e  worst node u=%.3e T=%.3e" % (eu, eT, nu_, nT))
    assert eu <= tol and eT <= tol
    assert nu_ <= node_tol(tol) and nT <= node_tol(tol)


def test_row_acceleration_batched_with_plain_domain(Solver):
    """One launch advances a domain with a per-row acceleration and a cavity
    without one; each matches its own oracle."""
    cases = [workloads.paper_channel(25, nx=40, s_v=1.2, Re=10.0),
             cavity(48, Ra=1e4, Da=1e-2, phi=0.6)]
    log("batched channel 40x25 + cavity 48, 1500 steps")
    s = Solver(cases)
    start(s, 0, cases[0])
    T = inputs.cavity_initial_T(48, seed=2)
    s.set_state(1, T)
    lats = [oracle_lattice(c) for c in cases]
    lats[0].init_equilibrium(0.5, ux=0.0, uy=cases[0]["bc_v"][2])
    lats[1].init_equilibrium(T)
    s.step(1500)
    for k, lat in enumerate(lats):
        lat.step(1500)
        g, o = s.macros(k), lat.macros()
        eu, eT = vel_rel_l2(g, o), rel_l2(g["T"], o["T"])
        nu_, nT = node_errors(g, o)
        log("domain %d rel-L2 u=%.3e T=%.3e  worst node u=%.3e T=%.3e" % (k, eu, eT, nu_, nT))
        assert eu <= TOL32 and eT <= TOL32
        assert nu_ <= node_tol(TOL32) and nT <= node_tol(TOL32)


def test_paper_channel_second_order(Solver):
    """The N_y study of Section 3.1 (s_v = 1, Re = 5, Da = 0.01, phi = 0.6):
    six channel heights in one context, 120k steps (about 13 H^2 at the
    largest, well past steady state).  The slopes of the global errors of
    Eq. 45 against the closed form must lie within 0.25 of the paper's 2.032
    (u) and 1.996 (T); the two smallest heights must equal the oracle's
    steady state."""
    ns = (17, 25, 33, 49, 65, 97)
    cases = [workloads.paper_channel(n, s_v=1.0, Re=5.0) for n in ns]
    log("paper channel N_y study", ns)
    s = Solver(cases)
    for k, c in enumerate(cases):
        start(s, k, c)
    s.step(120_000)
    eu, eT = [], []
    for k, c in enumerate(cases):
        a, b = errors(s.macros(k), c)
        eu.append(a)
        eT.append(b)
        log("N_y=%d  E(u)=%.4e  E(T)=%.4e" % (c["ny"], a, b))
    su, sT = slope(ns, eu), slope(ns, eT)
    log("slopes u %.3f T %.3f" % (su, sT))
    assert abs(su - 2.032) < 0.25 and abs(sT - 1.996) < 0.25
    assert eu[-1] < 1e-3 and eT[-1] < 5e-3
    for k in (0, 1):
        lat = oracle_lattice(cases[k])
        lat.init_equilibrium(0.5, ux=0.0, uy=cases[k]["bc_v"][2])
        lat.step(20 * (ns[k] - 1) ** 2)
        g, o = s.macros(k), lat.macros()
        d_u, d_T = vel_rel_l2(g, o), rel_l2(g["T"], o["T"])
        nu_, nT = node_errors(g, o)
        log("N_y=%d steady state vs oracle: u %.3e T %.3e  worst node u=%.3e T=%.3e"
            % (ns[k], d_u, d_T, nu_, nT))
        assert d_u <= TOL32 and d_T <= TOL32
        assert nu_ <= node_tol(TOL32) and nT <= node_tol(TOL32)


def test_low_viscosity_channel_stays_bounded(Solver):
    """Fig. 4: nu = 5e-4 (tau_v = 0.5015), Re = 5, 32 x 32, past t = 2200."""
    tau = 0.5015
    case = workloads.paper_channel(32, nx=32, s_v=1.0 / tau, Re=5.0)
    log("low-viscosity channel 32x32 tau_v=%.4f, 3000 steps" % tau)
    s = Solver(case)
    start(s, 0, case)
    s.step(3000)
    m = s.macros()
    u1 = case["bc_v"][2]
    assert all(np.all(np.isfinite(v)) for v in m.values())
    assert np.max(np.abs(m["ux"])) < 10 * u1 and np.max(np.abs(m["uy"] - u1)) < 10 * u1
