"""GPU against closed forms, independently of the oracle: flows whose steady
state the equations fix exactly, so that a boundary or forcing mistake shared
by both implementations would still show.

- uniform Darcy-Forchheimer flow in a periodic box (Eqs. 4, 21-23 at F = 0);
- pure conduction between isothermal walls (T linear, Nu = 1; walls on the
  nodes, L = n - 1, the boundary reconstruction, the Nusselt discretisation);
- the Darcy-Brinkman channel (cosh profile), second order in the height;
- plane Poiseuille flow between an inlet and an outlet side.
FP32 storage; tolerances allow its rounding noise (~1e-7 relative).  The
lattice constants of the closed forms (nu, K, F_phi) come from the oracle's
derivation of the parameters, not from the library's.
"""
import math
import sys

import numpy as np
import pytest

from tests.cases import oracle_values

pytestmark = pytest.mark.gpu

PERIODIC = ("periodic",) * 4


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "needs the MI355X"
    import paper_2110_05943_amd._binding as b
    return b


def test_uniform_darcy_forchheimer_flow(B):
    # At the fixed point F = 0: (phi F_phi / sqrt K) u^2 + (phi nu / K) u = phi a.
    base = dict(nx=64, ny=64, bc=PERIODIC, s_v=1.2, zeta_a=1.0, phi=0.5, Da=8.0 / 63 ** 2,
                a=(2e-4, 0.0), Ra=0.0, T_init=0.5)
    cases = [dict(base, F_phi=0.6), dict(base, F_phi=0.0)]
    s = B.Solver(cases)
    s.step(20000)
    for k, c in enumerate(cases):
        v = oracle_values(c)  # nu, K and F_phi by the oracle's own derivation
        nu, K, Fp, ax = v["nu"], v["K"], v["Fphi"], c["a"][0]
        if Fp > 0:
            b = Fp / math.sqrt(K)
            u = (-(nu / K) + math.sqrt((nu / K) ** 2 + 4 * b * ax)) / (2 * b)
        else:
            u = ax * K / nu  # Brinkman limit
        m = s.macros(k)
        err = np.max(np.abs(m["ux"] - u)) / u
        log("F_phi=%.2f: u exact %.8e, max rel err %.2e, max |v| %.1e"
            % (Fp, u, err, np.max(np.abs(m["uy"]))))
        assert err < 1e-6 and np.max(np.abs(m["uy"])) < 1e-6 * u


def test_pure_conduction_cavity(B):
    n = 33
    c = dict(nx=n, ny=n, bc=("wall_T", "wall_T", "wall_adiabatic", "wall_adiabatic"),
             bc_T=(1.0, 0.0, 0.0, 0.0), s_v=1.1, zeta_a=1.0, phi=0.6, Da=30.0 / (n - 1) ** 2,
             F_phi=0.3, Ra=0.0, T_init=0.5)
    s = B.Solver(c)
    s.step(80000)
    m = s.macros()
    x = np.arange(n)[None, :] * np.ones((n, 1))
    dT = np.max(np.abs(m["T"] - (1 - x / (n - 1))))
    nu_w, nu_e = s.nusselt(0, B.WEST), s.nusselt(0, B.EAST)
    log("max |T - linear| %.2e, Nu west %.8f east %.8f, max |u| %.1e"
        % (dT, nu_w, nu_e, np.max(np.abs(m["ux"]))))
    assert dT < 1e-6
    assert abs(nu_w - 1.0) < 2e-5 and abs(nu_e - 1.0) < 2e-5
    assert np.max(np.abs(m["ux"])) < 1e-7


def test_darcy_brinkman_channel_second_order(B):
    # u(y) = (a K / nu) [1 - cosh(r (y - H/2)) / cosh(r H / 2)], r = sqrt(phi / (J K))
    ns, phi, Da = (17, 33, 65), 0.6, 0.01
    cases = []
    for ny in ns:
        H = ny - 1
        K = Da * H * H
        nu = (1 / 1.0 - 0.5) / 3.0
        cases.append(dict(nx=8, ny=ny, bc=("periodic", "periodic", "wall_T", "wall_T"),
                          bc_T=(0.0, 0.0, 0.5, 0.5), scaling="channel", s_v=1.0, zeta_a=1.0,
                          phi=phi, Da=Da, F_phi=0.0, a=(1e-3 * nu / K, 0.0), Ra=0.0,
                          T_init=0.5))
    s = B.Solver(cases)
    s.step(150000)
    errs = []
    for k, (c, ny) in enumerate(zip(cases, ns)):
        v = oracle_values(c)
        H, K, nu = ny - 1, v["K"], v["nu"]
        r = math.sqrt(phi / K)
        y = np.arange(ny)
        exact = c["a"][0] * K / nu * (1 - np.cosh(r * (y - H / 2)) / np.cosh(r * H / 2))
        u = s.macros(k)["ux"]
        assert np.max(np.abs(u - u[:, :1])) < 1e-9  # uniform along x
        errs.append(np.linalg.norm(u[:, 0] - exact) / np.linalg.norm(exact))
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    log("errors %s, slope %.3f" % (["%.3e" % e for e in errs], slope))
    assert errs[-1] < 1e-3
    assert 1.8 < slope < 2.3


def test_inlet_outlet_poiseuille_flow(B):
    # The developed parabolic inflow stays parabolic: shape, pressure gradient
    # 12 nu U / H^2 (p = rho c_s^2) and one mass flux through every column.
    nx, ny, U = 49, 17, 0.02
    c = dict(nx=nx, ny=ny, bc=("inlet", "outlet", "wall_T", "wall_T"), bc_T=(0.5, 0.5, 0.5, 0.5),
             inlet_U=U, scaling="channel", s_v=1.0, zeta_a=1.0, phi=1.0, Da=0.0, F_phi=0.0,
             Ra=0.0, T_init=0.5)
    s = B.Solver(c)
    s.step(12000)
    m = s.macros()
    nu = oracle_values(c)["nu"]
    H = ny - 1
    t = np.arange(ny) / H
    par = 6 * U * t * (1 - t)
    mid = m["ux"][:, nx // 2]
    shape = np.max(np.abs(mid / mid.max() - par / par.max()))
    slope = np.polyfit(np.arange(nx), m["rho"][ny // 2], 1)[0] / (-12 * nu * U / H ** 2 * 3)
    flux = (m["rho"] * m["ux"])[1:-1, 1:-1].sum(axis=0)
    spread = (flux.max() - flux.min()) / flux.mean()
    log("shape err %.2e, pressure gradient ratio %.4f, flux spread %.2e" % (shape, slope, spread))
    assert shape < 1e-3 and abs(slope - 1) < 0.03 and spread < 1e-3
    assert abs(flux.mean() / par[1:-1].sum() - 1) < 0.02
