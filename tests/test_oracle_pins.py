"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: algebraic
identities between the paper's printed matrices and the moment definitions,
a brute-force re-derivation on a 4x4 lattice, conservation laws, closed-form
flows (uniform Darcy-Forchheimer flow, Darcy-Brinkman channel, the paper's
mixed-convection channel of Eqs. 43-44), decay rates of linear waves, pure
conduction, and second-order spatial convergence.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import params
from tests import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")
rng = np.random.Generator(np.random.PCG64(20211012))


def rand_u(scale=0.1):
    return rng.uniform(-scale, scale, 2)


# ------------------------------------------------------------------ P1, P2

def test_M_is_eq7_on_eq6_velocities(orc):
    # Eq. 13 must equal the raw-moment definition Eq. 7 on the velocity set Eq. 6.
    assert np.array_equal(orc.matrix("M"), brute.raw_moment_matrix(9))
    assert np.array_equal(orc.matrix("MT"), brute.raw_moment_matrix(5))
    assert np.allclose(orc.matrix("M") @ orc.matrix("Minv"), np.eye(9), atol=1e-15)
    assert np.allclose(orc.matrix("MT") @ orc.matrix("MTinv"), np.eye(5), atol=1e-15)


@pytest.mark.parametrize("trial", range(5))
def test_printed_inverses(orc, trial):
    ux, uy = rand_u(0.3)
    phi = rng.uniform(0.2, 1.0)
    sigma = rng.uniform(0.5, 2.0)
    assert np.allclose(orc.matrix("N", ux, uy, phi) @ orc.matrix("Ninv", ux, uy, phi), np.eye(9),
                       atol=1e-14)
    assert np.allclose(orc.matrix("NT", ux, uy, sigma) @ orc.matrix("NTinv", ux, uy, sigma),
                       np.eye(5), atol=1e-14)
    # the oracle's N is Eq. 14 as independently typed in the brute-force module
    assert np.allclose(orc.matrix("N", ux, uy, phi), brute.shift_N(ux, uy, phi), atol=0)
    assert np.allclose(orc.matrix("NT", ux, uy, sigma), brute.shift_NT(ux, uy, sigma), atol=0)


@pytest.mark.parametrize("trial", range(5))
def test_equilibria_and_sources_shift_consistently(orc, trial):
    # N m^eq (Eq. 19) = m~^eq (Eq. 16); N S (Eq. 19) = S~ (Eq. 17);
    # N_T n^eq (Eq. 33) = n~^eq (Eq. 32); M_T^-1 n^eq = g^eq (Eq. 34).
    rho = rng.uniform(0.8, 1.2)
    ux, uy = rand_u(0.2)
    Fx, Fy = rand_u(0.05)
    phi = rng.uniform(0.2, 1.0)
    sigma = rng.uniform(0.5, 2.0)
    T = rng.uniform(-1, 2)
    varpi = rng.uniform(0.1, 0.9)
    N = orc.matrix("N", ux, uy, phi)
    assert np.allclose(N @ orc.meq(rho, ux, uy, phi), orc.mteq(rho), atol=1e-15)
    assert np.allclose(N @ orc.Sraw(rho, ux, uy, Fx, Fy, phi), orc.St(rho, Fx, Fy), atol=1e-15)
    NT = orc.matrix("NT", ux, uy, sigma)
    neq = orc.neq(T, ux, uy, sigma, varpi)
    nt = NT @ neq
    cT2 = varpi / 2
    assert np.allclose(nt, [sigma * T, 0, 0, cT2 * T, cT2 * T], atol=1e-14)
    assert np.allclose(orc.matrix("MTinv") @ neq, orc.geq(T, ux, uy, sigma, varpi), atol=1e-15)


def test_rest_equilibrium_is_d2q9_weights(orc):
    assert np.allclose(orc.feq(1.0, 0.0, 0.0, 0.6), [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, atol=1e-16)
    # and for phi = 1 at finite u it is the textbook second-order-complete D2Q9
    # product form f_i = rho prod_a w(e_ia) [e_ia^2 u_a^2 ... ]: check the raw moments instead
    ux, uy = 0.05, -0.03
    m = brute.raw_moment_matrix(9) @ orc.feq(1.1, ux, uy, 1.0)
    assert np.isclose(m[1], 1.1 * ux) and np.isclose(m[2], 1.1 * uy)


@pytest.mark.parametrize("trial", range(4))
def test_phi1_central_moments_are_eq8(orc, trial):
    # At phi = 1 (and sigma = 1) N M f and N_T M_T g are the literal central
    # moments of Eqs. 8 and 25.
    f = rng.uniform(0.01, 0.3, 9)
    g = rng.uniform(0.01, 0.3, 5)
    ux, uy = rand_u(0.3)
    lit9 = np.array([(f * (brute.E[:9, 0] - ux) ** m * (brute.E[:9, 1] - uy) ** n).sum()
                     for (m, n) in brute.MN9])
    assert np.allclose(orc.matrix("N", ux, uy, 1.0) @ orc.matrix("M") @ f, lit9, atol=1e-15)
    lit5 = np.array([(g * (brute.E[:5, 0] - ux) ** m * (brute.E[:5, 1] - uy) ** n).sum()
                     for (m, n) in brute.MN5])
    assert np.allclose(orc.matrix("NT", ux, uy, 1.0) @ orc.matrix("MT") @ g, lit5, atol=1e-15)


def test_phi_not_one_differs_from_eq8(orc):
    # The porous shift is deliberately not the literal central moment (reading
    # of Eq. 12/14 over Eq. 8); a regression that replaced N by Eq. 8 would fail.
    f = rng.uniform(0.01, 0.3, 9)
    ux, uy = 0.1, 0.07
    lit9 = np.array([(f * (brute.E[:9, 0] - ux) ** m * (brute.E[:9, 1] - uy) ** n).sum()
                     for (m, n) in brute.MN9])
    assert not np.allclose(orc.matrix("N", ux, uy, 0.5) @ orc.matrix("M") @ f, lit9, atol=1e-6)


# --------------------------------------------------------------------- P3

def _lattice_kwargs():
    return dict(nu=0.08, s0=1.3, s1=0.9, s_b=1.4, s_v=1.1, s3=1.2, s4=1.8, zT=1.1, za=0.8,
                ze=1.3, zn=0.7, varpi=0.3, T0=0.5, gb=(0.002, 0.003), a=(1e-3, -2e-3),
                K=6.0, Fphi=0.4)


def test_brute_force_4x4(orc):
    nx = ny = 4
    kw = _lattice_kwargs()
    sigma = 1.13
    phi = rng.uniform(0.3, 0.95, (ny, nx))
    lat = oracle.Lattice(nx, ny, sigma=sigma, phi=phi, **kw)
    f0 = rng.uniform(0.02, 0.2, (ny, nx, 9))
    g0 = rng.uniform(0.02, 0.2, (ny, nx, 5))
    lat.f[:] = f0.reshape(-1)
    lat.g[:] = g0.reshape(-1)
    lat.step(1)
    fb, gb = brute.step(np.moveaxis(f0, 2, 0).copy(), np.moveaxis(g0, 2, 0).copy(), phi=phi,
                        sigma=sigma, nu=kw["nu"], K=kw["K"], Fphi=kw["Fphi"], gb=kw["gb"],
                        T0=kw["T0"], a=kw["a"],
                        s=(kw["s0"], kw["s1"], kw["s_b"], kw["s_v"], kw["s3"], kw["s4"]),
                        zeta=(kw["zT"], kw["za"], kw["ze"], kw["zn"]), varpi=kw["varpi"])
    fo = np.moveaxis(lat.f.reshape(ny, nx, 9), 2, 0)
    go = np.moveaxis(lat.g.reshape(ny, nx, 5), 2, 0)
    assert np.max(np.abs(fo - fb)) / np.max(np.abs(fb)) < 1e-13
    assert np.max(np.abs(go - gb)) / np.max(np.abs(gb)) < 1e-13


def test_implicit_velocity_closed_form(orc):
    # Eq. 22 is the exact root of Eq. 21: compare with a fixed-point solve.
    lat = oracle.Lattice(3, 3, sigma=1.0, phi=0.55, **_lattice_kwargs())
    for _ in range(5):
        f = rng.uniform(0.02, 0.2, 9)
        g = rng.uniform(0.02, 0.2, 5)
        rho, ux, uy, T, Fx, Fy = lat.node_macros(f, g)
        kw = _lattice_kwargs()
        G = np.array(kw["gb"]) * (T - kw["T0"]) + np.array(kw["a"])
        j = brute.raw_moment_matrix(9)[1:3] @ f
        u, F = brute.implicit_velocity(j, rho, 0.55, G, kw["nu"], kw["K"], kw["Fphi"])
        assert np.allclose([ux, uy], u, rtol=1e-13, atol=1e-16)
        assert np.allclose([Fx, Fy], F, rtol=1e-12, atol=1e-17)


# --------------------------------------------------------------------- P4

@pytest.mark.parametrize("s1", [0.6, 1.0, 1.7])
def test_consistent_forcing(orc, s1):
    # Post-collision first moments are j + rho F (momentum gains rho F per step)
    # and the post-collision central first moments are rho F / 2, for any s1.
    kw = _lattice_kwargs()
    kw["s1"] = s1
    lat = oracle.Lattice(3, 3, sigma=1.0, phi=0.7, **kw)
    M = brute.raw_moment_matrix(9)
    for _ in range(3):
        f = rng.uniform(0.02, 0.2, 9)
        rho, ux, uy, T, Fx, Fy = lat.node_macros(f, rng.uniform(0.02, 0.2, 5))
        fs = lat.collide_f(f, rho, ux, uy, Fx, Fy, 0.7)
        j = M[1:3] @ f
        js = M[1:3] @ fs
        assert np.allclose(js, j + rho * np.array([Fx, Fy]), rtol=1e-13, atol=1e-16)
        assert np.isclose(fs.sum(), rho, rtol=1e-15)
        cen = orc.matrix("N", ux, uy, 0.7) @ (M @ fs)
        assert np.allclose(cen[1:3], 0.5 * rho * np.array([Fx, Fy]), rtol=1e-12, atol=1e-17)


# --------------------------------------------------------------------- P5

def test_mass_and_heat_conservation_periodic(orc):
    n = 24
    phi = rng.uniform(0.35, 0.9, (n, n))
    kw = _lattice_kwargs()
    lat = oracle.Lattice(n, n, sigma=0.85, phi=phi, **kw)
    T = 0.5 + 0.3 * rng.uniform(-1, 1, (n, n))
    ux = 0.02 * rng.uniform(-1, 1, (n, n))
    uy = 0.02 * rng.uniform(-1, 1, (n, n))
    lat.init_equilibrium(T, ux, uy)
    m0, h0 = lat.f.sum(), lat.g.sum()
    lat.step(1500)
    assert abs(lat.f.sum() - m0) / m0 < 1e-12
    assert abs(lat.g.sum() - h0) / h0 < 1e-12
    assert np.all(np.isfinite(lat.f))


# --------------------------------------------------------------------- P6

def test_uniform_darcy_forchheimer_flow(orc):
    # Periodic uniform flow driven by a_x: at the fixed point F = 0, i.e.
    # (F_phi/sqrt K) u^2 + (nu/K) u - a = 0 (Eqs. 4, 21-23).
    nu, K, Fp, ax, phi = 0.1, 8.0, 0.6, 2e-4, 0.5
    lat = oracle.Lattice(3, 3, nu=nu, s_v=1.2, za=1.0, phi=phi, K=K, Fphi=Fp, a=(ax, 0.0),
                         nthreads=1)
    lat.init_equilibrium(0.5)
    lat.step(12000)
    b = Fp / math.sqrt(K)
    u_exact = (-(nu / K) + math.sqrt((nu / K) ** 2 + 4 * b * ax)) / (2 * b)
    m = lat.macros()
    assert np.allclose(m["ux"], u_exact, rtol=1e-11)
    assert np.allclose(m["uy"], 0.0, atol=1e-15)
    # Brinkman limit (F_phi = 0): u = a K / nu exactly
    lat = oracle.Lattice(3, 3, nu=nu, s_v=1.2, za=1.0, phi=phi, K=K, Fphi=0.0, a=(ax, 0.0),
                         nthreads=1)
    lat.init_equilibrium(0.5)
    lat.step(12000)
    assert np.allclose(lat.macros()["ux"], ax * K / nu, rtol=1e-11)


# --------------------------------------------------------------------- P7, P8

def _decay_rate(lat, field, key, n0, n1):
    lat.step(n0)
    a0 = np.abs(np.fft.rfft(lat.macros()[key][field])[1])
    lat.step(n1 - n0)
    a1 = np.abs(np.fft.rfft(lat.macros()[key][field])[1])
    return math.log(a0 / a1) / (n1 - n0)


def test_shear_wave_decay_with_darcy_drag(orc):
    # u_x = A sin(k y): decays at nu_e k^2 + phi nu / K (linearised Eq. 2).
    errs = []
    for n in (16, 32):
        k = 2 * math.pi / n
        s_v, phi, J = 1.25, 0.7, 1.0
        nu_e = (1 / s_v - 0.5) / 3
        nu = nu_e / J
        K = 400.0 * (n / 16) ** 2
        lat = oracle.Lattice(3, n, nu=nu, s_v=s_v, za=1.0, phi=phi, K=K, Fphi=0.0, nthreads=1)
        y = np.arange(n)[:, None] * np.ones((1, 3))
        lat.init_equilibrium(0.5, ux=1e-4 * np.sin(k * y), uy=0.0)
        rate = _decay_rate(lat, (slice(None), 0), "ux", 20 * (n // 16) ** 2, 120 * (n // 16) ** 2)
        exact = nu_e * k * k + phi * nu / K
        errs.append(abs(rate - exact) / exact)
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 3.0  # second order


@pytest.mark.parametrize("sigma", [0.7, 1.6])
def test_heat_capacity_ratio_diffusion(orc, sigma):
    # u = 0, T = T0 + A sin(k x): sigma dT/dt = alpha_e d2T/dx2 (Eq. 3) with
    # alpha_e = c_sT^2 (1/zeta_a - 1/2) (Eq. 37).
    errs = []
    for n in (16, 32):
        k = 2 * math.pi / n
        za, varpi = 1.2, 0.25
        alpha_e = varpi / 2 * (1 / za - 0.5)
        lat = oracle.Lattice(n, 3, nu=0.1, s_v=1.0, za=za, sigma=sigma, varpi=varpi,
                             nthreads=1)
        x = np.ones((3, 1)) * np.arange(n)[None, :]
        lat.init_equilibrium(0.5 + 1e-3 * np.sin(k * x))
        rate = _decay_rate(lat, (0, slice(None)), "T", 30 * (n // 16) ** 2, 200 * (n // 16) ** 2)
        exact = alpha_e * k * k / sigma
        errs.append(abs(rate - exact) / exact)
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 3.0


# --------------------------------------------------------------------- P9

def test_pure_conduction_cavity(orc):
    # No buoyancy: steady T is linear between the isothermal walls and the hot
    # wall Nusselt number is exactly 1 (checks walls-on-nodes, L = n - 1, the
    # boundary reconstruction and the Nusselt discretisation).
    n = 17
    lat = oracle.Lattice(n, n, bc=("wall_T", "wall_T", "wall_adiabatic", "wall_adiabatic"),
                         bc_T=(1.0, 0.0, 0.0, 0.0), nu=0.1, s_v=1.1, za=1.0, phi=0.6, K=30.0,
                         Fphi=0.3, nthreads=1)
    lat.init_equilibrium(0.5)
    lat.step(12000)
    m = lat.macros()
    x = np.arange(n)[None, :] * np.ones((n, 1))
    assert np.max(np.abs(m["T"] - (1 - x / (n - 1)))) < 1e-10
    assert abs(lat.nusselt(oracle.WEST) - 1.0) < 1e-10
    assert abs(lat.nusselt(oracle.EAST) - 1.0) < 1e-10
    assert np.max(np.abs(m["ux"])) < 1e-14


# --------------------------------------------------------------------- P10

def _fit_slope(ns, errs):
    return -np.polyfit(np.log(ns), np.log(errs), 1)[0]


def test_darcy_brinkman_channel_second_order(orc):
    # Periodic-x channel between no-slip walls driven by a_x:
    # u(y) = (a K / nu) [1 - cosh(r (y - H/2)) / cosh(r H / 2)], r = sqrt(phi / (J K)).
    phi, J, Da, s_v = 0.6, 1.0, 0.01, 1.0
    nu = (1 / s_v - 0.5) / 3 / J
    errs, ns = [], (17, 33, 65)
    for ny in ns:
        H = ny - 1
        K = Da * H * H
        ax = 1e-3 * nu / K  # keeps u_max ~ 1e-3
        lat = oracle.Lattice(3, ny, bc=("periodic", "periodic", "wall_T", "wall_T"),
                             bc_T=(0, 0, 0.5, 0.5), nu=nu, s_v=s_v, za=1.0, phi=phi, K=K,
                             Fphi=0.0, a=(ax, 0.0), nthreads=1)
        lat.init_equilibrium(0.5)
        lat.step(40 * H)
        prev = lat.macros()["ux"][:, 0].copy()
        for _ in range(200):
            lat.step(500)
            cur = lat.macros()["ux"][:, 0]
            if np.max(np.abs(cur - prev)) < 1e-15:
                break
            prev = cur.copy()
        y = np.arange(ny)
        r = math.sqrt(phi / (J * K))
        exact = ax * K / nu * (1 - np.cosh(r * (y - H / 2)) / np.cosh(r * H / 2))
        errs.append(np.linalg.norm(cur - exact) / np.linalg.norm(exact))
    assert errs[-1] < 1e-3
    assert 1.8 < _fit_slope(ns, errs) < 2.3


# --------------------------------------------------------------------- P11

def _paper_channel(ny, Re=5.0, s_v=1.0, phi=0.6, Da=0.01, Ra=100.0, J=1.0, nx=3):
    """Mixed convection in the porous channel of Section 3.1 (Eqs. 39-44)."""
    H = ny - 1
    nu = (1 / s_v - 0.5) / 3 / J
    u1 = Re * nu / H
    u0 = u1
    P = params.channel(ny, Re=Re, Ra=Ra, Pr=1.0, Da=Da, phi=phi, u_ref=u1, J=J)
    assert abs(P["s_v"] - s_v) < 1e-12
    alpha_e = P["alpha_e"]
    gbdT = P["gbeta_dT"]
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    ay = P["nu"] / P["K"] * u1 - gbdT * (np.exp(y * u1 / alpha_e) - 1) / (math.exp(H * u1 / alpha_e) - 1)
    accel = np.stack([np.zeros_like(ay), ay], axis=-1)
    lat = oracle.Lattice(nx, ny, bc=("periodic", "periodic", "wall_T", "wall_T"),
                         bc_u=(0, 0, 0.0, u0), bc_v=(0, 0, u1, u1), bc_T=(0, 0, 0.0, 1.0),
                         nu=P["nu"], s_v=P["s_v"], za=P["za"], phi=phi, K=P["K"], Fphi=0.0,
                         gb=(0.0, gbdT), T0=0.5, accel=accel, nthreads=1)
    lat.init_equilibrium(0.5, ux=0.0, uy=u1)
    th1 = Re / (2 * phi * J)
    th2 = math.sqrt(Re ** 2 + 4 * phi ** 3 * J / Da) / (2 * phi * J)
    eta = np.arange(ny) / H
    ux_a = u0 * np.exp(th1 * (eta - 1)) * np.sinh(th2 * eta) / math.sinh(th2)
    PrRe = (P["nu"] / alpha_e) * Re
    T_a = (np.exp(PrRe * eta) - 1) / (math.exp(PrRe) - 1)
    return lat, ux_a, u1, T_a


def _run_to_steady(lat, chunk, tol, max_chunks=400):
    prev = lat.macros()
    for _ in range(max_chunks):
        lat.step(chunk)
        cur = lat.macros()
        d = max(np.max(np.abs(cur["ux"] - prev["ux"])), np.max(np.abs(cur["T"] - prev["T"])))
        if d < tol:
            return cur
        prev = cur
    return cur


def test_paper_channel_profiles_and_convergence(orc):
    gold = json.load(open(os.path.join(GOLD, "paper_numbers.json")))
    ns = (17, 25, 33, 49, 65)
    eu, eT = [], []
    for ny in ns:
        lat, ux_a, u1, T_a = _paper_channel(ny)
        H = ny - 1
        m = _run_to_steady(lat, 20 * H, 1e-14)
        ux, uy, T = m["ux"][:, 0], m["uy"][:, 0], m["T"][:, 0]
        ea = np.sqrt(np.sum((ux - ux_a) ** 2 + (uy - u1) ** 2) / np.sum(ux_a ** 2 + u1 ** 2))
        eu.append(ea)
        eT.append(np.linalg.norm(T - T_a) / np.linalg.norm(T_a))
    su, sT = _fit_slope(ns, eu), _fit_slope(ns, eT)
    # The paper reports 2.032 (u) and 1.996 (T) for this setting.
    assert abs(su - gold["channel_convergence_slope_u"]["value"]) < 0.25, (su, eu)
    assert abs(sT - gold["channel_convergence_slope_T"]["value"]) < 0.25, (sT, eT)
    assert eu[-1] < 1e-3 and eT[-1] < 1e-2


def test_low_viscosity_channel_stays_finite(orc):
    # tau_v = 0.5015 (nu = 5e-4) on 32 x 32, the CLB stays stable past t = 2200.
    gold = json.load(open(os.path.join(GOLD, "paper_numbers.json")))
    tau = gold["clb_stable_tau_v"]["value"]
    lat, ux_a, u1, T_a = _paper_channel(32, Re=5.0, s_v=1 / tau, nx=32)
    lat.step(3000)
    m = lat.macros()
    assert all(np.all(np.isfinite(v)) for v in m.values())
    assert np.max(np.abs(m["ux"])) < 10 * np.max(np.abs(ux_a)) + 10 * u1


# ------------------------------------------------------ inlet and outlet (C8)

def test_inlet_outlet_channel_develops_poiseuille_flow(orc):
    # Clear fluid (phi = 1, no drag), parabolic inflow of mean U at the west
    # side, the outlet reading at the east side, no-slip walls.  The inflow is
    # already the developed profile, so the steady state is plane Poiseuille
    # flow: a parabolic profile everywhere, a linear pressure drop of
    # 12 nu U / H^2 (rho c_s^2 = p), and the same mass flux through every
    # interior column.
    nx, ny, U, s_v = 49, 17, 0.02, 1.0
    nu = (1 / s_v - 0.5) / 3
    lat = oracle.Lattice(nx, ny, bc=("inlet", "outlet", "wall_T", "wall_T"),
                         bc_T=(0.5, 0.5, 0.5, 0.5), inlet_U=U, nu=nu, s_v=s_v, za=1.0, phi=1.0,
                         Fphi=0.0, nthreads=1)
    lat.init_equilibrium(0.5)
    m = _run_to_steady(lat, 500, 1e-14)
    H = ny - 1
    t = np.arange(ny) / H
    par = 6 * U * t * (1 - t)
    ux, rho = m["ux"], m["rho"]
    mid = ux[:, nx // 2]
    assert np.max(np.abs(mid / mid.max() - par / par.max())) < 1e-3   # parabolic shape
    assert np.max(np.abs(ux[:, 0] - par)) < 1e-12                      # inlet nodes carry u_b
    slope = np.polyfit(np.arange(nx), rho[ny // 2], 1)[0]
    assert abs(slope / (-12 * nu * U / H ** 2 * 3) - 1) < 0.03         # Poiseuille gradient
    flux = (rho * ux)[1:-1, 1:-1].sum(axis=0)
    assert (flux.max() - flux.min()) / flux.mean() < 1e-3              # mass conserved
    assert abs(flux.mean() / par[1:-1].sum() - 1) < 0.02
    assert np.max(np.abs(m["uy"])) < 5e-3 * U                           # nearly parallel


# ---------------------------------------------------------- parameter derivation

def test_cavity_parameters_satisfy_definitions():
    # Eq. 46 plus u_c = Ma c_s must reproduce the dimensionless groups of Eq. 38.
    for n, Ra, Pr, Da in [(64, 1e3, 1.0, 1e-2), (128, 1e5, 0.71, 1e-4), (512, 1e7, 7.0, 1e-5)]:
        P = params.cavity(n, Ra=Ra, Pr=Pr, Da=Da, phi=0.6)
        L = n - 1
        assert math.isclose(P["nu_e"], (P["tau_v"] - 0.5) / 3, rel_tol=1e-14)
        assert math.isclose(P["alpha_e"], 0.125 * (P["tau_a"] - 0.5), rel_tol=1e-13)
        assert math.isclose(P["gbeta_dT"] * L ** 3 / (P["nu"] * P["alpha"]), Ra, rel_tol=1e-12)
        assert math.isclose(P["nu"] / P["alpha"], Pr, rel_tol=1e-14)
        assert math.isclose(math.sqrt(P["gbeta_dT"] * L) / math.sqrt(1 / 3), 0.1, rel_tol=1e-14)
        assert math.isclose(P["K"] / L ** 2, Da, rel_tol=1e-14)
