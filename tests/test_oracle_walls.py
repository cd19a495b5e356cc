"""Pins of the oracle's boundary nodes (readings of the boundary scheme the
paper cites without writing out, Section 3): walls, corners between sides of
every kind, inlet and outlet.

- A brute-force step (tests/brute.py: population-space reconstruction with
  numerically solved equilibria, fixed-point implicit velocity, explicit
  streaming loops) on small walled lattices, against the oracle's
  moment-matrix step, over two steps and every corner branch: the x-side's
  Dirichlet temperature, the y-side's, and the extrapolated one.
- Pure conduction in a square with one hot side and three cold ones (two
  Dirichlet sides meet at every corner): the interior field converges at
  second order to its Fourier series and the cold far side's mean Nusselt
  number to the series value 8/pi sum_k odd 1/(k sinh(k pi)).
- The corner temperature between two Dirichlet sides decides only which of
  the two sides books the flux of the corner gap: the sum of the two sides'
  trapezoid fluxes does not depend on it.
"""
import math

import numpy as np
import pytest

import oracle
from tests import brute

rng = np.random.Generator(np.random.PCG64(20211013))

KW = dict(nu=0.08, s0=1.3, s1=0.9, s_b=1.4, s_v=1.1, s3=1.2, s4=1.8, zT=1.1, za=0.8, ze=1.3,
          zn=0.7, varpi=0.3, T0=0.5, gb=(0.002, 0.003), a=(1e-3, -2e-3), K=6.0, Fphi=0.4)

# side kinds W, E, S, N; temperatures; velocities of the sides
WALLED = [
    # two Dirichlet sides at every corner: the x-side's value wins
    (("wall_T", "wall_T", "wall_T", "wall_T"), (1.0, 0.0, 0.3, 0.7), (0, 0, 0.02, -0.01),
     (0, 0, 0, 0)),
    # adiabatic x-side, Dirichlet y-side (y-side's value); adiabatic pair (extrapolated)
    (("wall_adiabatic", "wall_T", "wall_T", "wall_adiabatic"), (0.0, 0.2, 0.9, 0.0),
     (0, 0, 0, 0.03), (0, 0, 0, 0)),
    # inlet / outlet with Dirichlet walls: inlet (x-side, Dirichlet) wins at its corners,
    # the wall at the outlet's
    (("inlet", "outlet", "wall_T", "wall_T"), (0.1, 0.0, 1.0, 0.0), (0, 0, 0, 0),
     (0, 0, 0, 0)),
    # inlet on the south side (y-side Dirichlet), outlet north, adiabatic x-sides
    (("wall_adiabatic", "wall_adiabatic", "inlet", "outlet"), (0.0, 0.0, 0.8, 0.0),
     (0, 0, 0, 0), (0, 0, 0, 0)),
    # periodic in x, walls in y
    (("periodic", "periodic", "wall_T", "wall_adiabatic"), (0.0, 0.0, 0.6, 0.0),
     (0, 0, 0, 0.02), (0, 0, 0, 0)),
]


@pytest.mark.parametrize("case", range(len(WALLED)))
def test_walled_brute_force(orc, case):
    bc, bc_T, bc_u, bc_v = WALLED[case]
    nx, ny = 6, 5
    sigma = 1.07
    phi = rng.uniform(0.3, 0.95, (ny, nx))
    lat = oracle.Lattice(nx, ny, bc=bc, bc_T=bc_T, bc_u=bc_u, bc_v=bc_v, inlet_U=0.015,
                         sigma=sigma, phi=phi, **KW)
    # near-equilibrium random state (positive populations, |u| ~ 0.02)
    T0 = rng.uniform(0.2, 0.8, (ny, nx))
    u0 = rng.uniform(-0.02, 0.02, (ny, nx))
    v0 = rng.uniform(-0.02, 0.02, (ny, nx))
    lat.init_equilibrium(T0, u0, v0)
    lat.f[:] *= 1 + rng.uniform(-0.05, 0.05, lat.f.shape)
    lat.g[:] *= 1 + rng.uniform(-0.05, 0.05, lat.g.shape)
    f = np.moveaxis(lat.f.reshape(ny, nx, 9), 2, 0).copy()
    g = np.moveaxis(lat.g.reshape(ny, nx, 5), 2, 0).copy()
    for _ in range(2):
        lat.step(1)
        f, g = brute.walled_step(
            f, g, bc=bc, bc_u=bc_u, bc_v=bc_v, bc_T=bc_T, inlet_U=0.015, phi=phi, sigma=sigma,
            nu=KW["nu"], K=KW["K"], Fphi=KW["Fphi"], gb=KW["gb"], T0=KW["T0"], a=KW["a"],
            s=(KW["s0"], KW["s1"], KW["s_b"], KW["s_v"], KW["s3"], KW["s4"]),
            zeta=(KW["zT"], KW["za"], KW["ze"], KW["zn"]), varpi=KW["varpi"])
        fo = np.moveaxis(lat.f.reshape(ny, nx, 9), 2, 0)
        go = np.moveaxis(lat.g.reshape(ny, nx, 5), 2, 0)
        assert np.max(np.abs(fo - f)) / np.max(np.abs(f)) < 1e-12
        assert np.max(np.abs(go - g)) / np.max(np.abs(g)) < 1e-12


def test_corner_rule_is_what_the_brute_force_states(orc):
    # A plausible slip (the y-side's Dirichlet value at a corner where both
    # sides are Dirichlet) changes the result: the pin above can tell.
    bc, bc_T, bc_u, bc_v = WALLED[0]
    nx, ny = 6, 5
    phi = np.full((ny, nx), 0.6)
    lat = oracle.Lattice(nx, ny, bc=bc, bc_T=bc_T, bc_u=bc_u, bc_v=bc_v, sigma=1.0, phi=phi, **KW)
    lat.init_equilibrium(0.5)
    m = lat.macros()
    # corners report the x-side's temperature
    assert m["T"][0, 0] == bc_T[0] and m["T"][-1, 0] == bc_T[0]
    assert m["T"][0, -1] == bc_T[1] and m["T"][-1, -1] == bc_T[1]
    # the other sides' nodes report their own
    assert np.all(m["T"][0, 1:-1] == bc_T[2]) and np.all(m["T"][-1, 1:-1] == bc_T[3])


def fourier_T(x, y, terms=400):
    """Steady conduction in the unit square, T = 1 at x = 0 and 0 on the
    other sides: sum over odd k of 4/(k pi) sin(k pi y) sinh(k pi (1-x)) /
    sinh(k pi), evaluated as exp differences to avoid overflow."""
    T = np.zeros_like(x, dtype=np.float64)
    for k in range(1, 2 * terms, 2):
        kp = k * math.pi
        ratio = (np.exp(-kp * x) - np.exp(-kp * (2 - x))) / (1 - math.exp(-2 * kp))
        T += 4 / kp * np.sin(kp * y) * ratio
    return T


def fourier_cold_side_nu():
    """Mean Nusselt number of the side opposite the hot one:
    sum over odd k of 8 / (k pi sinh(k pi))."""
    return sum(8 / (k * math.pi * math.sinh(k * math.pi)) for k in range(1, 41, 2))


def _conduction(n):
    L = n - 1
    lat = oracle.Lattice(n, n, bc=("wall_T",) * 4, bc_T=(1.0, 0.0, 0.0, 0.0), nu=1 / 6,
                         s_v=1.0, za=0.6, gb=(0.0, 0.0), phi=1.0, nthreads=0)
    xs = np.arange(n) / L
    X, Y = np.meshgrid(xs, xs)
    T0 = fourier_T(np.maximum(X, 1e-9), Y)
    T0[:, 0] = 1.0
    lat.init_equilibrium(T0)
    prev = lat.macros()["T"]
    for _ in range(400):
        lat.step(200)
        cur = lat.macros()["T"]
        if np.max(np.abs(cur - prev)) < 1e-13:
            break
        prev = cur
    return lat, X, Y


def test_two_dirichlet_corners_conduction_converges_to_fourier(orc):
    ns = (17, 33, 65)
    err, dnu = [], []
    exact_nu = fourier_cold_side_nu()
    assert abs(exact_nu - 0.2206) < 1e-3
    for n in ns:
        lat, X, Y = _conduction(n)
        m = lat.macros()
        assert np.max(np.abs(m["ux"])) == 0 and np.max(np.abs(m["uy"])) == 0
        far = X >= 0.25  # away from the two singular hot corners
        Ta = fourier_T(X[far], Y[far])
        err.append(np.linalg.norm(m["T"][far] - Ta) / np.linalg.norm(Ta))
        dnu.append(abs(lat.nusselt(oracle.EAST) - exact_nu))
    slope_T = -np.polyfit(np.log(ns), np.log(err), 1)[0]
    slope_nu = -np.polyfit(np.log(ns), np.log(dnu), 1)[0]
    assert slope_T > 1.8, (err, slope_T)
    # second order once the grid resolves the corners (1.62, then 1.83 per doubling)
    assert slope_nu > 1.7 and dnu[-1] < 3e-4, (dnu, slope_nu)


def test_corner_value_moves_flux_between_its_sides_only():
    # The trapezoid Nusselt sums of the two sides meeting at the hot-cold
    # corner (T_c at the corner node, T = 1 along the x-side, T = 0 along the
    # y-side): the x-side's end term is 3 T_c / 2 (times L), the y-side's
    # (3 - 3 T_c) / 2, so their sum does not depend on T_c.  The reading
    # (x-side wins, T_c = 1) books the corner gap on the hot side.
    for Tc in (0.0, 0.5, 1.0):
        hot_end = -(-3 * Tc + 4 * 0.0 - 0.0) / 2   # along the hot side, into the cold one
        cold_end = (-3 * Tc + 4 * 1.0 - 1.0) / 2   # along the cold side, into the hot one
        assert math.isclose(hot_end + cold_end, 1.5)
