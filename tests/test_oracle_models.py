"""Pins of the raw-moment (MRT, N = N_T = I) and single-rate (BGK) variants of
the oracle: the end of Section 2 and Table 2 define the MRT method as the
present method with unit shift matrices."""
import math

import numpy as np
import pytest

import oracle
from tests.cases import cavity, oracle_lattice


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_mrt_equals_cascaded_at_rest():
    """With u = 0 and no force the shift matrices are the identity, so both
    collisions are the same map (D2Q9 and D2Q5)."""
    r = rng(1)
    for phi in (0.4, 1.0):
        f = oracle.feq(1.0, 0.0, 0.0, phi) + r.uniform(-1e-3, 1e-3, 9)
        jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8]
        jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8]
        f[1] -= jx / 2
        f[3] += jx / 2
        f[2] -= jy / 2
        f[4] += jy / 2
        kw = dict(nu=0.1, s_v=1.3, s_b=1.5, s3=1.2, s4=1.8, za=1.1, ze=0.9, zn=1.2, sigma=1.3)
        a = oracle.Lattice(4, 4, **kw)
        b = oracle.Lattice(4, 4, model="mrt", **kw)
        assert np.abs(a.collide_f(f, f.sum(), 0, 0, 0, 0, phi) -
                      b.collide_f(f, f.sum(), 0, 0, 0, 0, phi)).max() < 1e-15
        g = oracle.geq(0.6, 0, 0, 1.3, 0.25) + r.uniform(-1e-3, 1e-3, 5)
        g[1] -= (g[1] - g[3]) / 2
        g[3] = g[1]
        g[2] -= (g[2] - g[4]) / 2
        g[4] = g[2]
        T = g.sum() / 1.3
        assert np.abs(a.collide_g(g, T, 0, 0) - b.collide_g(g, T, 0, 0)).max() < 1e-15
    # and they differ once the fluid moves
    f = oracle.feq(1.0, 0.05, 0.02, 0.7)
    assert np.abs(a.collide_f(f, 1.0, 0.05, 0.02, 1e-4, 0, 0.7) -
                  b.collide_f(f, 1.0, 0.05, 0.02, 1e-4, 0, 0.7)).max() > 1e-6


@pytest.mark.parametrize("model", ["mrt", "bgk"])
def test_uniform_darcy_forchheimer_flow_raw_models(model):
    """The fixed point F = 0 of Eqs. 4, 21-23 holds for any collision that
    moves the first moments by rho F per step."""
    nu, K, Fp, ax, phi, s_v = 0.1, 8.0, 0.6, 2e-4, 0.5, 1.2
    rates = dict(s_b=s_v, s1=s_v, s3=s_v, s4=s_v) if model == "bgk" else {}
    lat = oracle.Lattice(3, 3, nu=nu, s_v=s_v, za=1.0, phi=phi, K=K, Fphi=Fp, a=(ax, 0.0),
                         nthreads=1, model=model, **rates)
    lat.init_equilibrium(0.5)
    lat.step(12000)
    b = Fp / math.sqrt(K)
    u_exact = (-(nu / K) + math.sqrt((nu / K) ** 2 + 4 * b * ax)) / (2 * b)
    assert np.allclose(lat.macros()["ux"], u_exact, rtol=1e-11)


@pytest.mark.parametrize("model", ["mrt", "bgk"])
def test_shear_wave_decay_raw_models(model):
    """u_x = A sin(k y) decays at nu_e k^2 + phi nu / K, second order."""
    errs = []
    for n in (16, 32):
        k = 2 * math.pi / n
        s_v, phi = 1.25, 0.7
        nu = (1 / s_v - 0.5) / 3
        K = 400.0 * (n / 16) ** 2
        rates = dict(s_b=s_v, s1=s_v, s3=s_v, s4=s_v) if model == "bgk" else {}
        lat = oracle.Lattice(3, n, nu=nu, s_v=s_v, za=1.0, phi=phi, K=K, Fphi=0.0, nthreads=1,
                             model=model, **rates)
        y = np.arange(n)[:, None] * np.ones((1, 3))
        lat.init_equilibrium(0.5, ux=1e-4 * np.sin(k * y), uy=0.0)
        n0, n1 = 20 * (n // 16) ** 2, 120 * (n // 16) ** 2
        lat.step(n0)
        a0 = np.abs(np.fft.rfft(lat.macros()["ux"][:, 0])[1])
        lat.step(n1 - n0)
        a1 = np.abs(np.fft.rfft(lat.macros()["ux"][:, 0])[1])
        rate = math.log(a0 / a1) / (n1 - n0)
        exact = nu * k * k + phi * nu / K
        errs.append(abs(rate - exact) / exact)
    assert errs[1] < 5e-3 and errs[0] / errs[1] > 3.0


@pytest.mark.parametrize("model", ["mrt", "bgk"])
def test_pure_conduction_raw_models(model):
    """No buoyancy: the steady temperature is linear and Nu = 1 exactly."""
    case = cavity(17, Ra=1e3, model=model, gbeta=1e-30)
    lat = oracle_lattice(case, nthreads=1)
    lat.init_equilibrium(0.5)
    lat.step(20000)
    assert abs(lat.nusselt(0, 1.0) - 1.0) < 1e-9
