"""Seeded synthetic inputs shared by the GPU path, the oracle, tests and the bench.

Holds none of the method's arithmetic: only random draws and their mapping to
the input ranges of the workloads (initial noise, porosity maps, per-domain
parameter sets).  All draws use numpy's PCG64 with an explicit seed.
"""
import math

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def cavity_initial_T(n, seed=1, amp=1e-6, T0=0.5, ny=None):
    """T = T0 + U(-amp, amp) on interior nodes, T0 on the wall nodes.

    The noise is drawn once, interior nodes in x-fastest order."""
    ny = n if ny is None else ny
    T = np.full((ny, n), T0, dtype=np.float64)
    T[1:-1, 1:-1] = T0 + rng(seed).uniform(-amp, amp, (ny - 2, n - 2))
    return T


def random_fields(nx, ny, seed, u_amp=0.02, T_amp=0.3, T0=0.5, smooth=4):
    """Smooth random (u, v, T) fields for state-level parity tests.

    White noise is box-filtered `smooth` times along each axis (periodic) so
    neighbouring nodes are correlated, then scaled to the given amplitudes."""
    g = rng(seed)
    out = []
    for amp in (u_amp, u_amp, T_amp):
        a = g.standard_normal((ny, nx))
        for _ in range(smooth):
            a = (a + np.roll(a, 1, 0) + np.roll(a, -1, 0)) / 3.0
            a = (a + np.roll(a, 1, 1) + np.roll(a, -1, 1)) / 3.0
        a = a / (np.max(np.abs(a)) + 1e-300) * amp
        out.append(a)
    return out[0], out[1], T0 + out[2]


def gaussian_random_field(nx, ny, ell, seed, gen=None):
    """Standardised Gaussian random field with covariance exp(-r^2 / ell^2).

    Periodic FFT filtering of white noise (from `gen`, else a generator
    seeded with `seed`) by the square root of the spectrum of that
    covariance, then shifted and scaled to zero mean, unit variance."""
    w = (gen if gen is not None else rng(seed)).standard_normal((ny, nx))
    kx = np.fft.fftfreq(nx) * 2 * math.pi
    ky = np.fft.fftfreq(ny) * 2 * math.pi
    k2 = ky[:, None] ** 2 + kx[None, :] ** 2
    # spectrum of exp(-r^2/l^2) is proportional to exp(-k^2 l^2 / 4)
    amp = np.exp(-k2 * ell * ell / 8.0)
    z = np.real(np.fft.ifft2(np.fft.fft2(w) * amp))
    z = (z - z.mean()) / z.std()
    return z


def normal_cdf(z):
    from scipy.special import ndtr
    return ndtr(z)


def porosity_map(nx, ny, ell, seed, eps_min=0.3, eps_max=0.9):
    """Porosity field with uniform marginal on [eps_min, eps_max].

    eps = eps_min + (eps_max - eps_min) * Phi(z) for a standardised Gaussian
    random field z; values are rounded to FP32 so the GPU (FP32 field) and the
    FP64 oracle see identical porosities."""
    z = gaussian_random_field(nx, ny, ell, seed)
    eps = eps_min + (eps_max - eps_min) * normal_cdf(z)
    return eps.astype(np.float32).astype(np.float64)


def particle_diameter_for_mean_Da(eps, Da_mean, H):
    """Input recipe: the particle diameter d_p for which the mean of
    eps^3 d_p^2 / (150 (1 - eps)^2) over the map equals Da_mean * H^2."""
    m = float(np.mean(eps ** 3 / (1.0 - eps) ** 2))
    return math.sqrt(150.0 * Da_mean * H * H / m)


def batch_cavities(count=256, seed=3, sizes=(64, 128, 256, 512)):
    """Per-domain parameters of the batched sweep, drawn in this order for each
    domain: N uniform over `sizes`, Ra log-uniform [1e3, 1e7], Da log-uniform
    [1e-5, 1e-1], porosity uniform [0.3, 0.95], Pr uniform over {0.71, 1, 7},
    sigma uniform [0.8, 1.2]."""
    g = rng(seed)
    out = []
    for _ in range(count):
        n = int(sizes[g.integers(len(sizes))])
        Ra = 10.0 ** g.uniform(3, 7)
        Da = 10.0 ** g.uniform(-5, -1)
        phi = g.uniform(0.3, 0.95)
        Pr = (0.71, 1.0, 7.0)[g.integers(3)]
        sigma = g.uniform(0.8, 1.2)
        out.append(dict(n=n, Ra=Ra, Da=Da, phi=phi, Pr=Pr, sigma=sigma))
    return out


def warmstart_draws(count, seed, n=128, ell=8.0, Ra=(1e3, 1e7), Da=(1e-5, 1e-1),
                    eps=(0.3, 0.95)):
    """Cavities of the learned warm start: for sample i, a generator seeded
    with (seed, i) draws, in this order, Ra log-uniform in Ra, Da log-uniform
    in Da (the mean Darcy number of the map), Pr uniform over {0.71, 1, 7},
    sigma uniform [0.8, 1.2], then a porosity map (Gaussian random field of
    correlation length `ell`, uniform marginal on eps).  Returns dicts with
    n, Ra, Da, Pr, sigma, eps (n x n)."""
    out = []
    for i in range(count):
        g = np.random.Generator(np.random.PCG64([seed, i]))
        d = dict(n=n, Ra=10.0 ** g.uniform(np.log10(Ra[0]), np.log10(Ra[1])),
                 Da=10.0 ** g.uniform(np.log10(Da[0]), np.log10(Da[1])),
                 Pr=(0.71, 1.0, 7.0)[g.integers(3)], sigma=g.uniform(0.8, 1.2))
        zf = gaussian_random_field(n, n, ell, None, gen=g)
        e = eps[0] + (eps[1] - eps[0]) * normal_cdf(zf)
        d["eps"] = e.astype(np.float32).astype(np.float64)
        out.append(d)
    return out
