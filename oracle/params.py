"""Lattice parameters from the paper's dimensionless groups (oracle side).

TEST INFRASTRUCTURE ONLY.  This is the oracle's own derivation; the GPU
library derives the same quantities in its host code, and the two share
nothing.  All relations are the ones of Section 3 of Feng, Liu & He
(arXiv:2110.05943): the definitions of Eq. 38, the relaxation rates of
Eq. 46 (cavity) and of Section 3.1 (channel), the viscosity relations below
Eq. 15 and Eq. 37, and the Ergun/Kozeny-Carman closures of Eq. 5.
"""
import math

import numpy as np

CS2 = 1.0 / 3.0  # D2Q9 c_s^2 with c = 1 (below Eq. 15)


def ergun_F(phi):
    """Inertia coefficient of Eq. 5."""
    return 1.75 / np.sqrt(150.0 * np.asarray(phi, dtype=np.float64) ** 3)


def kozeny_carman_K(phi, dp):
    """Permeability of Eq. 5."""
    return phi ** 3 * dp ** 2 / (150.0 * (1.0 - phi) ** 2)


def cavity(n, Ra, Pr, Da, phi, J=1.0, Gamma=1.0, sigma=1.0, Ma=0.1, varpi=0.25):
    """Natural convection in a square porous cavity of n x n nodes (Section 3.2).

    Walls lie on the outer nodes, so the characteristic length is L = n - 1.
    Eq. 46 fixes 1/s_v and 1/zeta_alpha; u_c = sqrt(g beta dT L) = Ma c_s
    fixes g beta dT; Da = K/L^2 fixes K.
    """
    L = n - 1
    tau_v = 0.5 + Ma * J * L * math.sqrt(3.0 * Pr) / math.sqrt(Ra)
    cT2 = 0.5 * varpi
    tau_a = 0.5 + Gamma * CS2 * (tau_v - 0.5) / (J * cT2 * Pr)
    nu_e = CS2 * (tau_v - 0.5)
    nu = nu_e / J
    gbdT = (Ma * math.sqrt(CS2)) ** 2 / L
    return dict(L=L, tau_v=tau_v, s_v=1.0 / tau_v, tau_a=tau_a, za=1.0 / tau_a,
                nu_e=nu_e, nu=nu, alpha=nu / Pr, alpha_e=Gamma * nu / Pr,
                gbeta_dT=gbdT, K=Da * L * L, Fphi=ergun_F(phi), phi=phi,
                sigma=sigma, varpi=varpi)


def channel(ny, Re, Ra, Pr, Da, phi, u_ref, J=1.0, Gamma=1.0, sigma=1.0, varpi=0.25):
    """Mixed convection in a porous channel (Section 3.1).

    H = ny - 1; Re = H u_ref / nu gives nu, and 1/s_v = 1/2 + J H u_ref/(c_s^2 Re)
    is the same statement; zeta_alpha follows the cavity formula; Ra fixes
    g beta dT = Ra nu alpha / H^3 (Eq. 38); Da fixes K = Da H^2.
    """
    H = ny - 1
    tau_v = 0.5 + J * H * u_ref / (CS2 * Re)
    cT2 = 0.5 * varpi
    tau_a = 0.5 + Gamma * CS2 * (tau_v - 0.5) / (J * cT2 * Pr)
    nu = H * u_ref / Re
    alpha = nu / Pr
    return dict(H=H, tau_v=tau_v, s_v=1.0 / tau_v, tau_a=tau_a, za=1.0 / tau_a,
                nu_e=J * nu, nu=nu, alpha=alpha, alpha_e=Gamma * alpha,
                gbeta_dT=Ra * nu * alpha / H ** 3, K=Da * H * H, phi=phi,
                sigma=sigma, varpi=varpi)


def injection_ay(ny, u1, P):
    """The y-acceleration of Eq. 42 on rows y = 0 .. ny-1 (H = ny - 1) of the
    injection channel of Section 3.1, from a channel() parameter set P:
    (nu/K) u1 - g beta dT (exp(y u1/alpha_e) - 1) / (exp(H u1/alpha_e) - 1)."""
    H = ny - 1
    y = np.arange(ny, dtype=np.float64)
    k = u1 / P["alpha_e"]
    prof = np.expm1(y * k) / math.expm1(H * k) if k != 0 else y / H
    return P["nu"] / P["K"] * u1 - P["gbeta_dT"] * prof
