"""Closed-form steady states used as pins (no lattice parameters involved).

The injection channel of Section 3.1: Eq. 43 (velocity) and Eq. 44
(temperature), written from the dimensionless inputs of a
workloads.paper_channel case.  The effective Prandtl number of Eq. 44 is
Pr_e = nu / alpha_e = Pr / Gamma: Eq. 37 with the zeta_alpha relation of
Section 3.1 gives alpha_e = Gamma nu / Pr.
"""
import math

import numpy as np


def paper_channel_exact(case):
    """(u_x, u_y, T) over the rows y = 0 .. H (H = ny - 1) of a paper_channel
    case: Eq. 43 with theta_1 = Re/(2 phi J), theta_2 = sqrt(Re^2 + 4 phi^3
    J / Da)/(2 phi J), u0 = the top plate's speed, u1 = the injection
    velocity; Eq. 44 with T_c = 0 (bottom), dT = 1."""
    ny = case["ny"]
    H = ny - 1
    Re, phi, Da = case["Re"], case["phi"], case["Da"]
    J, Gamma, Pr = case.get("J", 1.0), case.get("Gamma", 1.0), case["Pr"]
    u0, u1 = case["bc_u"][3], case["bc_v"][2]
    th1 = Re / (2 * phi * J)
    th2 = math.sqrt(Re * Re + 4 * phi ** 3 * J / Da) / (2 * phi * J)
    eta = np.arange(ny, dtype=np.float64) / H
    ux = u0 * np.exp(th1 * (eta - 1)) * np.sinh(th2 * eta) / math.sinh(th2)
    pe = Pr / Gamma * Re  # Pr_e Re
    T = np.expm1(pe * eta) / math.expm1(pe)
    return ux, np.full(ny, u1), T
