"""Brute-force re-derivation of one porous CLB step on a small periodic lattice.

Used only to pin the oracle.  It shares nothing with oracle/ except the
reading of the paper: the velocity set is generated from the trigonometric
form of Eq. 6, raw moments are the sums of Eq. 7 / Eq. 24 (no matrix M),
the way back from central moments to populations is a numerical linear
solve of (N M) f* = m~* (no printed inverse, no M^-1), the implicit velocity
is found by a fixed-point iteration of Eq. 21 (not the closed form of
Eq. 22), and streaming is a numpy roll.
"""
import math

import numpy as np

# (m, n) exponents of the moment sets, Eqs. 9 and 26.
MN9 = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]
MN5 = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2)]


def velocities():
    """Eq. 6 evaluated with c = 1 (rounded to the integer lattice)."""
    e = [(0.0, 0.0)]
    for i in range(1, 5):
        t = (i - 1) * math.pi / 2
        e.append((math.cos(t), math.sin(t)))
    for i in range(5, 9):
        t = (2 * i - 9) * math.pi / 4
        e.append((math.sqrt(2) * math.cos(t), math.sqrt(2) * math.sin(t)))
    return np.rint(np.array(e)).astype(int)


E = velocities()


def raw_moment_matrix(nq):
    """Row (m, n) holds e_x^m e_y^n over the velocities (Eq. 7 / Eq. 24)."""
    mn = MN9 if nq == 9 else MN5
    return np.array([[float(E[i, 0]) ** m * float(E[i, 1]) ** n for i in range(nq)] for (m, n) in mn])


def shift_N(ux, uy, phi):
    """Eq. 14 typed in independently of the oracle."""
    p = phi
    a, b = ux, uy
    N = np.eye(9)
    N[1, 0], N[2, 0] = -a, -b
    N[3, :2] = [a * a / p, -2 * a / p]
    N[4, [0, 2]] = [b * b / p, -2 * b / p]
    N[5, :3] = [a * b / p, -b / p, -a / p]
    N[6, :6] = [-a * a * b / p, 2 * a * b / p, a * a / p, -b, 0, -2 * a]
    N[7, :6] = [-b * b * a / p, b * b / p, 2 * a * b / p, 0, -a, -2 * b]
    N[8, :8] = [a * a * b * b / p ** 2, -2 * a * b * b / p ** 2, -2 * b * a * a / p ** 2,
                b * b / p, a * a / p, 4 * a * b / p, -2 * b / p, -2 * a / p]
    return N


def shift_NT(ux, uy, sigma):
    """Eq. 31 typed in independently of the oracle."""
    N = np.eye(5)
    N[1, 0], N[2, 0] = -ux / sigma, -uy / sigma
    N[3, 0], N[3, 1] = ux * ux / sigma, -2 * ux
    N[4, 0], N[4, 2] = uy * uy / sigma, -2 * uy
    return N


def implicit_velocity(j, rho, phi, G, nu, K, Fphi, iters=200):
    """Solve rho u = j + rho F(u) / 2 (Eq. 21 with F of Eq. 4) by iteration."""
    u = j / rho
    for _ in range(iters):
        umag = math.hypot(u[0], u[1])
        F = -phi * nu / K * u - phi * Fphi / math.sqrt(K) * umag * u + phi * G
        u = j / rho + 0.5 * F
    umag = math.hypot(u[0], u[1])
    F = -phi * nu / K * u - phi * Fphi / math.sqrt(K) * umag * u + phi * G
    return u, F


def step(f, g, *, phi, sigma, nu, K, Fphi, gb, T0, a, s, zeta, varpi):
    """One collide-and-stream step on a periodic lattice.

    f: (9, ny, nx), g: (5, ny, nx); phi: (ny, nx); s = (s0, s1, s_b, s_v, s3, s4);
    zeta = (zT, za, ze, zn).  Returns the post-streaming (f, g)."""
    s0, s1, sb, sv, s3, s4 = s
    sp, sm = (sb + sv) / 2, (sb - sv) / 2
    Lam = np.zeros((9, 9))
    Lam[0, 0], Lam[1, 1], Lam[2, 2] = s0, s1, s1
    Lam[3:5, 3:5] = [[sp, sm], [sm, sp]]
    Lam[5, 5], Lam[6, 6], Lam[7, 7], Lam[8, 8] = sv, s3, s3, s4
    zT, za, ze, zn = zeta
    Q = np.diag([zT, za, za, ze, zn])  # Eq. 28
    M9 = raw_moment_matrix(9)
    M5 = raw_moment_matrix(5)
    cs2, cT2 = 1.0 / 3.0, varpi / 2
    ny, nx = f.shape[1:]
    fs = np.empty_like(f)
    gs = np.empty_like(g)
    for y in range(ny):
        for x in range(nx):
            fn, gn = f[:, y, x], g[:, y, x]
            ph = phi[y, x]
            rho = fn.sum()
            j = np.array([(E[:9, 0] * fn).sum(), (E[:9, 1] * fn).sum()], dtype=float)
            T = gn.sum() / sigma
            G = np.asarray(gb) * (T - T0) + np.asarray(a)
            u, F = implicit_velocity(j, rho, ph, G, nu, K, Fphi)
            # D2Q9
            m = np.array([(fn * E[:9, 0] ** mm * E[:9, 1] ** nn).sum() for (mm, nn) in MN9])
            N = shift_N(u[0], u[1], ph)
            mt = N @ m
            eq = np.array([rho, 0, 0, rho * cs2, rho * cs2, 0, 0, 0, rho * cs2 * cs2])
            S = np.array([0, rho * F[0], rho * F[1], 0, 0, 0, cs2 * rho * F[1], cs2 * rho * F[0], 0])
            mts = mt - Lam @ (mt - eq) + (np.eye(9) - Lam / 2) @ S
            fs[:, y, x] = np.linalg.solve(N @ M9, mts)
            # D2Q5
            n = np.array([(gn * E[:5, 0] ** mm * E[:5, 1] ** nn).sum() for (mm, nn) in MN5])
            NT = shift_NT(u[0], u[1], sigma)
            nt = NT @ n
            neq = np.array([sigma * T, 0, 0, cT2 * T, cT2 * T])
            nts = nt - Q @ (nt - neq)
            gs[:, y, x] = np.linalg.solve(NT @ M5, nts)
    out_f = np.stack([np.roll(np.roll(fs[i], E[i, 1], axis=0), E[i, 0], axis=1) for i in range(9)])
    out_g = np.stack([np.roll(np.roll(gs[i], E[i, 1], axis=0), E[i, 0], axis=1) for i in range(5)])
    return out_f, out_g
