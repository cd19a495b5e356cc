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


# ------------------------------------------------- walls (boundary readings)

def equilibria(rho, ux, uy, T, phi, sigma, varpi):
    """Equilibrium populations from the central-moment equilibria of Eqs. 16
    and 32: the raw equilibria are N^-1 m~^eq (Eq. 19), so f^eq solves
    (N M) f^eq = m~^eq; likewise g^eq with N_T and M_T (Eq. 34).  Numerical
    solves with the matrices typed in above; no printed inverse."""
    cs2, cT2 = 1.0 / 3.0, varpi / 2
    eq9 = np.array([rho, 0, 0, rho * cs2, rho * cs2, 0, 0, 0, rho * cs2 * cs2])
    eq5 = np.array([sigma * T, 0, 0, cT2 * T, cT2 * T])
    feq = np.linalg.solve(shift_N(ux, uy, phi) @ raw_moment_matrix(9), eq9)
    geq = np.linalg.solve(shift_NT(ux, uy, sigma) @ raw_moment_matrix(5), eq5)
    return feq, geq


def walled_step(f, g, *, bc, bc_u, bc_v, bc_T, inlet_U=0.0, phi, sigma, nu, K, Fphi, gb, T0, a,
                s, zeta, varpi):
    """One step on a lattice whose sides may be walls, following the boundary
    readings of the solver (the paper cites the non-equilibrium extrapolation
    scheme of its Ref. [55] without writing it out):
      - a node on a non-periodic side is a boundary node; x_f is its inward
        normal neighbour (the diagonal one at a corner), x_ff the next node on
        that line;
      - before the collision its populations become
        f^eq(rho_b, u_b; phi_b) + f(x_f) - f^eq(rho_f, u_f; phi_f), and g
        likewise with g^eq(T_b, u_b) and g^eq(T_f, u_f);
      - rho_b = rho_f (1 at an outlet), u_b the side's velocity (the inflow
        profile 6 U t (1 - t) at an inlet, u_f at an outlet, 0 at a corner);
      - T_b the side's temperature at a Dirichlet side (wall_T, inlet),
        (4 T_f - T_ff)/3 at an adiabatic one, T_f at an outlet; at a corner
        the x-side's Dirichlet value if it has one, else the y-side's, else
        the extrapolated value;
      - the node collides with (rho_b, u_b, T_b) and the force F(u_b, T_b).
    Streaming leaves a population whose source lies outside a walled side at
    the node's own post-collision value.  bc: kind names for W, E, S, N."""
    s0, s1, sb, sv, s3, s4 = s
    sp, sm = (sb + sv) / 2, (sb - sv) / 2
    Lam = np.zeros((9, 9))
    Lam[0, 0], Lam[1, 1], Lam[2, 2] = s0, s1, s1
    Lam[3:5, 3:5] = [[sp, sm], [sm, sp]]
    Lam[5, 5], Lam[6, 6], Lam[7, 7], Lam[8, 8] = sv, s3, s3, s4
    zT, za, ze, zn = zeta
    Q = np.diag([zT, za, za, ze, zn])
    M9, M5 = raw_moment_matrix(9), raw_moment_matrix(5)
    cs2, cT2 = 1.0 / 3.0, varpi / 2
    ny, nx = f.shape[1:]
    dirichlet = ("wall_T", "inlet")

    def force(u, T, ph):
        G = np.asarray(gb) * (T - T0) + np.asarray(a)
        return -ph * nu / K * u - ph * Fphi / math.sqrt(K) * math.hypot(u[0], u[1]) * u + ph * G

    # fluid values of every node
    rho = f.sum(axis=0)
    T = g.sum(axis=0) / sigma
    U = np.zeros((ny, nx, 2))
    for y in range(ny):
        for x in range(nx):
            j = np.array([(E[:9, 0] * f[:, y, x]).sum(), (E[:9, 1] * f[:, y, x]).sum()], float)
            G = np.asarray(gb) * (T[y, x] - T0) + np.asarray(a)
            U[y, x], _ = implicit_velocity(j, rho[y, x], phi[y, x], G, nu, K, Fphi)
    fs = np.empty_like(f)
    gs = np.empty_like(g)
    for y in range(ny):
        for x in range(nx):
            fn, gn = f[:, y, x].copy(), g[:, y, x].copy()
            ph = phi[y, x]
            sx = 0 if x == 0 and bc[0] != "periodic" else (1 if x == nx - 1 and bc[1] != "periodic" else -1)
            sy = 2 if y == 0 and bc[2] != "periodic" else (3 if y == ny - 1 and bc[3] != "periodic" else -1)
            if sx < 0 and sy < 0:
                r, u, t = rho[y, x], U[y, x], T[y, x]
            else:
                dx = (1 if sx == 0 else -1) if sx >= 0 else 0
                dy = (1 if sy == 2 else -1) if sy >= 0 else 0
                xf, yf, xff, yff = x + dx, y + dy, x + 2 * dx, y + 2 * dy
                rf, uf, tf, tff = rho[yf, xf], U[yf, xf], T[yf, xf], T[yff, xff]
                extra = (4 * tf - tff) / 3
                r = rf
                if sx >= 0 and sy >= 0:
                    u = np.zeros(2)
                    t = (bc_T[sx] if bc[sx] in dirichlet else
                         (bc_T[sy] if bc[sy] in dirichlet else extra))
                else:
                    side = sx if sx >= 0 else sy
                    kind = bc[side]
                    if kind in ("wall_T", "wall_adiabatic"):
                        u = np.array([bc_u[side], bc_v[side]], float)
                        t = bc_T[side] if kind == "wall_T" else extra
                    elif kind == "inlet":
                        tt = y / (ny - 1) if side < 2 else x / (nx - 1)
                        un = 6 * inlet_U * tt * (1 - tt)
                        inward = {0: (un, 0.0), 1: (-un, 0.0), 2: (0.0, un), 3: (0.0, -un)}[side]
                        u = np.array(inward, float)
                        t = bc_T[side]
                    else:  # outlet
                        r, u, t = 1.0, uf.copy(), tf
                feb, geb = equilibria(r, u[0], u[1], t, ph, sigma, varpi)
                fef, gef = equilibria(rf, uf[0], uf[1], tf, phi[yf, xf], sigma, varpi)
                fn = feb + f[:, yf, xf] - fef
                gn = geb + g[:, yf, xf] - gef
            F = force(np.asarray(u, float), t, ph)
            m = M9 @ fn
            N = shift_N(u[0], u[1], ph)
            mt = N @ m
            eq = np.array([r, 0, 0, r * cs2, r * cs2, 0, 0, 0, r * cs2 * cs2])
            S = np.array([0, r * F[0], r * F[1], 0, 0, 0, cs2 * r * F[1], cs2 * r * F[0], 0])
            mts = mt - Lam @ (mt - eq) + (np.eye(9) - Lam / 2) @ S
            fs[:, y, x] = np.linalg.solve(N @ M9, mts)
            NT = shift_NT(u[0], u[1], sigma)
            nt = NT @ (M5 @ gn)
            neq = np.array([sigma * t, 0, 0, cT2 * t, cT2 * t])
            gs[:, y, x] = np.linalg.solve(NT @ M5, nt - Q @ (nt - neq))
    of, og = np.empty_like(f), np.empty_like(g)
    for y in range(ny):
        for x in range(nx):
            for i in range(9):
                xs, ys = x - E[i, 0], y - E[i, 1]
                inside = True
                if not 0 <= xs < nx:
                    if bc[0] == "periodic":
                        xs %= nx
                    else:
                        inside = False
                if not 0 <= ys < ny:
                    if bc[2] == "periodic":
                        ys %= ny
                    else:
                        inside = False
                if not inside:
                    xs, ys = x, y
                of[i, y, x] = fs[i, ys, xs]
                if i < 5:
                    og[i, y, x] = gs[i, ys, xs]
    return of, og
