"""Named synthetic workloads as parameter sets (clb_params field names).

Pure parameter packing: the dimensionless groups, boundary kinds and seeded
inputs of each workload.  The lattice values are derived by the library
(clb_derive) and, independently, by the test oracle.

  cavity:   square porous cavity heated from the west, cooled from the east,
            adiabatic top and bottom (Section 3.2);
  batch:    many cavities of mixed size and parameters in one context;
  channel:  mixed-convection channel with a parabolic inlet, an outlet, a hot
            bottom and a cold top wall, and a random porosity map;
  paper_channel: the periodic mixed-convection channel with injection of
            Section 3.1.
"""
from . import inputs

CAVITY_BC = ("wall_T", "wall_T", "wall_adiabatic", "wall_adiabatic")
CHANNEL_BC = ("periodic", "periodic", "wall_T", "wall_T")
INOUT_BC = ("inlet", "outlet", "wall_T", "wall_T")


def cavity(n, Ra=1e3, Pr=1.0, Da=1e-2, phi=0.6, sigma=1.0, ny=None, **kw):
    """Cavity of n x n nodes (L = n - 1), T_h = 1 (west), T_c = 0 (east),
    Ergun F_phi (Eq. 5), K = Da L^2, relaxation rates of Eq. 46."""
    c = dict(nx=n, ny=n if ny is None else ny, bc=CAVITY_BC, bc_T=(1.0, 0.0, 0.0, 0.0), Ra=Ra,
             Pr=Pr, Da=Da, phi=phi, F_phi=-1.0, sigma=sigma, scaling="cavity")
    c.update(kw)
    return c


def batch(count=256, seed=3, storage="f32", sizes=(64, 128, 256, 512)):
    """The batched sweep: `count` cavities with parameters drawn by
    inputs.batch_cavities (size, Ra, Da, porosity, Pr, sigma)."""
    return [cavity(d["n"], Ra=d["Ra"], Pr=d["Pr"], Da=d["Da"], phi=d["phi"], sigma=d["sigma"],
                   storage=storage)
            for d in inputs.batch_cavities(count=count, seed=seed, sizes=sizes)]


def hetero_channel(nx, ny, ell=32, seed=4, Da_mean=1e-3, Re=100.0, Ri=1.0, U=0.04, Pr=1.0,
                   storage="f32", eps=None):
    """Porous channel of nx x ny nodes (H = ny - 1): parabolic inflow of mean
    U and T = 0 at the west, outlet at the east, T = 1 on the bottom wall and
    T = 0 on the top wall, gravity along -y.  Re = U H / nu, Ri = g beta dT H /
    U^2.  Porosity: a Gaussian random field of correlation length `ell` mapped
    to a uniform marginal on [0.3, 0.9] (or the given map); K and F_phi per
    node from the Kozeny-Carman relation and Eq. 5, with the particle diameter
    that gives the mean Darcy number Da_mean."""
    H = ny - 1
    if eps is None:
        eps = inputs.porosity_map(nx, ny, ell=ell, seed=seed)
    dp = inputs.particle_diameter_for_mean_Da(eps, Da_mean, H)
    return dict(nx=nx, ny=ny, bc=INOUT_BC, bc_T=(0.0, 0.0, 1.0, 0.0), inlet_U=U, eps=eps, dp=dp,
                F_phi=-1.0, scaling="channel", Re=Re, u_ref=U, Pr=Pr, gbeta=Ri * U * U / H,
                T_init=0.0, T0=0.5, storage=storage)


def paper_channel(ny, Re=5.0, nx=3, u1=0.01, s_v=None, Ra=100.0, Pr=1.0, Da=0.01, phi=0.6,
                  storage="f32", **kw):
    """Mixed convection in the porous channel of Section 3.1 (Fig. 1), H = ny - 1.

    Periodic in x.  The bottom plate (T = 0) is static, the top plate (T = 1)
    moves along x at u0 = u1; fluid enters through the bottom and leaves
    through the top at the normal velocity u1.  Brinkman medium (no
    Forchheimer term), K = Da H^2.  The library adds the y-acceleration of
    Eq. 42 per row (forcing "injection"), which makes the steady state that
    of Eqs. 43-44.

    With s_v given (the convergence study of Section 3.1), the injection
    velocity is the one that gives Re at that s_v (Re = H u1 / nu with
    nu = (1/s_v - 1/2) / 3 / J); otherwise u1 is the given injection velocity
    and the library derives s_v from Re (the Re family)."""
    H = ny - 1
    J = kw.get("J", 1.0)
    if s_v is not None:
        u1 = Re * (1.0 / s_v - 0.5) / 3.0 / J / H
    c = dict(nx=nx, ny=ny, bc=CHANNEL_BC, bc_u=(0.0, 0.0, 0.0, u1), bc_v=(0.0, 0.0, u1, u1),
             bc_T=(0.0, 0.0, 0.0, 1.0), scaling="channel", Re=Re, u_ref=u1, Pr=Pr, Ra=Ra, Da=Da,
             phi=phi, F_phi=0.0, T_init=0.5, storage=storage, forcing="injection")
    c.update(kw)
    return c
