"""ctypes wrapper of the FP64 CPU oracle (oracle/clb_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The product path never imports this module.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3
KIND = {"periodic": 0, "wall_T": 1, "wall_adiabatic": 2, "inlet": 3, "outlet": 4}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        P = C.POINTER(_Params)
        for name in ("orc_matrix_M", "orc_matrix_Minv", "orc_matrix_MT", "orc_matrix_MTinv"):
            getattr(L, name).argtypes = [dp]
        for name in ("orc_matrix_N", "orc_matrix_Ninv", "orc_matrix_NT", "orc_matrix_NTinv"):
            getattr(L, name).argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_matrix_Lambda.argtypes = [P, dp]
        L.orc_meq.argtypes = [C.c_double] * 4 + [dp]
        L.orc_Sraw.argtypes = [C.c_double] * 6 + [dp]
        L.orc_mteq.argtypes = [C.c_double, dp]
        L.orc_St.argtypes = [C.c_double] * 3 + [dp]
        L.orc_feq.argtypes = [C.c_double] * 4 + [dp]
        L.orc_geq.argtypes = [C.c_double] * 5 + [dp]
        L.orc_neq.argtypes = [C.c_double] * 5 + [dp]
        L.orc_collide_f.argtypes = [P, dp] + [C.c_double] * 6 + [dp]
        L.orc_collide_g.argtypes = [P, dp] + [C.c_double] * 3 + [dp]
        L.orc_node_macros.argtypes = [P, dp, dp, C.c_int32, dp]
        L.orc_init_equilibrium.argtypes = [P, dp, dp, dp, dp, dp, dp]
        L.orc_init_equilibrium.restype = C.c_int
        L.orc_step.argtypes = [P, dp, dp, C.c_int64]
        L.orc_step.restype = C.c_int
        L.orc_macros.argtypes = [P, dp, dp, dp, dp, dp, dp]
        L.orc_macros.restype = C.c_int
        L.orc_nusselt.argtypes = [P, dp, dp, C.c_int32, C.c_double, dp]
        L.orc_nusselt.restype = C.c_double
        _lib = L
    return _lib


class _Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32 * 4),
        ("bc_u", C.c_double * 4), ("bc_v", C.c_double * 4), ("bc_T", C.c_double * 4),
        ("inlet_U", C.c_double), ("nu", C.c_double),
        ("s0", C.c_double), ("s1", C.c_double), ("s_b", C.c_double), ("s_v", C.c_double),
        ("s3", C.c_double), ("s4", C.c_double),
        ("zT", C.c_double), ("za", C.c_double), ("ze", C.c_double), ("zn", C.c_double),
        ("varpi", C.c_double), ("sigma", C.c_double), ("T0", C.c_double),
        ("gb", C.c_double * 2), ("a", C.c_double * 2),
        ("accel", C.POINTER(C.c_double)), ("phi", C.POINTER(C.c_double)),
        ("K", C.POINTER(C.c_double)), ("Fphi", C.POINTER(C.c_double)),
        ("nthreads", C.c_int32), ("model", C.c_int32),
    ]


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _vec(n):
    return np.zeros(n, dtype=np.float64)


# ------------------------------------------------------------ single-node API

def matrix(name, *args):
    """Return one of the paper's matrices as a numpy array.

    name in {"M", "Minv", "MT", "MTinv"} (no args) or {"N", "Ninv", "NT",
    "NTinv"} with (ux, uy, phi_or_sigma)."""
    n = 9 if name in ("M", "Minv", "N", "Ninv") else 5
    out = _vec(n * n)
    getattr(lib(), "orc_matrix_" + name)(*args, _ptr(out))
    return out.reshape(n, n)


def _scalar_fn(name, n, *args):
    out = _vec(n)
    getattr(lib(), name)(*[float(a) for a in args], _ptr(out))
    return out


def meq(rho, ux, uy, phi):
    return _scalar_fn("orc_meq", 9, rho, ux, uy, phi)


def Sraw(rho, ux, uy, Fx, Fy, phi):
    return _scalar_fn("orc_Sraw", 9, rho, ux, uy, Fx, Fy, phi)


def mteq(rho):
    return _scalar_fn("orc_mteq", 9, rho)


def St(rho, Fx, Fy):
    return _scalar_fn("orc_St", 9, rho, Fx, Fy)


def feq(rho, ux, uy, phi):
    return _scalar_fn("orc_feq", 9, rho, ux, uy, phi)


def geq(T, ux, uy, sigma, varpi=0.25):
    return _scalar_fn("orc_geq", 5, T, ux, uy, sigma, varpi)


def neq(T, ux, uy, sigma, varpi=0.25):
    return _scalar_fn("orc_neq", 5, T, ux, uy, sigma, varpi)


# ------------------------------------------------------------------- lattice

class Lattice:
    """An nx x ny lattice advanced by the oracle.

    Arrays are (ny, nx) with x fastest.  s_b defaults to 1.5, the reading of
    the bulk rate (garbled in the paper) for which the rest-state collision is
    linearly stable at every s_v; s_b=None means s_b = s_v.  `phi`, `K`, `Fphi` are scalars or
    (ny, nx) arrays; K = inf removes the Darcy drag.  bc is a 4-tuple of kind
    names for W, E, S, N.
    """

    def __init__(self, nx, ny, *, bc=("periodic",) * 4, bc_u=(0, 0, 0, 0), bc_v=(0, 0, 0, 0),
                 bc_T=(0, 0, 0, 0), inlet_U=0.0, nu, s_v, s_b=1.5, s0=1.0, s1=1.0, s3=1.2,
                 s4=1.8, za, zT=1.0, ze=1.0, zn=1.0, varpi=0.25, sigma=1.0, T0=0.5,
                 gb=(0.0, 0.0), a=(0.0, 0.0), accel=None, phi=1.0, K=math.inf, Fphi=0.0,
                 nthreads=0, model=0):
        self.nx, self.ny = int(nx), int(ny)
        n = self.nx * self.ny

        def field(v):
            arr = np.empty(n, dtype=np.float64)
            arr[:] = np.asarray(v, dtype=np.float64).reshape(-1) if np.ndim(v) else float(v)
            return arr

        self.phi = field(phi)
        self.K = field(K)
        self.Fphi = field(Fphi)
        self.accel = None
        if accel is not None:
            self.accel = np.ascontiguousarray(np.asarray(accel, dtype=np.float64).reshape(n, 2))
        p = _Params()
        p.nx, p.ny = self.nx, self.ny
        for s in range(4):
            p.bc[s] = KIND[bc[s]] if isinstance(bc[s], str) else int(bc[s])
            p.bc_u[s], p.bc_v[s], p.bc_T[s] = bc_u[s], bc_v[s], bc_T[s]
        p.inlet_U = inlet_U
        p.nu = nu
        p.s0, p.s1, p.s_v, p.s3, p.s4 = s0, s1, s_v, s3, s4
        p.s_b = s_v if s_b is None else s_b
        p.zT, p.za, p.ze, p.zn = zT, za, ze, zn
        p.varpi, p.sigma, p.T0 = varpi, sigma, T0
        p.gb[0], p.gb[1] = gb
        p.a[0], p.a[1] = a
        p.accel = _ptr(self.accel)
        p.phi, p.K, p.Fphi = _ptr(self.phi), _ptr(self.K), _ptr(self.Fphi)
        p.nthreads = nthreads
        p.model = {"clb": 0, "mrt": 1, "bgk": 1}.get(model, model)
        self.p = p
        self.f = _vec(9 * n)
        self.g = _vec(5 * n)
        self.steps = 0

    # state --------------------------------------------------------------
    def init_equilibrium(self, T, ux=None, uy=None, rho=None):
        n = self.nx * self.ny

        def flat(v):
            if v is None:
                return None
            arr = np.empty(n, dtype=np.float64)
            arr[:] = np.asarray(v, dtype=np.float64).reshape(-1) if np.ndim(v) else float(v)
            return arr

        T, ux, uy, rho = flat(T), flat(ux), flat(uy), flat(rho)
        rc = lib().orc_init_equilibrium(C.byref(self.p), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T),
                                        _ptr(self.f), _ptr(self.g))
        if rc:
            raise ValueError("oracle rejected the lattice parameters")
        self.steps = 0

    def step(self, n=1):
        rc = lib().orc_step(C.byref(self.p), _ptr(self.f), _ptr(self.g), int(n))
        if rc:
            raise RuntimeError("oracle step failed (%d)" % rc)
        self.steps += int(n)

    def macros(self):
        n = self.nx * self.ny
        rho, ux, uy, T = _vec(n), _vec(n), _vec(n), _vec(n)
        rc = lib().orc_macros(C.byref(self.p), _ptr(self.f), _ptr(self.g), _ptr(rho), _ptr(ux),
                              _ptr(uy), _ptr(T))
        if rc:
            raise RuntimeError("oracle macros failed")
        shp = (self.ny, self.nx)
        return dict(rho=rho.reshape(shp), ux=ux.reshape(shp), uy=uy.reshape(shp),
                    T=T.reshape(shp))

    def nusselt(self, side=WEST, dT=1.0, local=False):
        nw = self.ny if side in (WEST, EAST) else self.nx
        loc = _vec(nw)
        nu = lib().orc_nusselt(C.byref(self.p), _ptr(self.f), _ptr(self.g), int(side), float(dT),
                               _ptr(loc))
        return (nu, loc) if local else nu

    # single-node helpers bound to this lattice's relaxation set --------
    def collide_f(self, f, rho, ux, uy, Fx, Fy, phi):
        out = _vec(9)
        f = np.ascontiguousarray(f, dtype=np.float64)
        lib().orc_collide_f(C.byref(self.p), _ptr(f), rho, ux, uy, Fx, Fy, phi, _ptr(out))
        return out

    def collide_g(self, g, T, ux, uy):
        out = _vec(5)
        g = np.ascontiguousarray(g, dtype=np.float64)
        lib().orc_collide_g(C.byref(self.p), _ptr(g), T, ux, uy, _ptr(out))
        return out

    def node_macros(self, f, g, node=0):
        out = _vec(6)
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        lib().orc_node_macros(C.byref(self.p), _ptr(f), _ptr(g), int(node), _ptr(out))
        return out

    def Lambda(self):
        out = _vec(81)
        lib().orc_matrix_Lambda(C.byref(self.p), _ptr(out))
        return out.reshape(9, 9)
