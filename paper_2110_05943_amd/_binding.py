"""ctypes binding of libclb.so (include/clb.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides the device workspace (a uint8 tensor) and the HIP stream.
There is no fallback: importing this module without the built library, or
creating a solver without a ROCm GPU, raises.
"""
import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libclb.so")

OK, ERR_ARG, ERR_HIP, ERR_WORKSPACE, ERR_DIVERGED, ERR_STATE, NOT_CONVERGED = range(7)
PERIODIC, WALL_T, WALL_ADIABATIC, INLET, OUTLET = range(5)
WEST, EAST, SOUTH, NORTH = range(4)
STORE_F32, STORE_F16, STORE_MIXED, STORE_F32C = 0, 1, 2, 3
SCALE_CAVITY, SCALE_CHANNEL = 0, 1
KIND = {"periodic": PERIODIC, "wall_T": WALL_T, "wall_adiabatic": WALL_ADIABATIC,
        "inlet": INLET, "outlet": OUTLET}
STORAGE = {"f32": STORE_F32, "f16": STORE_F16, "mixed": STORE_MIXED, "f32c": STORE_F32C}
MODEL = {"clb": 0, "mrt": 1, "bgk": 2}
FORCING = {"none": 0, "injection": 1}
# bytes moved per node update (14 populations read and written)
BYTES_PER_UPDATE = {"f32": 112, "f16": 56, "mixed": 76, "f32c": 112}


class CLBError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what, _lib().clb_strerror(status).decode(), status))


class DivergedError(CLBError):
    pass


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32 * 4),
        ("bc_u", C.c_double * 4), ("bc_v", C.c_double * 4), ("bc_T", C.c_double * 4),
        ("inlet_U", C.c_double),
        ("phi", C.c_double), ("eps", C.POINTER(C.c_double)), ("dp", C.c_double),
        ("Da", C.c_double), ("F_phi", C.c_double),
        ("scaling", C.c_int32),
        ("Ra", C.c_double), ("Pr", C.c_double), ("Re", C.c_double), ("J", C.c_double),
        ("Gamma", C.c_double), ("sigma", C.c_double), ("Ma", C.c_double),
        ("u_ref", C.c_double), ("dT", C.c_double), ("T0", C.c_double),
        ("g_dir", C.c_double * 2), ("a", C.c_double * 2),
        ("nu", C.c_double), ("s_v", C.c_double), ("s_b", C.c_double), ("s1", C.c_double),
        ("s3", C.c_double), ("s4", C.c_double), ("zeta_a", C.c_double), ("zeta_e", C.c_double),
        ("zeta_nu", C.c_double), ("varpi", C.c_double), ("gbeta", C.c_double),
        ("T_init", C.c_double), ("storage", C.c_int32), ("model", C.c_int32),
        ("a_rows", C.POINTER(C.c_double)), ("forcing", C.c_int32),
    ]


class Derived(C.Structure):
    _fields_ = [(n, C.c_double) for n in (
        "L", "s_v", "s_b", "s1", "s3", "s4", "zeta_a", "zeta_e", "zeta_nu", "varpi",
        "nu_e", "nu", "alpha_e", "gbeta", "K", "F_phi", "sigma", "T0", "dT")]


EXPORTS = (
    "clb_params_default", "clb_derive", "clb_row_accel", "clb_workspace_bytes", "clb_create", "clb_step",
    "clb_macros", "clb_nusselt", "clb_nusselt_all", "clb_residual", "clb_residual_all",
    "clb_set_state", "clb_set_state_device", "clb_set_active", "clb_run", "clb_state_bytes", "clb_get_state", "clb_put_state",
    "clb_steps_done", "clb_set_launch", "clb_get_launch", "clb_set_steps_per_launch",
    "clb_get_steps_per_launch",
    "clb_autotune", "clb_destroy",
    "clb_strerror",
)

_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libclb.so is not built (run __graft_entry__.build() or "
                              "python paper_2110_05943_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        P, D, vp, dp = C.POINTER(Params), C.POINTER(Derived), C.c_void_p, C.POINTER(C.c_double)
        st = C.c_int
        sig = {
            "clb_params_default": (None, [P]),
            "clb_derive": (st, [P, D]),
            "clb_row_accel": (st, [P, dp]),
            "clb_workspace_bytes": (st, [P, C.c_int32, C.POINTER(C.c_size_t)]),
            "clb_create": (st, [P, C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "clb_step": (st, [vp, C.c_int64]),
            "clb_macros": (st, [vp, C.c_int32, dp, dp, dp, dp]),
            "clb_nusselt": (st, [vp, C.c_int32, C.c_int32, dp, dp]),
            "clb_nusselt_all": (st, [vp, C.c_int32, dp]),
            "clb_residual": (st, [vp, C.c_int32, dp, dp, dp]),
            "clb_residual_all": (st, [vp, dp, dp, dp, C.POINTER(C.c_int32)]),
            "clb_set_state": (st, [vp, C.c_int32, dp, dp, dp]),
            "clb_set_active": (st, [vp, C.POINTER(C.c_uint8)]),
            "clb_run": (st, [vp, C.c_int64, C.c_int32, C.c_double, C.c_int32, dp, C.c_int32,
                             C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
            "clb_state_bytes": (st, [vp, C.POINTER(C.c_size_t)]),
            "clb_get_state": (st, [vp, vp, C.c_size_t]),
            "clb_put_state": (st, [vp, vp, C.c_size_t]),
            "clb_steps_done": (st, [vp, C.POINTER(C.c_int64)]),
            "clb_set_launch": (st, [vp, C.c_int32, C.c_int32, C.c_int32]),
            "clb_set_steps_per_launch": (st, [vp, C.c_int32]),
            "clb_get_steps_per_launch": (st, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
            "clb_get_launch": (st, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)]),
            "clb_autotune": (st, [vp, C.c_char_p]),
            "clb_destroy": (None, [vp]),
            "clb_strerror": (C.c_char_p, [st]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _L = L
    return _L


def _check(status, what):
    if status == ERR_DIVERGED:
        raise DivergedError(status, what)
    if status != OK:
        raise CLBError(status, what)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def make_params(**kw):
    """A Params struct: library defaults, then the given fields.

    bc may be given as kind names; eps as an (ny, nx) array; a_rows as an
    (ny, 2) array of (a_x, a_y) per row; storage as "f32"/"f16"/"mixed"/"f32c"; two-element
    fields as sequences."""
    p = Params()
    _lib().clb_params_default(C.byref(p))
    keep = []
    for k, v in kw.items():
        if k == "bc":
            for s in range(4):
                p.bc[s] = KIND[v[s]] if isinstance(v[s], str) else int(v[s])
        elif k in ("bc_u", "bc_v", "bc_T"):
            for s in range(4):
                getattr(p, k)[s] = float(v[s])
        elif k in ("g_dir", "a"):
            getattr(p, k)[0], getattr(p, k)[1] = float(v[0]), float(v[1])
        elif k in ("eps", "a_rows"):
            if v is None:
                setattr(p, k, None)
            else:
                arr = np.ascontiguousarray(np.asarray(v, dtype=np.float64).reshape(-1))
                keep.append(arr)
                setattr(p, k, _dptr(arr))
        elif k == "storage":
            p.storage = STORAGE[v] if isinstance(v, str) else int(v)
        elif k == "model":
            p.model = MODEL[v] if isinstance(v, str) else int(v)
        elif k == "forcing":
            p.forcing = FORCING[v] if isinstance(v, str) else int(v)
        elif k == "scaling":
            p.scaling = {"cavity": SCALE_CAVITY, "channel": SCALE_CHANNEL}.get(v, v)
        else:
            setattr(p, k, v)
    p._keep = keep
    return p


def derive(**kw):
    """Lattice parameters the library derives for one domain (host only)."""
    p = make_params(**kw)
    d = Derived()
    _check(_lib().clb_derive(C.byref(p), C.byref(d)), "clb_derive")
    return {n: getattr(d, n) for n, _ in Derived._fields_}


def row_accel(**kw):
    """The per-row acceleration (ny, 2) the library applies to one domain:
    a_rows plus the built-in forcing (host only)."""
    p = make_params(**kw)
    out = np.zeros(2 * p.ny, dtype=np.float64)
    _check(_lib().clb_row_accel(C.byref(p), _dptr(out)), "clb_row_accel")
    return out.reshape(p.ny, 2)


class Solver:
    """One or many domains advanced by the HIP library on one GPU.

    params: a dict (one domain) or a list of dicts of make_params fields.
    The workspace is a torch uint8 tensor on `device`; all work runs on a
    dedicated torch stream (self.stream).
    """

    def __init__(self, params, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the CLB library needs a ROCm GPU; none is visible")
        plist = [params] if isinstance(params, dict) else list(params)
        self.count = len(plist)
        arr = (Params * self.count)()
        keep = []
        self.shapes = []
        for i, kw in enumerate(plist):
            p = make_params(**kw)
            keep.append(p._keep)
            arr[i] = p
            self.shapes.append((p.ny, p.nx))
        L = _lib()
        nbytes = C.c_size_t(0)
        _check(L.clb_workspace_bytes(arr, self.count, C.byref(nbytes)), "clb_workspace_bytes")
        self.device = torch.device(device)
        self.workspace_bytes = nbytes.value
        self._ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        ctx = C.c_void_p()
        _check(L.clb_create(arr, self.count, C.c_void_p(self._ws_ptr), nbytes.value,
                            C.c_void_p(self.stream.cuda_stream), C.byref(ctx)), "clb_create")
        self._ctx = ctx
        del keep

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            self.stream.synchronize()
            _lib().clb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(_lib().clb_step(self._ctx, int(n)), "clb_step")

    def synchronize(self):
        self.stream.synchronize()

    def macros(self, cavity=0):
        ny, nx = self.shapes[cavity]
        out = [np.empty((ny, nx), dtype=np.float64) for _ in range(4)]
        _check(_lib().clb_macros(self._ctx, cavity, *[_dptr(a) for a in out]), "clb_macros")
        return dict(rho=out[0], ux=out[1], uy=out[2], T=out[3])

    def nusselt(self, cavity=0, side=WEST, local=False):
        ny, nx = self.shapes[cavity]
        m = C.c_double()
        loc = np.empty(ny if side in (WEST, EAST) else nx, dtype=np.float64)
        _check(_lib().clb_nusselt(self._ctx, cavity, side, C.byref(m),
                                  _dptr(loc) if local else None), "clb_nusselt")
        return (m.value, loc) if local else m.value

    def nusselt_all(self, side=WEST):
        out = np.empty(self.count, dtype=np.float64)
        _check(_lib().clb_nusselt_all(self._ctx, side, _dptr(out)), "clb_nusselt_all")
        return out

    def residual(self, cavity=0):
        ru, rT, m = C.c_double(), C.c_double(), C.c_double()
        _check(_lib().clb_residual(self._ctx, cavity, C.byref(ru), C.byref(rT), C.byref(m)),
               "clb_residual")
        return ru.value, rT.value, m.value

    def residual_all(self):
        ru, rT, m = (np.empty(self.count) for _ in range(3))
        status = np.empty(self.count, dtype=np.int32)
        _check(_lib().clb_residual_all(self._ctx, _dptr(ru), _dptr(rT), _dptr(m),
                                       status.ctypes.data_as(C.POINTER(C.c_int32))),
               "clb_residual_all")
        return ru, rT, m, status

    def set_state(self, cavity, T, ux=None, uy=None):
        def flat(a):
            if a is None:
                return None
            return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
        T, ux, uy = flat(T), flat(ux), flat(uy)
        _check(_lib().clb_set_state(self._ctx, cavity, _dptr(ux), _dptr(uy), _dptr(T)),
               "clb_set_state")

    def set_active(self, active):
        a = np.ascontiguousarray(np.asarray(active, dtype=np.uint8))
        _check(_lib().clb_set_active(self._ctx, a.ctypes.data_as(C.POINTER(C.c_uint8))),
               "clb_set_active")

    def run(self, max_steps, check_every=100, tol=1e-8, nu_side=None, max_records=0):
        """Run the active domains to steady state (clb_run).

        Returns dict(steps=int64[count], status=int32[count], nu=(count,
        max_records) array or None)."""
        steps = np.zeros(self.count, dtype=np.int64)
        status = np.zeros(self.count, dtype=np.int32)
        nu = None
        if nu_side is not None and max_records > 0:
            nu = np.empty((self.count, max_records), dtype=np.float64)
        _check(_lib().clb_run(self._ctx, int(max_steps), int(check_every), float(tol),
                              -1 if nu_side is None else int(nu_side),
                              _dptr(nu), int(max_records),
                              steps.ctypes.data_as(C.POINTER(C.c_int64)),
                              status.ctypes.data_as(C.POINTER(C.c_int32))), "clb_run")
        return dict(steps=steps, status=status, nu=nu)

    def get_state(self):
        n = C.c_size_t()
        _check(_lib().clb_state_bytes(self._ctx, C.byref(n)), "clb_state_bytes")
        buf = np.empty(n.value, dtype=np.uint8)
        _check(_lib().clb_get_state(self._ctx, buf.ctypes.data_as(C.c_void_p), n.value),
               "clb_get_state")
        return buf

    def put_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        _check(_lib().clb_put_state(self._ctx, buf.ctypes.data_as(C.c_void_p), buf.size),
               "clb_put_state")

    @property
    def steps_done(self):
        s = C.c_int64()
        _check(_lib().clb_steps_done(self._ctx, C.byref(s)), "clb_steps_done")
        return s.value

    def set_launch(self, tile_x, tile_y, blocks=0):
        _check(_lib().clb_set_launch(self._ctx, tile_x, tile_y, blocks), "clb_set_launch")

    def set_steps_per_launch(self, steps):
        """1 or 2 time steps per kernel launch (any storage mode)."""
        _check(_lib().clb_set_steps_per_launch(self._ctx, int(steps)), "clb_set_steps_per_launch")

    def get_steps_per_launch(self):
        """(steps per launch, two-step tile width in nodes)."""
        a, b = C.c_int32(), C.c_int32()
        _check(_lib().clb_get_steps_per_launch(self._ctx, C.byref(a), C.byref(b)),
               "clb_get_steps_per_launch")
        return a.value, b.value

    def get_launch(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib().clb_get_launch(self._ctx, C.byref(a), C.byref(b), C.byref(c)),
               "clb_get_launch")
        return a.value, b.value, c.value

    def autotune(self, cache_path=None):
        _check(_lib().clb_autotune(self._ctx, cache_path.encode() if cache_path else None),
               "clb_autotune")
        return self.get_launch()
