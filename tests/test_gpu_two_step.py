"""GPU: two time steps per launch (clb_set_steps_per_launch(ctx, 2); FP32
planes with FP64 or FP32 arithmetic, FP16 and mixed planes with FP32
arithmetic) against single steps on the same inputs,
over every side kind, the porosity field, the per-row acceleration, the
raw-moment collision, ragged domains narrower and wider than the tiles
(64 x 8; 128 x 8 when every domain of the context is at least 128 wide),
and retirement in clb_run; and against the FP64 oracle.  Interior tiles of the 128-wide kernel skip the per-node side
tests; the wide cases hold both kinds.

Both launch modes do the same arithmetic on the same stored values.  With
FP64 arithmetic the two agree to the last bit (asserted within 1e-12
relative; bit equality is logged): the stochastic rounding into FP32 absorbs
the last-place differences that the compiler's separate choices of fused
multiply-adds in the two kernels can make.  With FP32 arithmetic such a
difference reaches the stored value, so the two modes are held to the FP32
tolerance (1e-6) against each other and against the oracle.  FP16 and mixed
storage are held to 1e-3 between the modes and against the oracle."""
import sys

import numpy as np
import pytest

from paper_2110_05943_amd import inputs, workloads
from tests.cases import cavity, node_errors, node_tol, oracle_lattice, rel_l2, vel_rel_l2

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "needs the MI355X"
    import paper_2110_05943_amd._binding as b
    return b


def hetero_periodic(nx, ny):
    eps = inputs.porosity_map(nx, ny, ell=8, seed=7, eps_min=0.3, eps_max=0.9)
    dp = inputs.particle_diameter_for_mean_Da(eps, 1e-2, nx - 1)
    return dict(nx=nx, ny=ny, bc=("periodic",) * 4, eps=eps, dp=dp, F_phi=-1.0, Ra=1e4, Pr=0.71,
                sigma=0.9, scaling="cavity")


def make_cases(name):
    """The domains of one case (built inside the test: the workloads call the
    library's parameter derivation)."""
    return {
        "cavity 97x70": lambda: [cavity(97, ny=70, Ra=1e5, Da=1e-3, phi=0.45, sigma=1.15)],
        "cavity 65x9 (one-column and one-row last tiles)": lambda: [cavity(65, ny=9, Ra=1e4,
                                                                           Da=1e-2)],
        "small cavity 5x4": lambda: [cavity(5, ny=4, Ra=1e3, Da=1e-2)],
        "periodic porosity map 96x80": lambda: [hetero_periodic(96, 80)],
        "periodic narrow 3x17 channel with rows": lambda: [workloads.paper_channel(17, nx=3,
                                                                                   Re=5.0)],
        "inlet/outlet with porosity map": lambda: [workloads.hetero_channel(130, 41, ell=4,
                                                                            seed=2)],
        "mrt batch": lambda: [cavity(64, Ra=1e4, model="mrt"),
                              cavity(70, ny=33, Ra=1e5, model="mrt")],
        "batch of four": lambda: [cavity(64, Ra=1e4), cavity(129, ny=66, Ra=1e5, Da=1e-3, phi=0.4),
                                  hetero_periodic(40, 24), workloads.paper_channel(33, nx=8)],
        # every domain at least 128 wide: 128 x 8 tiles
        "wide cavity 300x37 (ragged last tiles)": lambda: [cavity(300, ny=37, Ra=1e5, Da=1e-3,
                                                                  phi=0.5)],
        "wide periodic porosity map 256x40": lambda: [hetero_periodic(256, 40)],
        "wide mrt 150x30": lambda: [cavity(150, ny=30, Ra=1e5, model="mrt")],
        "wide batch: cavity, channel with rows, inlet/outlet": lambda: [
            cavity(128, ny=20, Ra=1e4), workloads.paper_channel(33, nx=130),
            workloads.hetero_channel(200, 24, ell=4, seed=5)],
        # a narrow domain keeps the 64 x 8 tiles (one general tile body) for
        # every domain of the context, wide ones included
        "mixed widths: 64 x 8 tiles on wide domains": lambda: [
            cavity(40, ny=24, Ra=1e4), cavity(200, ny=50, Ra=1e5, Da=1e-3),
            hetero_periodic(192, 40)],
        "mixed widths, mrt": lambda: [cavity(40, ny=24, Ra=1e4, model="mrt"),
                                      cavity(210, ny=44, Ra=1e5, model="mrt")],
    }[name]()


CASE_NAMES = ["cavity 97x70", "cavity 65x9 (one-column and one-row last tiles)",
              "small cavity 5x4", "periodic porosity map 96x80",
              "periodic narrow 3x17 channel with rows", "inlet/outlet with porosity map",
              "mrt batch", "batch of four", "wide cavity 300x37 (ragged last tiles)",
              "wide periodic porosity map 256x40", "wide mrt 150x30",
              "wide batch: cavity, channel with rows, inlet/outlet",
              "mixed widths: 64 x 8 tiles on wide domains", "mixed widths, mrt"]


def start(s, cases):
    for k, c in enumerate(cases):
        if "inlet_U" in c and c.get("bc", ("",))[0] == "inlet":
            continue  # the channel starts from its own initial state
        u, v, T = inputs.random_fields(c["nx"], c["ny"], seed=3 + k, u_amp=0.01, T_amp=0.2)
        s.set_state(k, T, u, v)


# FP32 planes with FP64 arithmetic on every case; with FP32 arithmetic on a
# subset reaching both tile widths, both tile paths, walls, periodic sides,
# inlet/outlet, per-row acceleration and MRT
F32C_CASES = ["cavity 97x70", "periodic narrow 3x17 channel with rows",
              "inlet/outlet with porosity map", "mrt batch", "wide cavity 300x37 (ragged last tiles)",
              "wide batch: cavity, channel with rows, inlet/outlet", "mixed widths, mrt"]


@pytest.mark.parametrize("name,storage", [(n, "f32") for n in CASE_NAMES] +
                         [(n, "f32c") for n in F32C_CASES] +
                         [(n, st) for n in F32C_CASES for st in ("f16", "mixed")])
def test_two_step_launches_match_single_steps(B, name, storage):
    cases = [dict(c, storage=storage) for c in make_cases(name)]
    log(name, storage)
    runs = []
    for k in (1, 2):
        s = B.Solver(cases)
        s.set_steps_per_launch(k)
        start(s, cases)
        s.step(1)
        s.step(77)   # odd: pairs plus a single step, graphs of 32
        s.step(64)
        runs.append(s)
    a, b = runs
    for i, c in enumerate(cases):
        ma, mb = a.macros(i), b.macros(i)
        d = max(vel_rel_l2(mb, ma), rel_l2(mb["T"], ma["T"]), rel_l2(mb["rho"] - 1, ma["rho"] - 1))
        same = all(np.array_equal(ma[k], mb[k]) for k in ma)
        log("  domain %d (%dx%d): max rel-L2 difference %.2e, bit-identical %s"
            % (i, c["nx"], c["ny"], d, same))
        assert d <= {"f32": 1e-12, "f32c": 1e-6}.get(storage, 1e-3)
    ra, rb = a.residual_all(), b.residual_all()
    if storage == "f32":
        assert np.allclose(ra[0], rb[0], rtol=1e-9, atol=0)
        assert np.allclose(ra[2], rb[2], rtol=1e-12)
    elif storage == "f32c":
        assert np.allclose(ra[2], rb[2], rtol=1e-9)  # mass
    else:
        assert np.allclose(ra[2], rb[2], rtol=1e-6)  # mass with FP16 flow planes
    assert a.steps_done == b.steps_done == 142


# (domains, the domains compared).  The 128-wide compared domain holds both
# edge tiles and interior tiles (regions clear of every side, run without the
# per-node side tests).
ORACLE_CASES = {
    "64 x 8 tiles": ([(100, 40)], [0]),
    "128 x 8 tiles": ([(260, 40)], [0]),
    "64 x 8 tiles, narrow and wide domain": ([(40, 24), (260, 40)], [0, 1]),
}


@pytest.mark.parametrize("name", list(ORACLE_CASES))
@pytest.mark.parametrize("storage", ["f32", "f32c", "mixed", "f16"])
def test_two_step_launches_match_oracle(B, name, storage):
    sizes, compared = ORACLE_CASES[name]
    cases = [cavity(nx, ny=ny, Ra=1e3, Da=1e-2, phi=0.6, storage=storage) for nx, ny in sizes]
    s = B.Solver(cases)
    s.set_steps_per_launch(2)
    for i, (nx, ny) in enumerate(sizes):
        s.set_state(i, inputs.cavity_initial_T(nx, seed=1, ny=ny))
    s.step(5000)
    # FP32 planes (FP64 or FP32 arithmetic): 1e-6; FP16 planes: 1e-3.  The
    # hot-wall Nusselt number with all-FP16 storage carries the FP16
    # temperature noise (~1e-4) times the wall gradient's length scale (the
    # domain width, up to 259 here): a standard deviation of 1e-2 on the
    # 260 x 40 cavity over 32 independent rounding streams, held to 4e-2.
    tol = {"f32": 1e-6, "f32c": 1e-6}.get(storage, 1e-3)
    tol_nu = 4e-2 if storage == "f16" else 1e-4
    for k in compared:
        case = cases[k]
        lat = oracle_lattice(case)
        lat.init_equilibrium(inputs.cavity_initial_T(sizes[k][0], seed=1, ny=sizes[k][1]))
        lat.step(5000)
        g, o = s.macros(k), lat.macros()
        eu, eT = vel_rel_l2(g, o), rel_l2(g["T"], o["T"])
        nu_, nT = node_errors(g, o)
        log("two-step %s %s, domain %dx%d, 5000 steps: rel-L2 u %.2e T %.2e  worst node u %.2e "
            "T %.2e" % (name, storage, case["nx"], case["ny"], eu, eT, nu_, nT))
        assert eu <= tol and eT <= tol
        assert nu_ <= node_tol(tol) and nT <= node_tol(tol)
        assert abs(s.nusselt(k, 0) - lat.nusselt(0)) <= tol_nu


def test_two_step_run_with_retirement_matches(B):
    cases = [cavity(32, Ra=1e3, Da=1e-2), cavity(48, Ra=1e4, Da=1e-2)]
    out = []
    for k in (1, 2):
        s = B.Solver(cases)
        s.set_steps_per_launch(k)
        for i in range(2):
            s.set_state(i, inputs.cavity_initial_T(cases[i]["nx"], seed=1))
        r = s.run(60000, check_every=1000, tol=1e-6)
        out.append((r["steps"].copy(), s.macros(1)["T"]))
    log("steps single %s two-step %s" % (out[0][0], out[1][0]))
    assert np.array_equal(out[0][0], out[1][0])
    assert rel_l2(out[1][1], out[0][1]) <= 1e-12


def test_steps_per_launch_argument(B):
    for st in ("f32", "f32c", "f16", "mixed"):
        s = B.Solver(cavity(32, Ra=1e3, storage=st))
        s.set_steps_per_launch(2)
        s.set_steps_per_launch(1)
        with pytest.raises(B.CLBError):
            s.set_steps_per_launch(3)


def test_default_launch_mode(B):
    """At creation: two steps per launch, on 128-wide tiles when every domain
    is at least 128 wide, else on 64-wide ones; all-FP16 storage takes two
    steps per launch only with 128-wide tiles, else one."""
    wide, mixed = [(260, 40)], [(40, 24), (260, 40)]
    for st in ("f32", "f32c", "mixed", "f16"):
        s = B.Solver([cavity(nx, ny=ny, storage=st) for nx, ny in wide])
        assert s.get_steps_per_launch() == (2, 128), st
        s.close()
        s = B.Solver([cavity(nx, ny=ny, storage=st) for nx, ny in mixed])
        assert s.get_steps_per_launch()[0] == (1 if st == "f16" else 2), st
        if st != "f16":
            assert s.get_steps_per_launch() == (2, 64), st
        s.close()


def test_wide_tiles_forced_on_a_narrow_domain(B, tmp_path):
    """clb_create picks 64-wide two-step tiles when a domain is narrower
    than 128; a cached tuning choice can impose 128-wide tiles on every
    domain (the narrow domain then sits in one masked 128 x 8 tile per row
    band) or per-domain widths (two launches per pair of steps, reported as
    width 0).  The results must equal single steps bit for bit."""
    cases = [cavity(40, ny=24, Ra=1e4, sigma=1.1), cavity(260, ny=40, Ra=1e5, Da=1e-3, phi=0.5)]
    Ts = [inputs.cavity_initial_T(c["nx"], seed=3 + k, ny=c["ny"]) for k, c in enumerate(cases)]
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    cache = tmp_path / "tune.txt"
    cache.write_text("storage=0;n=2;nodes=%d;first=40x24 0 0 0 128\n" % nodes)
    a = B.Solver(cases)
    assert a.get_steps_per_launch() == (2, 64)
    a.autotune(str(cache))
    assert a.get_steps_per_launch() == (2, 128) and a.steps_done == 0
    cache2 = tmp_path / "tune2.txt"
    cache2.write_text("storage=0;n=2;nodes=%d;first=40x24 0 0 0 1\n" % nodes)
    c = B.Solver(cases)
    c.autotune(str(cache2))
    assert c.get_steps_per_launch() == (2, 0) and c.steps_done == 0
    b = B.Solver(cases)
    b.set_steps_per_launch(1)
    for s in (a, b, c):
        for k, T in enumerate(Ts):
            s.set_state(k, T)
        s.step(101)
    for k in range(len(cases)):
        mb = b.macros(k)
        for name, s in (("forced 128-wide", a), ("per-domain", c)):
            ms = s.macros(k)
            same = all(np.array_equal(ms[q], mb[q]) for q in ms)
            log("%s tiles, domain %d: bit-identical %s" % (name, k, same))
            assert same
