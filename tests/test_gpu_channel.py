"""GPU parity on the heterogeneous mixed-convection channel: the full
2048 x 2048 workload on sampled nodes, and a 256 x 256 crop of its porosity
map as a channel of its own over 6000 steps."""
import math
import sys

import numpy as np
import pytest

from paper_2110_05943_amd import inputs, workloads
from tests.cases import (node_errors, node_tol, oracle_lattice, oracle_values, rel_l2,
                         sampled_oracle, vel_rel_l2)

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def Solver():
    import torch
    assert torch.cuda.is_available(), "needs the MI355X"
    from paper_2110_05943_amd import Solver as S
    return S


@pytest.fixture(scope="module")
def eps2048():
    return inputs.porosity_map(2048, 2048, ell=32, seed=4)


@pytest.mark.parametrize("storage,tol", [("f32", 2e-6), ("f32c", 2e-6), ("f16", 2e-3),
                                         ("mixed", 2e-3)])
def test_channel_2048_sampled(Solver, eps2048, storage, tol):
    """2048^2 channel with its porosity map in the default launch shape: 6
    steps from a smooth random state; 72 sampled nodes (inlet, outlet, walls,
    corners, interior) against the oracle on their dependence windows."""
    n, k = 2048, 6
    case = workloads.hetero_channel(n, n, eps=eps2048, storage=storage)
    fields = inputs.random_fields(n, n, seed=43, u_amp=0.03, T_amp=0.4, smooth=2)
    u, v, T = fields
    s = Solver(case)
    s.set_state(0, T, u, v)
    s.step(k)
    g = s.macros()
    r = inputs.rng(98)
    pts = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (0, 1), (0, 700), (0, n - 2),
           (1, 1500), (n - 1, 300), (n - 2, 5), (900, 0), (1200, n - 1), (3, n - 2)]
    pts += [(int(a), int(b)) for a, b in r.integers(0, n, (59, 2))]
    vals = oracle_values(case)
    worst = 0.0
    for (x, y) in pts:
        o = sampled_oracle(case, vals, fields, x, y, k)
        uo, vo, To = o["ux"], o["uy"], o["T"]
        du = math.hypot(g["ux"][y, x] - uo, g["uy"][y, x] - vo) / max(math.hypot(uo, vo), 1e-3)
        dT = abs(g["T"][y, x] - To)  # relative to the wall temperature difference (1)
        worst = max(worst, du, dT)
        assert du <= tol and dT <= tol, ((x, y), du, dT)
    log("2048^2 channel %s sampled worst relative error %.3e" % (storage, worst))
    s.close()


@pytest.fixture(scope="module")
def crop_oracle(eps2048):
    case = workloads.hetero_channel(256, 256, eps=eps2048[:256, :256].copy())
    lat = oracle_lattice(case)
    lat.init_equilibrium(0.0)
    lat.step(6000)
    return lat.macros(), lat.nusselt(2, 1.0)


@pytest.mark.parametrize("storage,tol", [("f32", 1e-6), ("f32c", 1e-6), ("mixed", 1e-3),
                                         ("f16", 1e-3)])
def test_channel_crop_256_6000_steps(Solver, eps2048, crop_oracle, storage, tol):
    """The 256^2 corner of the same porosity map as its own channel (H = 255,
    same U, Re, Ri), from rest at T = 0, 6000 steps (about one flow-through
    time)."""
    case = workloads.hetero_channel(256, 256, eps=eps2048[:256, :256].copy(), storage=storage)
    s = Solver(case)
    s.step(6000)
    g = s.macros()
    o, nu_o = crop_oracle
    eu, eT = vel_rel_l2(g, o), rel_l2(g["T"], o["T"])
    nu_, nT = node_errors(g, o)
    nu_g = s.nusselt(0, 2)
    log("crop 256 %s rel-L2 u=%.3e T=%.3e  worst node u=%.3e T=%.3e  Nu(bottom) gpu=%.6f "
        "oracle=%.6f" % (storage, eu, eT, nu_, nT, nu_g, nu_o))
    assert eu <= tol and eT <= tol
    assert nu_ <= node_tol(tol) and nT <= node_tol(tol)
    assert abs(nu_g - nu_o) <= (1e-4 if storage == "f32" else 1e-2) * max(1.0, abs(nu_o))
    s.close()
