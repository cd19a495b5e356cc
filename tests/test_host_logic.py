"""CPU checks of the host-side logic: input draws, workload parameter sets,
the steady-state bookkeeping of the warm-start driver."""
import math

import numpy as np
import pytest

from paper_2110_05943_amd import inputs, warmstart, workloads


def test_warmstart_draws_are_seeded_and_in_range():
    a = inputs.warmstart_draws(6, seed=0, n=32)
    b = inputs.warmstart_draws(6, seed=0, n=32)
    c = inputs.warmstart_draws(6, seed=1, n=32)
    for x, y in zip(a, b):
        assert x["Ra"] == y["Ra"] and np.array_equal(x["eps"], y["eps"])
    assert a[0]["Ra"] != c[0]["Ra"]
    # sample i does not depend on how many samples are drawn
    assert inputs.warmstart_draws(2, seed=0, n=32)[1]["Da"] == a[1]["Da"]
    for d in a:
        assert 1e3 <= d["Ra"] <= 1e7 and 1e-5 <= d["Da"] <= 1e-1
        assert d["Pr"] in (0.71, 1.0, 7.0) and 0.8 <= d["sigma"] <= 1.2
        assert d["eps"].min() >= 0.3 and d["eps"].max() <= 0.95
        assert np.array_equal(d["eps"], d["eps"].astype(np.float32).astype(np.float64))


def test_porosity_map_has_uniform_marginal_and_mean_darcy_number():
    eps = inputs.porosity_map(256, 256, ell=8, seed=4)
    hist, _ = np.histogram(eps, bins=6, range=(0.3, 0.9))
    assert hist.min() > 0.6 * hist.mean()  # roughly flat
    dp = inputs.particle_diameter_for_mean_Da(eps, 1e-3, 255)
    K = eps ** 3 * dp ** 2 / (150 * (1 - eps) ** 2)
    assert math.isclose(K.mean() / 255 ** 2, 1e-3, rel_tol=1e-12)


def test_groups_normalisation_spans_unit_range():
    lo = warmstart.groups_of(dict(Ra=1e3, Da=1e-5, Pr=0.71, sigma=0.8))
    hi = warmstart.groups_of(dict(Ra=1e7, Da=1e-1, Pr=7.0, sigma=1.2))
    assert np.allclose(lo, [-1, -1, -1.0, -1], atol=0.05)
    assert np.allclose(hi, [1, 1, 1.0, 1], atol=0.05)


def test_settle_steps():
    nu = [2.0, 1.5, 1.2, 1.10005, 1.1, 1.10002]
    # records after 100, 200, ... steps; within 1e-4 of 1.1 from record 3 on
    assert warmstart.settle_steps(nu, 1.1, 100) == 400
    assert warmstart.settle_steps([1.1, 1.1], 1.1, 100) == 100
    assert warmstart.settle_steps([1.0, 1.2], 1.1, 100) is None
    assert warmstart.settle_steps([], 1.1, 100) is None


def test_workload_parameter_sets():
    b = workloads.batch(16, seed=3)
    assert len(b) == 16 and {c["nx"] for c in b} <= {64, 128, 256, 512}
    assert all(c["bc"] == workloads.CAVITY_BC for c in b)
    ch = workloads.hetero_channel(64, 32, ell=4, seed=1)
    assert ch["bc"] == ("inlet", "outlet", "wall_T", "wall_T")
    assert ch["eps"].shape == (32, 64)
    # Ri = g beta dT H / U^2 = 1
    assert math.isclose(ch["gbeta"] * 31 / ch["inlet_U"] ** 2, 1.0)


def test_paper_channel_forcing_matches_eq42_and_closed_form():
    # The library's per-row acceleration (clb_row_accel: Eq. 42 evaluated in
    # clb_create from its own derivation) against Eq. 42 with the oracle's
    # derivation of nu, K, alpha_e and g beta dT, on every channel case of
    # the GPU tests; the closed form meets the plate conditions of Fig. 1.
    from paper_2110_05943_amd._binding import row_accel
    from tests.cases import injection_rows
    from tests.closed_forms import paper_channel_exact
    cases = [workloads.paper_channel(33, Re=5.0, u1=0.01),
             workloads.paper_channel(33, nx=8, Re=5.0),
             workloads.paper_channel(25, nx=40, s_v=1.2, Re=10.0),
             workloads.paper_channel(32, nx=32, s_v=1.0 / 0.5015, Re=5.0),
             workloads.paper_channel(32, nx=32, Re=1.0), workloads.paper_channel(32, nx=32, Re=20.0)]
    cases += [workloads.paper_channel(n, s_v=1.0, Re=5.0) for n in (17, 33, 49, 65, 81, 97)]
    for c in cases:
        lib = row_accel(**c)
        ay = injection_rows(c)
        assert np.all(lib[:, 0] == 0)
        assert np.allclose(lib[:, 1], ay, rtol=1e-12, atol=1e-18), c["ny"]
        ux, uy, T = paper_channel_exact(c)
        u1 = c["bc_v"][2]
        assert ux[0] == 0 and math.isclose(ux[-1], c["bc_u"][3]) and np.all(uy == u1)
        assert T[0] == 0 and math.isclose(T[-1], 1.0)
    # a_rows given beside the built-in forcing is added to it
    c = workloads.paper_channel(17, Re=5.0)
    extra = np.stack([np.full(17, 1e-6), np.full(17, 2e-6)], axis=1)
    both = row_accel(**dict(c, a_rows=extra))
    assert np.allclose(both, row_accel(**c) + extra, rtol=0, atol=1e-18)
    assert np.all(row_accel(**dict(c, forcing="none")) == 0)
    # the convergence-study form: u1 follows from s_v = 1 and Re
    c1 = workloads.paper_channel(17, s_v=1.0, Re=5.0)
    assert math.isclose(c1["u_ref"], 5.0 * (1 / 6) / 16)
    # Eq. 42 needs a uniform medium with a finite permeability
    from paper_2110_05943_amd._binding import CLBError
    with pytest.raises(CLBError):
        row_accel(**dict(c, Da=0.0))
