"""The seeded synthetic inputs (workloads.py) against the configurations they stand for:
extents, material parameters and the sampling rules of the sweep family.  A drifted
generator fails here before any parity test compares the wrong problem."""
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import workloads  # noqa: E402


def test_couette_fenep_configuration():
    """16x32x16, one component, tau = 1 (eta_s = 1/6), eta_p/(eta_s + eta_p) = 0.2, tau_p =
    1000, L^2 = 100, walls at -+0.01, linear start, C = I plus symmetric noise of 1e-3."""
    wl = workloads.couette_fenep()
    g, p = wl["grid"], wl["params"]
    assert (g["nx"], g["ny"], g["nz"], g["ncomp"]) == (16, 32, 16, 1)
    eta_s = (p["tau_A"] - 0.5) / 3.0
    assert abs(eta_s - 1.0 / 6.0) < 1e-15
    assert abs(p["eta_p"] / (eta_s + p["eta_p"]) - 0.2) < 1e-12
    assert p["tau_p"] == 1000.0 and p["L2"] == 100.0 and p["G"] == 0.0
    assert wl["walls"]["u_bottom"] == [-0.01, 0.0, 0.0] and wl["walls"]["u_top"] == [0.01, 0.0, 0.0]
    C = wl["C"]
    assert np.abs(C[:3] - 1.0).max() <= 1e-3 and np.abs(C[3:]).max() <= 1e-3 and np.abs(C[3:]).max() > 0
    # the start is the half-way-wall Couette profile: linear in y, odd about the centre
    u = wl["u"][0].reshape(16, 32, 16)[0, :, 0]
    assert np.allclose(u, -u[::-1]) and np.allclose(np.diff(u), 0.02 / 32)
    # the same seed gives the same noise
    assert np.array_equal(workloads.couette_fenep()["C"], C)


def test_droplet_configurations():
    """128x64x128 with R = 16 (2R/H = 0.5), polymer in the droplet, L^2 = 100; the large run
    1024x256x1024 with a Newtonian droplet R = 64 and a viscoelastic matrix (L^2 = 400,
    De = 1); both densities 1.0 inside / 0.04 outside, reversed for B."""
    w1 = workloads.droplet_cfg1(De=0.5, variant="physics")
    assert (w1["grid"]["nx"], w1["grid"]["ny"], w1["grid"]["nz"], w1["grid"]["ncomp"]) == (128, 64, 128, 2)
    assert w1["params"]["polymer_phase"] == "A" and w1["params"]["L2"] == 100.0
    rho = w1["rho"]
    assert set(np.unique(rho[0])) == {1.0, 0.04} and np.array_equal(rho[0] + rho[1], np.full(rho.shape[1], 1.04))
    inside = (rho[0] == 1.0).sum()
    assert abs(inside - 4.0 / 3.0 * math.pi * 16 ** 3) < 0.02 * inside
    # a 1-plane slab of the large configuration (the full grid is built slab by slab)
    w2 = workloads.droplet_cfg2(box=(0, 1024, 512, 1))
    p2 = w2["params"]
    assert w2["grid"]["ny"] == 256 and p2["polymer_phase"] == "B" and p2["L2"] == 400.0
    r2 = w2["rho"][0].reshape(256, 1024)
    # the central plane cuts the droplet through its equator: a disc of radius 64
    assert abs((r2 == 1.0).sum() - math.pi * 64 ** 2) < 0.02 * math.pi * 64 ** 2
    assert abs(workloads.G_PHYSICS_1_004 * (1.0 - 0.04) - math.log(1.0 / 0.04)) < 1e-12


def test_sweep_family_sampling_rules():
    """Seed 3: N_x = N_z in {64, 128, 192}, N_y in {32, 48, 64}, R in 8..24 with 2R/H <= 0.75
    and 4R <= N_x, Ca in [0.05, 0.4], De in [0.1, 2], lambda in [0.5, 2], L^2 in {50, 100,
    400}; scale shrinks every length alike; the same seed gives the same cases."""
    cases = workloads.sweep_cases(64, seed=3)
    assert len(cases) == 64 and cases == workloads.sweep_cases(64, seed=3)
    for c in cases:
        assert c["nx"] == c["nz"] and c["nx"] in (64, 128, 192) and c["ny"] in (32, 48, 64)
        assert 8 <= c["R"] <= 24 and 2 * c["R"] / c["ny"] <= 0.75 and 4 * c["R"] <= c["nx"]
        assert 0.05 <= c["Ca"] <= 0.4 and 0.1 <= c["De"] <= 2.0 and 0.5 <= c["lam"] <= 2.0
        assert c["L2"] in (50.0, 100.0, 400.0) and c["polymer_phase"] in ("A", "B")
    # both polymer placements and every grid size occur
    assert {c["polymer_phase"] for c in cases} == {"A", "B"}
    assert {c["nx"] for c in cases} == {64, 128, 192}
    half = workloads.sweep_cases(8, seed=3, scale=0.5)
    for c in half:
        assert c["nx"] in (32, 64, 96) and c["ny"] in (16, 24, 32)
    # the viscosity ratio sets tau_A against the matrix's tau_B
    w = workloads.sweep_workload(cases[0])
    tB = w["params"]["tau_B"]
    assert abs((w["params"]["tau_A"] - 0.5) / (tB - 0.5) - cases[0]["lam"]) < 1e-12
