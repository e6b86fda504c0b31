"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same
seeded inputs.  Tolerance: relative L2 <= 1e-5 on u, C, C - I and rho, the accuracy
target for FP32 populations and FP32 C (C - I is the informative part of C, whose norm I
dominates).  Sizes span several blocks with ragged tails; the full 128x64x128 droplet grid
is run directly."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads
from parity_helpers import check_diag, grid_shape

pytestmark = pytest.mark.gpu

I6 = np.array([1, 1, 1, 0, 0, 0.0])[:, None]


@pytest.fixture(scope="module")
def lb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1406_2686_amd

    return paper_1406_2686_amd


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def run_both(lb, wl, steps):
    lat = lb.from_workload(wl)
    lat.step(steps)
    g = lat.get_fields()
    dg = lat.diagnostics()
    o = oracle.from_workload(wl)
    assert o.step(steps) == 0
    r = o.get_fields()
    do = o.diagnostics()
    lat.close()
    return g, r, dg, do


def report(tag, g, r):
    errs = {"u": rel(g[1], r[1]), "C": rel(g[2], r[2]), "C-I": rel(g[2] - I6, r[2] - I6),
            "rho": rel(g[0], r[0]), "max|du|": float(np.max(np.abs(g[1] - r[1])))}
    print(tag, " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    return errs


def test_couette_fenep_16x32x16_4000_steps(lb):
    """Single-component FENE-P plane Couette, 4000 steps (noise on C)."""
    wl = workloads.couette_fenep()
    g, r, dg, do = run_both(lb, wl, 4000)
    e = report("couette4000", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-6
    assert e["C-I"] < 1e-5
    assert abs(dg["mass_A"] - do["mass_A"]) < 1e-6 * do["mass_A"]
    # total momentum is ~0 by symmetry: bound the difference by the momentum scale N max|u|
    scale = wl["rho"].size * do["max_u"]
    assert abs(dg["mom_x"] - do["mom_x"]) < 1e-6 * scale


@pytest.mark.parametrize("variant", ["as_written", "physics"])
def test_droplet_128x64x128_full_grid(lb, variant):
    """Two-component viscoelastic droplet on the full 128x64x128 grid, 100 steps."""
    wl = workloads.droplet_cfg1(De=1.0, variant=variant)
    g, r, dg, do = run_both(lb, wl, 100)
    e = report(f"cfg1-{variant}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5
    for k in ("mass_A", "mass_B"):
        assert abs(dg[k] - do[k]) < 1e-6 * do[k]
    assert abs(dg["D"] - do["D"]) < 1e-5 and abs(dg["xc"] - do["xc"]) < 1e-6 * do["xc"]
    check_diag(dg, do, f"cfg1-{variant}", g, r, grid_shape(wl), wl["params"])
    # polymer-phase mean of tr C - 3: the weight f+-(phi) has slope up to 1/(2 Delta) = 5 in
    # phi, so FP32 rounding of phi at interface nodes is amplified five-fold
    assert abs(dg["poly_trace_excess"] - do["poly_trace_excess"]) < 1e-4 * max(1e-3, abs(do["poly_trace_excess"]))


@pytest.mark.parametrize("De", [0.1, 0.5, 1.0])
def test_droplet_128x64x128_1000_steps_each_De(lb, De):
    """The viscoelastic droplet of 2R/H = 0.5 on the full 128x64x128 grid (G at the binodal,
    polymer in the droplet, Ca = 0.2), 1000 steps at each Deborah number of the sweep: u, C,
    C - I and the densities within 1e-5 relative L2 of the FP64 oracle, and every diagnostics
    field within the bounds its field differences allow."""
    wl = workloads.droplet_cfg1(De=De, variant="physics")
    g, r, dg, do = run_both(lb, wl, 1000)
    e = report(f"cfg1-1000-De{De:g}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["C-I"] < 1e-5 and e["rho"] < 1e-5, e
    check_diag(dg, do, f"cfg1-1000-De{De:g}", g, r, grid_shape(wl), wl["params"])


@pytest.mark.parametrize("De", [0.1, 0.5, 1.0])
def test_droplet_128x64x128_20000_steps_against_the_stored_oracle_reference(lb, De):
    """The specified length of the 128x64x128 droplet run: 20,000 steps at each Deborah
    number of the sweep, against the FP64 oracle's fields stored by
    tests/golden/droplet_long_reference.py (every 8th node in x and z, every 4th in y, 4096
    nodes): u, C, C - I and the densities within 1e-5 relative L2 on those nodes; D within
    1e-5 and the angle within 1e-3 degrees of the oracle's diagnostics; species mass to
    1e-6 relative (the FP32 collision's rounding moves a species' mass by about 3e-11 of it
    per step, the same sign every step: 6e-7 after 20,000 steps)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"droplet_long_De{De:g}.npz")
    if not os.path.exists(path):
        pytest.skip(f"no stored reference {os.path.basename(path)} (tests/golden/droplet_long_reference.py writes it)")
    ref = np.load(path)
    steps = int(ref["step"])
    od = json.loads(str(ref["diags"]))[str(steps)]
    wl = workloads.droplet_cfg1(De=De, variant="physics")
    g = grid_shape(wl)
    sel = np.zeros((g[2], g[1], g[0]), bool)
    sel[::8, ::4, ::8] = True
    sel = sel.ravel()
    lat = lb.from_workload(wl)
    lat.step(steps)
    rho, u, C = lat.get_fields()
    d = lat.diagnostics()
    lat.close()
    cmi = C[:, sel] - I6
    e = {"u": rel(u[:, sel], ref["u"]), "C": rel(C[:, sel], ref["CmI"] + I6), "C-I": rel(cmi, ref["CmI"]),
         "rho": rel(rho[:, sel], ref["rho"]), "D": abs(d["D"] - od["D"]), "theta": abs(d["theta_deg"] - od["theta_deg"]),
         "mass": max(abs(d["mass_A"] - od["mass_A"]) / od["mass_A"], abs(d["mass_B"] - od["mass_B"]) / od["mass_B"])}
    print(f"cfg1-{steps}-De{De:g}", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["C-I"] < 1e-5 and e["rho"] < 1e-5, e
    assert e["D"] < 1e-5 and e["theta"] < 1e-3 and e["mass"] < 1e-6, e


@pytest.mark.parametrize("case", ["polyA", "polyB", "visc_ratio", "ragged"])
def test_droplet_long_runs(lb, case):
    """Smaller droplets over 1500 steps: polymer in droplet / matrix, viscosity ratio
    (tau_A != tau_B), and a ragged odd-sized grid."""
    G = workloads.G_PHYSICS_1_004
    if case == "polyA":
        wl = workloads.droplet_shear(nx=48, ny=24, nz=40, R=7.0, G=G, polymer_phase="A", De=1.0,
                                     U=0.01)
    elif case == "polyB":
        wl = workloads.droplet_shear(nx=48, ny=24, nz=40, R=7.0, G=G, polymer_phase="B", L2=400.0,
                                     De=1.0, U=0.01)
    elif case == "visc_ratio":
        wl = workloads.droplet_shear(nx=48, ny=24, nz=40, R=7.0, G=G, tau_A=1.4, tau_B=0.9,
                                     polymer_phase="A", De=0.5, U=0.01)
    else:
        wl = workloads.droplet_shear(nx=37, ny=21, nz=29, R=6.0, G=G, polymer_phase="B", De=0.5,
                                     U=0.008)
    g, r, dg, do = run_both(lb, wl, 1500)
    e = report(f"long-{case}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5
    assert abs(dg["D"] - do["D"]) < 1e-5
    check_diag(dg, do, f"long-{case}", g, r, grid_shape(wl), wl["params"])


@pytest.mark.parametrize("scheme", ["default", "paper"])
@pytest.mark.parametrize("shape", [(1, 3, 1), (5, 3, 2), (65, 7, 3), (3, 9, 70)])
def test_degenerate_and_ragged_shapes(lb, shape, scheme):
    """Minimal wall gap (ny = 3), single-node periodic directions and tails that do
    not fill a 256-thread block, with the default schemes and with the paper's scheme
    throughout (MRT, stress in the equilibrium, Cholesky-log integrator)."""
    nx, ny, nz = shape
    rho, u, C = workloads.random_state(nx, ny, nz, 2, seed=nx * 100 + nz, amp_rho=0.05,
                                       amp_u=0.01, amp_C=0.1)
    rho[0] += 0.5
    wl = {"grid": {"nx": nx, "ny": ny, "nz": nz, "ncomp": 2},
          "params": {"tau_A": 0.9, "tau_B": 1.1, "G": 1.2, "delta": 0.1, "rho0": [1.5, 1.0],
                     "polymer_phase": "A", "eta_p": 0.1, "tau_p": 50.0, "L2": 60.0},
          "walls": {"u_bottom": [-0.01, 0, 0.005], "u_top": [0.01, 0, -0.002]},
          "rho": rho, "u": u, "C": C}
    if scheme == "paper":
        wl["params"].update(collision="mrt", fene="cholesky_ab2", kappa=0.01, coupling="stress")
    g, r, _, _ = run_both(lb, wl, 60)
    e = report(f"shape{shape}-{scheme}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5


def test_random_configurations_match_oracle(lb):
    """Seeded random configurations: extents (ragged, ny = 3, nz = 1), one or two
    components, polymer phase, relaxation times, wall velocities, the three options, and
    the launch path, tile and z-chunk (a path without an option steps on the split
    path), each against the oracle after 50 steps."""
    rng = np.random.default_rng(20261203)
    for k in range(12):
        nx = int(rng.integers(1, 80))
        ny = int(rng.integers(3, 24))
        nz = int(rng.integers(1, 40))
        nc = int(rng.integers(1, 3))
        rho, u, C = workloads.random_state(nx, ny, nz, nc, seed=1000 + k, amp_rho=0.05, amp_u=0.01, amp_C=0.1)
        if nc == 2:
            rho[0] += 0.5
        params = {"tau_A": float(rng.uniform(0.6, 1.5)), "tau_B": float(rng.uniform(0.6, 1.5)),
                  "G": float(rng.uniform(0.0, 1.5)) if nc == 2 else 0.0, "delta": 0.1,
                  "rho0": [1.5, 1.0] if nc == 2 else [1.0, 0.0],
                  "polymer_phase": str(rng.choice(["A", "B", "all", "none"])) if nc == 2 else "all",
                  "eta_p": float(rng.uniform(0.0, 0.1)), "tau_p": float(rng.uniform(20, 200)),
                  "L2": float(rng.choice([30.0, 100.0, 400.0])),
                  "collision": str(rng.choice(["bgk", "mrt"])), "fene": str(rng.choice(["upwind_euler", "cholesky_ab2"])),
                  "kappa": float(rng.choice([0.0, 0.01])), "coupling": str(rng.choice(["force", "stress"]))}
        walls = {"u_bottom": [float(rng.uniform(-0.02, 0.02)), 0.0, float(rng.uniform(-0.01, 0.01))],
                 "u_top": [float(rng.uniform(-0.02, 0.02)), 0.0, float(rng.uniform(-0.01, 0.01))]}
        wl = {"grid": {"nx": nx, "ny": ny, "nz": nz, "ncomp": nc}, "params": params, "walls": walls,
              "rho": rho, "u": u, "C": C}
        path = int(rng.choice([lb.PATH_FUSED, lb.PATH_SPLIT, lb.PATH_TWOPASS, lb.PATH_CHAINED]))
        tile = str(rng.choice(["32x8", "16x16", "64x8"])) if path == lb.PATH_TWOPASS else (
            "64x8" if path == lb.PATH_CHAINED else str(rng.choice(["32x8", "16x16"])))
        zc = int(rng.choice([0, 1, 3, 8]))
        tag = f"random{k} {nx}x{ny}x{nz} nc={nc} path={path} {tile} zc={zc} " + \
              " ".join(f"{key}={params[key]}" for key in ("collision", "fene", "coupling", "polymer_phase"))
        print(tag, flush=True)
        lat = lb.from_workload(wl)
        lat.set_tuning(path, tile, zc)
        lat.step(50)
        g = lat.get_fields()
        assert lat.flags() == 0, tag
        lat.close()
        o = oracle.from_workload(wl)
        assert o.step(50) == 0, tag
        e = report(tag, g, o.get_fields())
        assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5, tag


def test_zero_steps_returns_initial_fields(lb):
    wl = workloads.droplet_shear(nx=20, ny=10, nz=12, R=3.0, G=2.0, polymer_phase="A", U=0.01)
    g, r, _, _ = run_both(lb, wl, 0)
    e = report("zero-steps", g, r)
    assert e["u"] < 1e-6 and e["C"] < 1e-7 and e["rho"] < 1e-7


def test_two_components_at_zero_coupling_match_one_component(lb):
    nx, ny, nz = 24, 12, 10
    rho1, u, C = workloads.random_state(nx, ny, nz, 1, seed=3, amp_rho=0.02, amp_u=0.01, amp_C=0.05)
    share = np.random.default_rng(4).uniform(0.3, 0.7, rho1.shape[1])
    rho2 = np.stack([rho1[0] * share, rho1[0] * (1 - share)])
    base = {"tau_A": 0.8, "tau_B": 0.8, "G": 0.0, "delta": 0.1, "polymer_phase": "all",
            "eta_p": 0.05, "tau_p": 40.0, "L2": 30.0}
    walls = {"u_bottom": [-0.01, 0, 0], "u_top": [0.01, 0, 0]}
    w1 = {"grid": {"nx": nx, "ny": ny, "nz": nz, "ncomp": 1}, "params": dict(base, rho0=[1.0, 0]),
          "walls": walls, "rho": rho1, "u": u, "C": C}
    w2 = {"grid": {"nx": nx, "ny": ny, "nz": nz, "ncomp": 2},
          "params": dict(base, rho0=[0.5, 0.5]), "walls": walls, "rho": rho2, "u": u, "C": C}
    l1 = lb.from_workload(w1)
    l2 = lb.from_workload(w2)
    l1.step(200)
    l2.step(200)
    a = l1.get_fields()
    b = l2.get_fields()
    assert rel(b[0].sum(0), a[0][0]) < 1e-6
    assert rel(b[1], a[1]) < 1e-5 and rel(b[2], a[2]) < 1e-6


def test_mass_conservation_and_determinism(lb):
    """Per-component mass (FP64 reduction) drifts by less than 1e-6 relative over 2000
    steps; repeated runs and a checkpoint split N + N reproduce 2N bitwise."""
    wl = workloads.droplet_shear(nx=64, ny=32, nz=48, R=8.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="A", De=1.0, U=0.01)
    lat = lb.from_workload(wl)
    d0 = lat.diagnostics()
    lat.step(1000)
    blob = lat.get_state()
    lat.step(1000)
    d1 = lat.diagnostics()
    f_a = lat.get_fields()
    for k in ("mass_A", "mass_B"):
        assert abs(d1[k] - d0[k]) < 1e-6 * d0[k]
    lat2 = lb.from_workload(wl)
    lat2.step(2000)
    f_b = lat2.get_fields()
    lat3 = lb.from_workload(wl)
    lat3.set_state(blob)
    lat3.step(1000)
    f_c = lat3.get_fields()
    for x, y, z in zip(f_a, f_b, f_c):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    assert lat3.diagnostics()["step"] == 2000


def test_fault_flags_and_argument_errors(lb):
    wl = workloads.couette_fenep(nx=8, ny=8, nz=8)
    lat = lb.from_workload(wl)
    # host-side validation
    with pytest.raises(lb.LbfdError) as ei:
        lat.set_walls([0, 0.01, 0], [0, 0, 0])
    assert ei.value.status == lb.EINVAL
    bad = wl["C"].copy()
    bad[0, 5] = np.nan
    with pytest.raises(lb.LbfdError):
        lat.set_fields(wl["rho"], wl["u"], bad)
    bad = wl["C"].copy()
    bad[0, 5] = 200.0
    with pytest.raises(lb.LbfdError):
        lat.set_fields(wl["rho"], wl["u"], bad)
    with pytest.raises(lb.LbfdError):
        lat.set_params(dict(wl["params"], tau_A=0.5))
    # device-side detection, forced from the host with valid but extreme parameters:
    # a relaxation time far below one step overshoots C through zero (not SPD)
    C = wl["C"].copy()
    C[0] += 0.2
    lat.set_params(dict(wl["params"], tau_p=0.01))
    lat.set_fields(wl["rho"], wl["u"], C)
    st = lat.step_status(1)
    assert st == lb.ENOTSPD
    assert lat.diagnostics()["flags"] & lb.FLAG_NOT_SPD
    # extensibility: a trace close to L^2 = 3.5 pushed over it by stretching
    lat.set_params(dict(wl["params"], L2=3.5, tau_p=1e6))
    C = wl["C"].copy()
    C[3] = 0.3
    lat.set_walls([-0.5, 0, 0], [0.5, 0, 0])
    lat.set_fields(wl["rho"], wl["u"], C)
    st = lat.step_status(50)
    assert st in (lb.EEXTENSIBILITY, lb.ENOTSPD, lb.ENONFINITE)
    assert lat.flags() & (lb.FLAG_EXTENSIBILITY | lb.FLAG_NOT_SPD | lb.FLAG_NONFINITE)
    lat.close()
    # stepping before fields are set is a state error
    lat2 = lb.Lattice(8, 8, 8, 1, wl["params"])
    assert lat2.step_status(1) == lb.ESTATE


def test_fused_launch_shapes_agree_bitwise_and_match_split_path(lb):
    """Every tile shape and z-chunk of the fused single-pass step performs the same
    per-node arithmetic, so results are bitwise identical; the three-pass split path
    computes the same step in a different order (agreement to FP32 rounding)."""
    wl = workloads.droplet_shear(nx=45, ny=19, nz=23, R=6.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="B", De=0.5, U=0.01)
    ref = None
    for tile, zc in [("32x8", 0), ("32x16", 5), ("16x16", 3), ("32x8", 1), ("32x8", 23)]:
        lat = lb.from_workload(wl)
        lat.set_tuning(lb.PATH_FUSED, tile, zc)
        lat.step(40)
        f = lat.get_fields()
        lat.close()
        if ref is None:
            ref = f
        else:
            for a, b in zip(f, ref):
                assert np.array_equal(a, b), (tile, zc)
    lat = lb.from_workload(wl)
    lat.set_tuning(lb.PATH_SPLIT)
    lat.step(40)
    s = lat.get_fields()
    lat.close()
    e = report("fused-vs-split", ref, s)
    assert e["u"] < 2e-6 and e["C"] < 1e-7 and e["rho"] < 1e-7
    # two-pass step (moments pass + one pass over the tile): same arithmetic per node as the
    # fused pass except the order of the two species' momenta in j, bitwise identical
    # across its own launch shapes
    ref2 = None
    for tile, zc in [("32x8", 0), ("16x16", 3), ("64x8", 5), ("64x8", 0), ("32x8", 23)]:
        lat = lb.from_workload(wl)
        lat.set_tuning(lb.PATH_TWOPASS, tile, zc)
        lat.step(40)
        f = lat.get_fields()
        lat.close()
        if ref2 is None:
            ref2 = f
        else:
            for a, b in zip(f, ref2):
                assert np.array_equal(a, b), ("two-pass", tile, zc)
    e = report("fused-vs-two-pass", ref, ref2)
    assert e["u"] < 2e-6 and e["C"] < 1e-7 and e["rho"] < 1e-7


@pytest.mark.parametrize("case", ["cfg1_physics", "couette", "ragged_polyB"])
def test_two_pass_step_matches_oracle(lb, case):
    """The two-pass launch shape against the FP64 oracle on the full 128x64x128 droplet,
    the FENE-P Couette and a ragged droplet grid."""
    if case == "cfg1_physics":
        wl, steps = workloads.droplet_cfg1(De=1.0, variant="physics"), 100
    elif case == "couette":
        wl, steps = workloads.couette_fenep(), 4000
    else:
        wl = workloads.droplet_shear(nx=37, ny=21, nz=29, R=6.0, G=workloads.G_PHYSICS_1_004,
                                     polymer_phase="B", De=0.5, U=0.008)
        steps = 1500
    lat = lb.from_workload(wl)
    lat.set_tuning(lb.PATH_TWOPASS)
    lat.step(steps)
    g = lat.get_fields()
    dg = lat.diagnostics()
    lat.close()
    o = oracle.from_workload(wl)
    assert o.step(steps) == 0
    r = o.get_fields()
    do = o.diagnostics()
    e = report(f"two-pass-{case}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5
    assert abs(dg["D"] - do["D"]) < 1e-5


def test_chained_launch_shapes_agree_bitwise_and_match_two_pass(lb):
    """The chained step (the second pass also forms the next level's moments) sums the
    same values in the same order for every z-chunk, including one plane per workgroup,
    where every plane is also collided as a neighbour of two chunks: results are bitwise
    identical across z-chunks.  Against the two-pass step (moments from a separate pass,
    summed in another order) they agree to FP32 rounding."""
    wl = workloads.droplet_shear(nx=45, ny=19, nz=23, R=6.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="B", De=0.5, U=0.01)
    ref = None
    for zc in (0, 1, 3, 7, 23):
        lat = lb.from_workload(wl)
        lat.set_tuning(lb.PATH_CHAINED, "64x8", zc)
        lat.step(40)
        f = lat.get_fields()
        lat.close()
        if ref is None:
            ref = f
        else:
            for a, b in zip(f, ref):
                assert np.array_equal(a, b), ("chained", zc)
    lat = lb.from_workload(wl)
    lat.set_tuning(lb.PATH_TWOPASS, "64x8", 0)
    lat.step(40)
    t = lat.get_fields()
    lat.close()
    e = report("chained-vs-two-pass", ref, t)
    # the moments of every step are FP32 sums in another order: |du| ~ 1e-7 against
    # |u| ~ 1e-2, a relative L2 of a few 1e-6 after 40 steps
    assert e["u"] < 5e-6 and e["C"] < 1e-7 and e["rho"] < 1e-7


@pytest.mark.parametrize("case", ["cfg1_physics", "couette", "ragged_polyB", "wide_ragged_polyA"])
def test_chained_step_matches_oracle(lb, case):
    """The chained step against the FP64 oracle: the full 128x64x128 droplet, the
    one-component FENE-P Couette, and ragged grids (several 64-wide tiles with a partial
    one, ny not a multiple of 8, several z-chunks)."""
    if case == "cfg1_physics":
        wl, steps = workloads.droplet_cfg1(De=1.0, variant="physics"), 100
    elif case == "couette":
        wl, steps = workloads.couette_fenep(), 4000
    elif case == "ragged_polyB":
        wl = workloads.droplet_shear(nx=37, ny=21, nz=29, R=6.0, G=workloads.G_PHYSICS_1_004,
                                     polymer_phase="B", De=0.5, U=0.008)
        steps = 1500
    else:
        wl = workloads.droplet_shear(nx=150, ny=27, nz=20, R=8.0, G=workloads.G_PHYSICS_1_004,
                                     polymer_phase="A", De=1.0, U=0.01)
        steps = 300
    lat = lb.from_workload(wl)
    lat.set_tuning(lb.PATH_CHAINED, "64x8", 6 if case == "wide_ragged_polyA" else 0)
    lat.step(steps)
    g = lat.get_fields()
    dg = lat.diagnostics()
    lat.close()
    o = oracle.from_workload(wl)
    assert o.step(steps) == 0
    r = o.get_fields()
    do = o.diagnostics()
    e = report(f"chained-{case}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5
    assert abs(dg["D"] - do["D"]) < 1e-5
    check_diag(dg, do, f"chained-{case}", g, r, grid_shape(wl), wl["params"])


def test_chained_step_restarts_and_diagnostics_bitwise(lb):
    """The chained step carries the moments from step to step.  Diagnostics and field
    reads use them without recomputing them, and a checkpoint holds them, so a run with
    diagnostics, a run without, and a run restarted from a checkpoint agree bitwise."""
    wl = workloads.droplet_shear(nx=64, ny=32, nz=48, R=8.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="A", De=1.0, U=0.01)

    def chained():
        lat = lb.from_workload(wl)
        lat.set_tuning(lb.PATH_CHAINED, "64x8", 0)
        return lat

    a = chained()
    d0 = a.diagnostics()
    for _ in range(5):
        a.step(100)
        a.diagnostics()
    blob = a.get_state()
    a.step(500)
    fa = a.get_fields()
    b = chained()
    b.step(1000)
    fb = b.get_fields()
    c = chained()
    c.set_state(blob)
    c.step(500)
    fc = c.get_fields()
    d1 = c.diagnostics()
    for x, y, z in zip(fa, fb, fc):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    assert d1["step"] == 1000
    for k in ("mass_A", "mass_B"):
        assert abs(d1[k] - d0[k]) < 1e-6 * d0[k]
    for lat in (a, b, c):
        lat.close()


@pytest.mark.parametrize("Lam,coupling", [(0.625, "force"), (2.5, "force"), (2.5, "stress")])
def test_gpu_steady_shear_matches_lindner_closed_form(lb, Lam, coupling):
    """The GPU step against the paper directly, not only against the oracle: plane Couette
    with feedback on, run for 20 polymer times, gives the closed-form steady-shear
    conformation C = sigma_P / Z of Sec. 3.1 (eqs. lindner, lindner2) at L^2 = 100, with
    C_yy = C_zz (no second normal-stress difference) and the linear velocity profile (a
    uniform stress moves no fluid), in both couplings."""
    from paper_closed_forms import lindner_N, lindner_S, steady_shear_conformation

    ny, tau_p, L2 = 16, 1000.0 if Lam < 1 else 200.0, 100.0
    U = Lam / tau_p * ny / 2.0
    wl = workloads.couette_fenep(nx=2, ny=ny, nz=2, U=U, tau_p=tau_p, L2=L2, noise=0.0, coupling=coupling)
    wl["params"]["eta_p"] = 1.0 / 24.0
    lat = lb.from_workload(wl)
    lat.step(int(20 * tau_p))
    _, u, C = lat.get_fields()
    assert lat.flags() == 0
    lat.close()
    ref = steady_shear_conformation(Lam, L2)
    keys = ("xx", "yy", "zz", "xy", "xz", "yz")
    for k, key in enumerate(keys):
        assert np.allclose(C[k], ref[key], rtol=5e-5, atol=5e-6), (key, C[k][:4], ref[key])
    assert np.max(np.abs(C[1] - C[2])) < 1e-6 and np.max(np.abs(C[4:])) < 1e-6
    tr = C[0] + C[1] + C[2]
    f = (L2 - 3) / (L2 - tr)
    assert np.allclose(f * C[3], lindner_S(Lam, L2), rtol=5e-5)
    assert np.allclose(f * C[0] - 1, lindner_N(Lam, L2), rtol=2e-4)
    Y = np.repeat(np.arange(ny), 2)[None, :].repeat(2, 0).ravel()
    assert np.allclose(u[0], -U + 2 * U * (Y + 0.5) / ny, atol=1e-4 * U)


@pytest.mark.parametrize("path", ["chained", "split"])
@pytest.mark.parametrize("case", ["droplet_visc_ratio", "couette_tau13", "droplet_stress_coupling"])
def test_mrt_collision_matches_oracle(lb, case, path):
    """The multiple-relaxation-time collision (Sec. 2; bulk and shear modes at the local
    tau, species momenta at tau_M = 1, other modes at 1) in the chained one-launch step (its
    default) and on the per-node split path against the oracle's MRT: a droplet with
    viscosity ratio 0.4 (tau_A = 0.62, tau_B = 1.1, so tau varies across the interface), the
    FENE-P Couette at tau = 1.3, and the stress coupling."""
    if case == "droplet_visc_ratio":
        wl = workloads.droplet_shear(nx=40, ny=24, nz=28, R=6.0, G=workloads.G_PHYSICS_1_004,
                                     polymer_phase="B", De=0.5, U=0.01, tau_A=0.62, tau_B=1.1)
        steps = 400
    elif case == "couette_tau13":
        wl, steps = workloads.couette_fenep(nx=8, ny=32, nz=8, tau=1.3), 2000
    else:
        wl = workloads.droplet_shear(nx=37, ny=21, nz=29, R=6.0, G=workloads.G_PHYSICS_1_004,
                                     polymer_phase="A", De=1.0, U=0.01, tau_A=0.8, coupling="stress")
        steps = 400
    wl["params"]["collision"] = "mrt"
    lat = lb.from_workload(wl)
    if path == "split":
        lat.set_tuning(lb.PATH_SPLIT)
    assert lat.get_tuning()["path"] == (lb.PATH_SPLIT if path == "split" else lb.PATH_CHAINED)
    lat.step(steps)
    g = lat.get_fields()
    dg = lat.diagnostics()
    lat.close()
    o = oracle.from_workload(wl)
    assert o.step(steps) == 0
    r = o.get_fields()
    do = o.diagnostics()
    e = report(f"mrt-{case}-{path}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5
    for k in ("mass_A", "mass_B"):
        assert abs(dg[k] - do[k]) <= 1e-6 * abs(do[k]) + 1e-9
    if case != "couette_tau13":  # (a steady linear profile is the same under both)
        # the two collisions differ here (tau != 1 at the droplet): MRT is not silently BGK
        wl["params"]["collision"] = "bgk"
        ob = oracle.from_workload(wl)
        assert ob.step(steps) == 0
        assert rel(ob.get_fields()[1], r[1]) > 100 * max(e["u"], 1e-7)


@pytest.mark.parametrize("fene", ["upwind_euler", "cholesky_ab2"])
def test_chained_options_agree_bitwise_across_zchunks_and_match_split(lb, fene):
    """MRT in the chained step collides halo nodes (tile-edge lanes, neighbouring rows,
    corners, the planes next to a z-chunk) from all 19 of their populations with the
    function the node's own tile uses, so results are bitwise identical across z-chunks
    (one plane per workgroup included).  Against the split path, which sums the
    projection per direction and the moments in another order, they agree to FP32
    rounding."""
    wl = workloads.droplet_shear(nx=45, ny=19, nz=23, R=6.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="B", De=0.5, U=0.01, tau_A=0.7, tau_B=1.15)
    wl["params"]["collision"] = "mrt"
    wl["params"]["fene"] = fene
    ref = None
    for zc in (0, 1, 3, 7, 23):
        lat = lb.from_workload(wl)
        lat.set_tuning(lb.PATH_CHAINED, "64x8", zc)
        lat.step(40)
        f = lat.get_fields()
        assert lat.flags() == 0
        lat.close()
        if ref is None:
            ref = f
        else:
            for a, b in zip(f, ref):
                assert np.array_equal(a, b), ("chained mrt", fene, zc)
    lat = lb.from_workload(wl)
    lat.set_tuning(lb.PATH_SPLIT)
    lat.step(40)
    t = lat.get_fields()
    lat.close()
    e = report(f"chained-mrt-vs-split-{fene}", ref, t)
    assert e["u"] < 5e-6 and e["C"] < 1e-6 and e["rho"] < 1e-7


def test_mrt_at_unit_tau_agrees_with_bgk_and_batches_check_options(lb):
    """At tau = 1 every MRT rate is 1 and the step is the BGK step (FP32 rounding apart).
    A batch refuses instances whose options differ, and options on the fused batch body,
    which has none of them."""
    wl = workloads.droplet_shear(nx=40, ny=20, nz=24, R=6.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="A", De=0.5, U=0.01)
    out = []
    for coll in ("mrt", "bgk"):
        w = dict(wl, params=dict(wl["params"], collision=coll))
        lat = lb.from_workload(w)
        lat.set_tuning(lb.PATH_SPLIT)
        lat.step(100)
        out.append(lat.get_fields())
        lat.close()
    e = report("mrt-vs-bgk-tau1", out[0], out[1])
    assert e["u"] < 2e-6 and e["rho"] < 1e-7 and e["C"] < 1e-7
    w = dict(wl, params=dict(wl["params"], collision="mrt"))
    b = lb.Batch([w, wl])
    with pytest.raises(lb.LbfdError) as ei:
        b.step(2)
    assert ei.value.status == lb.EINVAL
    b.close()
    b = lb.Batch([w, w])
    b.set_tuning("32x8", 0, path=lb.PATH_FUSED)
    with pytest.raises(lb.LbfdError) as ei:
        b.step(2)
    assert ei.value.status == lb.EINVAL
    b.close()


@pytest.mark.parametrize("path", ["chained", "split"])
@pytest.mark.parametrize("case", ["couette", "droplet_kappa", "ragged_polyB"])
def test_cholesky_ab2_fene_matches_oracle(lb, case, path):
    """The paper's FENE-P integrator (Cholesky factor of f C with ln l_ii, central
    differences, artificial diffusivity, Adams-Bashforth 2) against the oracle, in the
    chained one-launch step (its default) and on the per-node split path: the FENE-P
    Couette, a droplet with kappa = 0.02, and a ragged droplet grid."""
    if case == "couette":
        wl, steps = workloads.couette_fenep(), 4000
    elif case == "droplet_kappa":
        wl = workloads.droplet_shear(nx=40, ny=24, nz=28, R=6.0, G=workloads.G_PHYSICS_1_004,
                                     polymer_phase="A", De=1.0, U=0.01)
        wl["params"]["kappa"] = 0.02
        steps = 600
    else:
        wl = workloads.droplet_shear(nx=37, ny=21, nz=29, R=6.0, G=workloads.G_PHYSICS_1_004,
                                     polymer_phase="B", De=0.5, U=0.008)
        steps = 800
    wl["params"]["fene"] = "cholesky_ab2"
    lat = lb.from_workload(wl)
    if path == "split":
        lat.set_tuning(lb.PATH_SPLIT)
    assert lat.get_tuning()["path"] == (lb.PATH_SPLIT if path == "split" else lb.PATH_CHAINED)
    lat.step(steps)
    g = lat.get_fields()
    assert lat.flags() == 0
    lat.close()
    o = oracle.from_workload(wl)
    assert o.step(steps) == 0
    r = o.get_fields()
    e = report(f"cholesky-{case}-{path}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5


@pytest.mark.parametrize("path", ["chained", "split"])
def test_mrt_with_cholesky_ab2_matches_oracle(lb, path):
    """Both of the paper's options at once (MRT collision and the Cholesky-log integrator)
    against the oracle with both, in the chained step and on the split path."""
    wl = workloads.droplet_shear(nx=36, ny=20, nz=26, R=5.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="A", De=1.0, U=0.01, tau_A=0.7, tau_B=1.2)
    wl["params"]["collision"] = "mrt"
    wl["params"]["fene"] = "cholesky_ab2"
    wl["params"]["kappa"] = 0.01
    lat = lb.from_workload(wl)
    if path == "split":
        lat.set_tuning(lb.PATH_SPLIT)
    assert lat.get_tuning()["path"] == (lb.PATH_SPLIT if path == "split" else lb.PATH_CHAINED)
    lat.step(400)
    g = lat.get_fields()
    assert lat.flags() == 0
    lat.close()
    o = oracle.from_workload(wl)
    assert o.step(400) == 0
    e = report(f"mrt+cholesky-{path}", g, o.get_fields())
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5


def test_papers_full_scheme_matches_oracle(lb):
    """The paper's own scheme throughout, in the chained one-launch step: MRT collision,
    polymer stress through the equilibrium's second moment, and the Cholesky-log
    Adams-Bashforth-2 integrator with artificial diffusivity, against the oracle with the
    same three options on a ragged droplet grid."""
    wl = workloads.droplet_shear(nx=37, ny=21, nz=29, R=6.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="A", De=1.0, U=0.01, tau_A=0.8, coupling="stress")
    wl["params"].update(collision="mrt", fene="cholesky_ab2", kappa=0.01)
    lat = lb.from_workload(wl)
    assert lat.get_tuning()["path"] == lb.PATH_CHAINED
    lat.step(500)
    g = lat.get_fields()
    dg = lat.diagnostics()
    assert lat.flags() == 0
    lat.close()
    o = oracle.from_workload(wl)
    assert o.step(500) == 0
    e = report("paper-scheme", g, o.get_fields())
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5
    assert abs(dg["D"] - o.diagnostics()["D"]) < 1e-5


def test_options_take_the_paths_that_implement_them(lb):
    """A tuned path that lacks an option falls back to the split path (the MRT collision and
    the Cholesky integrator are in the chained tile body only).  The autotuner times only
    paths that implement the options and leaves the state, the rate history included,
    unchanged: a run that autotunes midway equals one that does not, bitwise."""
    wl = workloads.droplet_shear(nx=40, ny=20, nz=24, R=6.0, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase="A", De=1.0, U=0.01)
    wc = dict(wl, params=dict(wl["params"], fene="cholesky_ab2"))
    wm = dict(wl, params=dict(wl["params"], collision="mrt"))
    for w in (wc, wm):
        lat = lb.from_workload(w)
        for path, want in ((lb.PATH_FUSED, lb.PATH_SPLIT), (lb.PATH_TWOPASS, lb.PATH_SPLIT),
                           (lb.PATH_CHAINED, lb.PATH_CHAINED), (lb.PATH_SPLIT, lb.PATH_SPLIT)):
            lat.set_tuning(path, "64x8" if path == lb.PATH_CHAINED else "32x8", 0)
            assert lat.get_tuning()["path"] == want
        lat.close()
    for w, want in ((wc, lb.PATH_CHAINED), (wm, lb.PATH_CHAINED)):
        a = lb.from_workload(w)
        a.step(7)
        before = a.get_fields()
        t = a.autotune(reps=1)
        assert t["path"] == want and a.get_tuning()["path"] == want
        for x, y in zip(a.get_fields(), before):
            assert np.array_equal(x, y)
        a.step(9)
        b = lb.from_workload(w)
        if want == lb.PATH_CHAINED:
            b.step(16)
        else:
            b.step(7)
            b.set_tuning(lb.PATH_SPLIT)
            b.step(9)
        for x, y in zip(a.get_fields(), b.get_fields()):
            assert np.array_equal(x, y)
        assert a.flags() == 0
        a.close()
        b.close()


def test_cholesky_ab2_steady_shear_and_restart(lb):
    """GPU Cholesky scheme against the paper directly (steady shear at Lambda = 2.5,
    L^2 = 100, eqs. lindner, lindner2), and a checkpoint split N + N that reproduces 2N
    bitwise (the checkpoint carries the Adams-Bashforth history)."""
    from paper_closed_forms import steady_shear_conformation

    ny, tau_p, L2, Lam = 16, 200.0, 100.0, 2.5
    U = Lam / tau_p * ny / 2.0
    wl = workloads.couette_fenep(nx=2, ny=ny, nz=2, U=U, tau_p=tau_p, L2=L2, noise=0.0)
    wl["params"]["eta_p"] = 1.0 / 24.0
    wl["params"]["fene"] = "cholesky_ab2"
    lat = lb.from_workload(wl)
    lat.step(int(20 * tau_p))
    C = lat.get_fields()[2]
    lat.close()
    ref = steady_shear_conformation(Lam, L2)
    for k, key in enumerate(("xx", "yy", "zz", "xy")):
        assert np.allclose(C[k], ref[key], rtol=5e-5, atol=5e-6), key
    wl2 = workloads.droplet_shear(nx=40, ny=20, nz=24, R=6.0, G=workloads.G_PHYSICS_1_004,
                                  polymer_phase="A", De=1.0, U=0.01)
    wl2["params"]["fene"] = "cholesky_ab2"
    a = lb.from_workload(wl2)
    a.step(150)
    blob = a.get_state()
    a.step(150)
    b = lb.from_workload(wl2)
    b.step(300)
    c = lb.from_workload(wl2)
    c.set_state(blob)
    c.step(150)
    for x, y, z in zip(a.get_fields(), b.get_fields(), c.get_fields()):
        assert np.array_equal(x, y) and np.array_equal(x, z)
    for lat in (a, b, c):
        lat.close()


@pytest.mark.parametrize("collision,fene,coupling", [
    ("bgk", "upwind_euler", "force"), ("mrt", "upwind_euler", "force"), ("bgk", "cholesky_ab2", "force"),
    ("mrt", "cholesky_ab2", "force"), ("mrt", "cholesky_ab2", "stress")])
def test_full_size_droplet_sampled_window(lb, collision, fene, coupling):
    """The 1024x256x1024 droplet (268M nodes) in the launch configuration the benchmark
    times (the chained step, with the default schemes, with the paper's MRT collision and
    Cholesky-log integrator, and with the paper's whole scheme including the stress in the
    equilibrium), checked against the oracle on a sampled window.  One step moves information at
    most two nodes (the Shan-Chen and stress-divergence stencils of the half-force
    velocity), so after k steps the centre of a window whose margin exceeds 2k is exact on
    a window-sized periodic oracle run.  The window straddles the droplet interface and
    spans both walls; the sample is its central 48 x 256 x 48 block.  Whole-grid
    properties (mass per species, fault flags) are checked on the full lattice."""
    import torch

    nx, ny, nz = 1024, 256, 1024
    steps, bx, bz, m = 10, 96, 96, 24
    assert m > 2 * steps
    free, _ = torch.cuda.mem_get_info()
    need = lb.state_bytes(nx, ny, nz, 2)
    if free < need + (4 << 30):
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory")
    wl0 = workloads.droplet_cfg2(nx=nx, ny=ny, nz=nz, box=(0, nx, 0, 1))
    wl0["params"].update(collision=collision, fene=fene, coupling=coupling)
    lat = lb.Lattice(nx, ny, nz, 2, wl0["params"])
    lat.set_walls(wl0["walls"]["u_bottom"], wl0["walls"]["u_top"])
    assert lat.get_tuning()["path"] == lb.PATH_CHAINED
    for z0 in range(0, nz, 16):
        w = workloads.droplet_cfg2(nx=nx, ny=ny, nz=nz, box=(0, nx, z0, 16))
        lat.set_fields_box(0, 0, z0, nx, ny, 16, w["rho"], w["u"], w["C"])
    lat.reset_counters()
    d0 = lat.diagnostics()
    lat.step(steps)
    d1 = lat.diagnostics()
    assert d1["flags"] == 0
    for k in ("mass_A", "mass_B"):
        assert abs(d1[k] - d0[k]) < 1e-6 * d0[k]
    # window centred in z on the droplet, in x on its left interface (x = 511.5 - 64)
    x0, z0 = 448 - bx // 2, 512 - bz // 2
    g = lat.get_fields_box(x0, 0, z0, bx, ny, bz)
    lat.close()
    del lat
    torch.cuda.empty_cache()
    wl = workloads.droplet_cfg2(nx=nx, ny=ny, nz=nz, box=(x0, bx, z0, bz))
    wl["params"].update(collision=collision, fene=fene, coupling=coupling)
    o = oracle.from_workload(wl)
    assert o.step(steps) == 0
    r = o.get_fields()
    sel = np.zeros((bz, ny, bx), dtype=bool)
    sel[m:bz - m, :, m:bx - m] = True
    sel = sel.ravel()
    gs = tuple(a[:, sel] for a in g)
    rs = tuple(a[:, sel] for a in r)
    e = report(f"full-size window {collision}/{fene}/{coupling}", gs, rs)
    # the sample contains the interface: both phases are present
    assert rs[0][0].max() > 0.5 and rs[0][0].min() < 0.1
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5


@pytest.mark.parametrize("case", ["couette", "droplet_polyA", "droplet_polyB_visc"])
def test_stress_coupling_matches_oracle(lb, case):
    """Polymer stress fed through the equilibrium's second moment (Sec. 2, eq.
    MODEtransformation) instead of a body force: the fused step against the oracle, and
    the three-pass split path against the fused one."""
    G = workloads.G_PHYSICS_1_004
    if case == "couette":
        wl = workloads.couette_fenep(coupling="stress")
        steps = 4000
    elif case == "droplet_polyA":
        wl = workloads.droplet_shear(nx=48, ny=24, nz=40, R=7.0, G=G, polymer_phase="A", De=1.0,
                                     U=0.01, coupling="stress")
        steps = 1500
    else:
        wl = workloads.droplet_shear(nx=37, ny=21, nz=29, R=6.0, G=G, tau_A=1.4, tau_B=0.9,
                                     polymer_phase="B", De=0.5, U=0.008, coupling="stress")
        steps = 1500
    g, r, dg, do = run_both(lb, wl, steps)
    e = report(f"stress-{case}", g, r)
    assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5
    assert abs(dg["D"] - do["D"]) < 1e-5
    if case != "couette":
        # at an interface the two couplings differ (the modulated stress is not uniform):
        # the body-force run departs from the stress-coupled oracle beyond the parity error
        wl_f = dict(wl, params=dict(wl["params"], coupling="force"))
        lat = lb.from_workload(wl_f)
        lat.step(steps)
        gf = lat.get_fields()
        lat.close()
        d = max(rel(gf[1], r[1]), rel(gf[2] - I6, r[2] - I6))
        print(f"stress-{case}: force-coupled run differs by {d:.2e}")
        assert d > 10 * max(e["u"], e["C-I"])
    lat = lb.from_workload(wl)
    lat.set_tuning(lb.PATH_SPLIT)
    lat.step(steps)
    s = lat.get_fields()
    lat.close()
    es = report(f"stress-{case}-split", s, r)
    assert es["u"] < 1e-5 and es["C"] < 1e-5 and es["rho"] < 1e-5
