"""GPU tests of batched execution: uneven instances stepped by one launch per step (with
the captured step graph replayed) reproduce single-lattice runs bitwise; retired
instances stay frozen; the run-to-steady controller and both autotuners leave results
unchanged."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1406_2686_amd

    return paper_1406_2686_amd


def small_cases():
    G = workloads.G_PHYSICS_1_004
    return [
        workloads.droplet_shear(nx=40, ny=16, nz=24, R=5.0, G=G, polymer_phase="A", De=0.5, U=0.01),
        workloads.droplet_shear(nx=64, ny=32, nz=48, R=8.0, G=G, polymer_phase="B", De=1.0, U=0.02,
                                tau_A=1.3),
        workloads.droplet_shear(nx=37, ny=21, nz=13, R=4.0, G=G, polymer_phase="A", L2=400.0, U=0.005),
        workloads.droplet_shear(nx=96, ny=24, nz=32, R=6.0, G=G, polymer_phase="B", De=0.3, U=0.015,
                                tau_A=0.8),
        workloads.droplet_shear(nx=16, ny=8, nz=16, R=3.0, G=2.5, polymer_phase="A", U=0.01),
    ]


def singles(lb, cases, steps, path=None):
    """Single-lattice references on the tile body the batch launch runs: the fused
    single-pass step by default (the default chained step agrees with it to FP32 rounding
    only), or the chained step for a chained batch."""
    out = []
    for wl in cases:
        lat = lb.from_workload(wl)
        if path is None or path == lb.PATH_FUSED:
            lat.set_tuning(lb.PATH_FUSED)
        else:
            lat.set_tuning(path, "64x8", 0)
        lat.step(steps)
        out.append(lat.get_fields())
        lat.close()
    return out


def test_batch_matches_single_lattices_bitwise_over_graph_replays(lb):
    """Each call replays the two-step graph; odd counts add eager steps; diagnostics and
    field reads run between the replays.  Every checkpoint is compared bitwise."""
    cases = small_cases()
    b = lb.Batch(cases)
    b.set_tuning("32x8", 0, path=lb.PATH_FUSED)
    total = 0
    for n in (10, 7, 24, 1):
        b.step(n)
        total += n
        b.diagnostics()
        ref = singles(lb, cases, total)
        for i in range(len(cases)):
            got = b.get_fields(i)
            for a, r in zip(got, ref[i]):
                assert np.array_equal(a, r), (i, total)
    b.close()


@pytest.mark.parametrize("tile", ["64x8", "32x16"])
def test_chained_batch_matches_chained_single_lattices_bitwise(lb, tile):
    """The chained body over the batch work table (64x8 or 32x16 tiles, each instance's
    moments carried from step to step in its own buffers) against single lattices on the
    chained step (64x8 tiles): bitwise over graph replays, odd step counts, diagnostics in
    between, a retired instance (its moments wait with it) and its return.  The cases
    include lattices narrower than a tile in x (16) and in y (8), and ragged ones."""
    cases = small_cases()
    b = lb.Batch(cases)
    assert b.get_tuning()["path"] == lb.PATH_CHAINED  # the default
    b.set_tuning(tile, 0, path=lb.PATH_CHAINED)
    total = 0
    for n in (10, 7, 1):
        b.step(n)
        total += n
        b.diagnostics()
        ref = singles(lb, cases, total, lb.PATH_CHAINED)
        for i in range(len(cases)):
            for a, r in zip(b.get_fields(i), ref[i]):
                assert np.array_equal(a, r), (i, total)
    b.set_active([True, False, True, True, True])
    b.step(5)
    b.set_active([True] * 5)
    b.step(3)
    ref = singles(lb, cases, total + 8, lb.PATH_CHAINED)
    ref1 = singles(lb, [cases[1]], total + 3, lb.PATH_CHAINED)[0]
    for i in range(len(cases)):
        for a, r in zip(b.get_fields(i), ref1 if i == 1 else ref[i]):
            assert np.array_equal(a, r), (i, "after retire")
    b.close()


@pytest.mark.parametrize("tile", ["64x8", "32x16"])
def test_single_component_chained_batch_matches_single_lattices_bitwise(lb, tile):
    """One-component lattices (FENE-P Couette with noise on C, one of them ragged and one
    narrower than a tile) in the chained batch body against single chained lattices,
    bitwise: the one-component body runs eight wavefronts, two of which collide the
    neighbouring rows."""
    cases = [workloads.couette_fenep(nx=16, ny=32, nz=16, seed=1),
             workloads.couette_fenep(nx=40, ny=21, nz=9, seed=2, U=0.02),
             workloads.couette_fenep(nx=96, ny=12, nz=20, seed=3, tau=0.8)]
    b = lb.Batch(cases)
    b.set_tuning(tile, 0, path=lb.PATH_CHAINED)
    b.step(25)
    ref = singles(lb, cases, 25, lb.PATH_CHAINED)
    for i in range(len(cases)):
        for a, r in zip(b.get_fields(i), ref[i]):
            assert np.array_equal(a, r), (tile, i)
    b.close()


def test_default_chained_tile_follows_the_instance_widths(lb):
    """A new batch runs the chained body on 32x16 tiles when its lattices would leave 64x8
    tiles emptier by a tenth of the lanes or more (32 and 96 nodes wide), else on 64x8."""
    G = workloads.G_PHYSICS_1_004
    narrow = [workloads.droplet_shear(nx=32, ny=16, nz=16, R=4.0, G=G, U=0.01),
              workloads.droplet_shear(nx=96, ny=16, nz=16, R=4.0, G=G, U=0.01)]
    wide = [workloads.droplet_shear(nx=64, ny=16, nz=16, R=4.0, G=G, U=0.01),
            workloads.droplet_shear(nx=128, ny=8, nz=16, R=3.0, G=G, U=0.01)]
    for cases, tile in ((narrow, "32x16"), (wide, "64x8")):
        b = lb.Batch(cases)
        t = b.get_tuning()
        assert t["path"] == lb.PATH_CHAINED and t["tile"] == tile, (t, tile)
        b.close()


@pytest.mark.parametrize("collision,fene,tile", [("mrt", "upwind_euler", "64x8"), ("bgk", "cholesky_ab2", "64x8"),
                                                ("mrt", "cholesky_ab2", "64x8"), ("mrt", "cholesky_ab2", "32x16")])
def test_batches_with_the_papers_schemes_match_single_lattices_bitwise(lb, collision, fene, tile):
    """The paper's MRT collision and Cholesky-log integrator in the chained batch body
    (every instance with the same options) against single chained lattices, bitwise: the
    first step after the fields are set is forward Euler in both (the batch takes it
    eagerly, before the graph replays), odd step counts and diagnostics between the
    calls, and a retired instance whose rate history waits with it."""
    cases = [dict(w, params=dict(w["params"], collision=collision, fene=fene, kappa=0.01))
             for w in small_cases()]
    b = lb.Batch(cases)
    b.set_tuning(tile, 0, path=lb.PATH_CHAINED)
    total = 0
    for n in (10, 7, 1):
        b.step(n)
        total += n
        b.diagnostics()
        ref = singles(lb, cases, total, lb.PATH_CHAINED)
        for i in range(len(cases)):
            for a, r in zip(b.get_fields(i), ref[i]):
                assert np.array_equal(a, r), (collision, fene, i, total)
    b.set_active([True, False, True, True, True])
    b.step(5)
    b.set_active([True] * 5)
    b.step(3)
    ref = singles(lb, cases, total + 8, lb.PATH_CHAINED)
    ref1 = singles(lb, [cases[1]], total + 3, lb.PATH_CHAINED)[0]
    for i in range(len(cases)):
        for a, r in zip(b.get_fields(i), ref1 if i == 1 else ref[i]):
            assert np.array_equal(a, r), (collision, fene, i, "after retire")
    res = b.autotune(reps=1)
    assert res["path"] == lb.PATH_CHAINED   # the only body with the options
    b.close()


def test_retired_instances_stay_frozen(lb):
    cases = small_cases()[:3]
    b = lb.Batch(cases)
    b.set_tuning("32x8", 0, path=lb.PATH_FUSED)
    b.step(6)
    frozen = b.get_fields(1)
    b.set_active([True, False, True])
    b.step(9)
    for a, r in zip(b.get_fields(1), frozen):
        assert np.array_equal(a, r)
    ref = singles(lb, cases, 15)
    for i in (0, 2):
        for a, r in zip(b.get_fields(i), ref[i]):
            assert np.array_equal(a, r)
    d = b.diagnostics()
    assert d[1]["step"] == 6 and d[0]["step"] == 15
    b.set_active([True, True, True])
    b.step(9)
    ref1 = singles(lb, [cases[1]], 15)[0]
    for a, r in zip(b.get_fields(1), ref1):
        assert np.array_equal(a, r)
    b.close()


def test_autotuners_pick_a_shape_and_leave_the_state_unchanged(lb):
    cases = small_cases()[:2]
    b = lb.Batch(cases)
    b.set_tuning("32x8", 0, path=lb.PATH_FUSED)
    b.step(4)
    before = [b.get_fields(i) for i in range(2)]
    res = b.autotune(reps=2)
    assert res["tile"] in ("32x8", "16x16", "64x8", "32x16") and res["zchunk"] >= 4 and res["ms_per_step"] > 0
    assert (res["path"] == lb.PATH_CHAINED) == (res["tile"] in ("64x8", "32x16"))
    for i in range(2):
        for a, r in zip(b.get_fields(i), before[i]):
            assert np.array_equal(a, r)
    b.step(6)  # on the shape the autotuner chose
    for i in range(2):
        lat = lb.from_workload(cases[i])
        lat.set_tuning(lb.PATH_FUSED)
        lat.step(4)
        if res["path"] == lb.PATH_CHAINED:
            lat.set_tuning(lb.PATH_CHAINED, "64x8", 0)
        lat.step(6)
        for a, r in zip(b.get_fields(i), lat.get_fields()):
            assert np.array_equal(a, r)
        lat.close()
    b.close()
    lat = lb.from_workload(cases[1])
    lat.step(3)
    s0 = lat.get_fields()
    t = lat.autotune(reps=2)
    assert t["ms_per_step"] > 0 and t["tile"] in ("32x8", "16x16", "64x8")
    assert t["path"] in (lb.PATH_FUSED, lb.PATH_TWOPASS, lb.PATH_CHAINED)
    for a, r in zip(lat.get_fields(), s0):
        assert np.array_equal(a, r)
    assert lat.diagnostics()["step"] == 3


def test_run_to_steady_retires_converged_instances(lb):
    """A uniform mixture (phi = 0 everywhere, so no droplet and D = 0) is steady at the
    first test; a sheared droplet keeps deforming.  The controller reports the step at
    which each met |D(t) - D(t - window)| < tol (over one window, or each of several
    consecutive ones) and stops advancing it."""
    still = workloads.droplet_shear(nx=24, ny=12, nz=16, R=3.0, rho_in=0.5, rho_out=0.5, G=0.0,
                                    polymer_phase="none", U=0.01)
    moving = workloads.droplet_shear(nx=48, ny=24, nz=32, R=6.0, G=workloads.G_PHYSICS_1_004,
                                     polymer_phase="A", De=0.5, U=0.03)
    b = lb.Batch([still, moving])
    seen = []
    diags, ss = b.run_to_steady(every=10, window=20, tol=1e-6, max_steps=200,
                                progress=lambda step, active: seen.append((step, active)))
    assert ss[0] == 30  # three samples are needed for a window of two intervals
    # the progress report: after every chunk of steps, with the instances still stepping
    assert [s for s, _ in seen] == list(range(10, 10 * len(seen) + 1, 10))
    assert seen[2] == (30, 1) and seen[1] == (20, 2)
    assert seen[-1][0] == (200 if ss[1] == -1 else ss[1])
    assert diags[0]["step"] == ss[0]
    assert ss[1] == -1 or ss[1] > ss[0]
    assert diags[1]["step"] == (200 if ss[1] == -1 else ss[1])
    b.close()
    # two consecutive windows: five samples for the still mixture; the sheared droplet
    # never qualifies earlier than under one window
    b = lb.Batch([still, moving])
    diags2, ss2 = b.run_to_steady(every=10, window=20, tol=1e-6, max_steps=200, windows=2)
    assert ss2[0] == 50 and diags2[0]["step"] == 50
    assert ss2[1] == -1 or (ss[1] != -1 and ss2[1] >= ss[1])
    with pytest.raises(lb.LbfdError):
        b.run_to_steady(every=10, window=20, tol=1e-6, max_steps=20, windows=-1)
    b.close()


@pytest.mark.parametrize("scheme,tile", [("default", "64x8"), ("paper", "64x8"), ("default", "32x16")])
def test_batch_instances_match_the_oracle(lb, scheme, tile):
    """Each instance of one batch of three uneven lattices (one ragged in every direction,
    one with a viscosity ratio, one with a narrow wall gap) against the FP64 oracle run on
    the same seeded inputs: fields to the 1e-5 relative-L2 bar of the single-lattice tests
    and every diagnostics field.  `paper` runs the paper's scheme throughout (MRT
    collision, stress in the equilibrium, Cholesky-log integrator with artificial
    diffusivity) in the chained batch body; `default` the default schemes."""
    import oracle
    from parity_helpers import I6, check_diag, grid_shape, rel

    G = workloads.G_PHYSICS_1_004
    cases = [
        workloads.droplet_shear(nx=40, ny=16, nz=24, R=5.0, G=G, polymer_phase="A", De=0.5, U=0.01),
        workloads.droplet_shear(nx=37, ny=21, nz=13, R=4.0, G=G, polymer_phase="B", L2=400.0, De=1.0,
                                U=0.005, tau_A=1.3),
        workloads.droplet_shear(nx=72, ny=12, nz=30, R=4.0, G=G, polymer_phase="A", De=1.0, U=0.015,
                                tau_A=0.8),
    ]
    if scheme == "paper":
        cases = [dict(w, params=dict(w["params"], collision="mrt", fene="cholesky_ab2", coupling="stress",
                                     kappa=0.01)) for w in cases]
    steps = 300
    b = lb.Batch(cases)
    assert b.get_tuning()["path"] == lb.PATH_CHAINED
    b.set_tuning(tile, 0, path=lb.PATH_CHAINED)
    b.step(steps)
    dgs = b.diagnostics()
    got = [b.get_fields(i) for i in range(len(cases))]
    b.close()
    for i, wl in enumerate(cases):
        o = oracle.from_workload(wl)
        assert o.step(steps) == 0
        r = o.get_fields()
        g = got[i]
        e = {"u": rel(g[1], r[1]), "C": rel(g[2], r[2]), "C-I": rel(g[2] - I6, r[2] - I6),
             "rho": rel(g[0], r[0])}
        print(f"batch-{scheme}-{tile}-{i}", " ".join(f"{k}={v:.2e}" for k, v in e.items()), flush=True)
        assert e["u"] < 1e-5 and e["C"] < 1e-5 and e["rho"] < 1e-5 and e["C-I"] < 1e-5, (i, e)
        check_diag(dgs[i], o.diagnostics(), f"batch-{scheme}-{i}", g, r, grid_shape(wl), wl["params"])
