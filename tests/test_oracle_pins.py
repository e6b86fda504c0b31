"""Field-level pins of the FP64 oracle: exact lattice closed forms of the Shan-Chen
force and the polymer-stress divergence, conservation and antisymmetry invariants,
the Newtonian Couette profile, linearity (G = 0 two-component = one component), the
Shan-Chen critical coupling and printed bulk densities, and the droplet-shape
diagnostics on synthetic ellipsoids."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def coords(nx, ny, nz):
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return X.ravel().astype(float), Y.ravel().astype(float), Z.ravel().astype(float)


def make(nx, ny, nz, nc, rho, u=None, C=None, **params):
    o = oracle.Oracle(nx, ny, nz, nc)
    o.set_params(**params)
    o.set_walls([0, 0, 0], [0, 0, 0])
    N = nx * ny * nz
    if u is None:
        u = np.zeros((3, N))
    if C is None:
        C = np.zeros((6, N))
        C[:3] = 1.0
    o.set_fields(rho, u, C)
    return o


@pytest.mark.parametrize("axis", [0, 2])
def test_shan_chen_force_sine_closed_form(axis):
    """rho_B = a + b sin(k x_axis): the D3Q19 sum over links with c_axis = +-1 has total
    weight 1/6 per side, so sum_a w_a rho_B(x + c_a) c_a = (b/3) sin(k) cos(k x) e_axis
    exactly and g_A = -G rho_A (b/3) sin(k) cos(k x) (Sec. 2, eq. SCforce).  Its Taylor
    expansion is the paper's -c_s^2 G rho_A grad rho_B - (c_s^4/2) G rho_A Lap grad rho_B."""
    nx, ny, nz = (16, 3, 4) if axis == 0 else (4, 3, 16)
    X, Y, Z = coords(nx, ny, nz)
    s = X if axis == 0 else Z
    n = nx if axis == 0 else nz
    k = 2 * math.pi / n
    a, b, G = 0.7, 0.05, 1.3
    rho = np.zeros((2, X.size))
    rho[0] = 0.9 + 0.02 * np.cos(k * s)
    rho[1] = a + b * np.sin(k * s)
    o = make(nx, ny, nz, 2, rho, G=G)
    g, _, _ = o.get_forces()
    sB = (b / 3.0) * math.sin(k) * np.cos(k * s)
    sA = -(0.02 / 3.0) * math.sin(k) * np.sin(k * s)
    exp_gA = -G * rho[0] * sB
    exp_gB = -G * rho[1] * sA
    assert np.allclose(g[0, axis], exp_gA, rtol=0, atol=1e-15)
    assert np.allclose(g[1, axis], exp_gB, rtol=0, atol=1e-15)
    for d in range(3):
        if d != axis:
            assert np.allclose(g[:, d], 0, atol=1e-16)
    # long-wavelength agreement with the printed Taylor expansion
    cs2 = 1.0 / 3.0
    taylor = -G * rho[0] * (cs2 * b * k * np.cos(k * s) - 0.5 * cs2 ** 2 * b * k ** 3 * np.cos(k * s))
    assert np.allclose(g[0, axis], taylor, atol=abs(G * b) * k ** 5)


def test_shan_chen_wall_neighbours_copy_wall_layer():
    """Across a y wall the Shan-Chen neighbours see the wall-adjacent layer (neutral
    wetting): for rho varying only with y, sum_a w_a rho(x+c_a) c_a,y = (rho(y+1) -
    rho(y-1))/6 with rho(-1) = rho(0) and rho(ny) = rho(ny-1)."""
    nx, ny, nz = 3, 8, 3
    X, Y, Z = coords(nx, ny, nz)
    prof = np.array([0.3, 0.45, 0.2, 0.9, 0.55, 0.1, 0.7, 0.35])
    rho = np.zeros((2, X.size))
    rho[0] = 1.0
    rho[1] = prof[Y.astype(int)]
    G = 0.8
    o = make(nx, ny, nz, 2, rho, G=G)
    g, _, _ = o.get_forces()
    ext = np.concatenate([[prof[0]], prof, [prof[-1]]])
    expect_y = -G * 1.0 * (ext[2:] - ext[:-2]) / 6.0
    assert np.allclose(g[0, 1], expect_y[Y.astype(int)], atol=1e-16)
    assert np.allclose(g[0, 0], 0, atol=1e-16) and np.allclose(g[0, 2], 0, atol=1e-16)


def test_shan_chen_pairwise_antisymmetry():
    """For any field uniform in y (walls inert), sum_x (g_A + g_B) = 0: the interaction
    is pairwise and antisymmetric under x -> x + c_a, a -> opposite(a)."""
    nx, ny, nz = 8, 3, 6
    rng = np.random.default_rng(3)
    base = rng.uniform(0.05, 1.2, size=(2, nz, 1, nx))
    rho = np.broadcast_to(base, (2, nz, ny, nx)).reshape(2, -1).copy()
    o = make(nx, ny, nz, 2, rho, G=2.1)
    g, _, _ = o.get_forces()
    tot = g.sum(axis=(0, 2))
    scale = np.abs(g).sum()
    assert np.all(np.abs(tot) < 1e-14 * scale)
    assert scale > 1e-2


def test_polymer_force_closed_form():
    """C_xx = c0 + b sin(kz), C_zz = c0 - b sin(kz), C_yy = 1: the trace is uniform so
    f(r) = (L^2 - 3)/(L^2 - tr C) is a constant, T_zz = (eta_p/tau_p) m (f C_zz - 1) and the
    central divergence gives F_p,z = -(eta_p/tau_p) m f b sin(k) cos(kz), F_p,x = F_p,y = 0.
    C_xz = e sin(kz) adds F_p,x = (eta_p/tau_p) m f e sin(k) cos(kz).  Two components with
    uniform phi = 0.2 and polymer in A give m = f+(phi) = (1 + tanh(phi/0.1))/2 and the force
    split F_A = (rho_A/rho) F_p (Sec. 2, FENE-P feedback, eqs. smoothingvisco, MODEtransformation)."""
    nx, ny, nz = 3, 3, 12
    X, Y, Z = coords(nx, ny, nz)
    k = 2 * math.pi / nz
    c0, b, e, L2 = 1.5, 0.1, 0.05, 60.0
    C = np.zeros((6, X.size))
    C[0] = c0 + b * np.sin(k * Z)
    C[1] = 1.0
    C[2] = c0 - b * np.sin(k * Z)
    C[4] = e * np.sin(k * Z)
    rho = np.zeros((2, X.size))
    rho[0], rho[1] = 0.6, 0.4
    eta_p, tau_p = 0.3, 50.0
    o = make(nx, ny, nz, 2, rho, C=C, G=0.0, polymer_phase="A", eta_p=eta_p, tau_p=tau_p, L2=L2)
    g, Fp, F = o.get_forces()
    fr = (L2 - 3.0) / (L2 - (2 * c0 + 1.0))
    m = 0.5 * (1 + math.tanh(0.2 / GOLD["smoothing_delta"]["value"]))
    pre = eta_p / tau_p * m * fr
    assert np.allclose(Fp[2], -pre * b * math.sin(k) * np.cos(k * Z), atol=1e-17)
    assert np.allclose(Fp[0], pre * e * math.sin(k) * np.cos(k * Z), atol=1e-17)
    assert np.allclose(Fp[1], 0, atol=1e-18)
    assert np.allclose(F[0], 0.6 * Fp, atol=1e-18)
    assert np.allclose(F[1], 0.4 * Fp, atol=1e-18)
    # polymer in B uses f-(phi); no feedback at all for polymer_phase none
    o.set_params(G=0.0, polymer_phase="B", eta_p=eta_p, tau_p=tau_p, L2=L2)
    _, Fp_b, _ = o.get_forces()
    mb = 0.5 * (1 - math.tanh(0.2 / 0.1))
    assert np.allclose(Fp_b, Fp * mb / m, atol=1e-18)
    o.set_params(G=0.0, polymer_phase="none", eta_p=eta_p, tau_p=tau_p, L2=L2)
    _, Fp_n, _ = o.get_forces()
    assert np.all(Fp_n == 0)


def test_polymer_force_telescopes():
    """Central differences telescope: sum_x F_p = 0 for any field uniform in y."""
    nx, ny, nz = 6, 3, 5
    rng = np.random.default_rng(11)
    _, _, C = workloads.random_state(nx, 1, nz, 1, seed=4)
    C = np.broadcast_to(C.reshape(6, nz, 1, nx), (6, nz, ny, nx)).reshape(6, -1).copy()
    rho = np.ones((1, nx * ny * nz))
    o = make(nx, ny, nz, 1, rho, C=C, polymer_phase="all", eta_p=0.2, tau_p=10.0, L2=50.0)
    _, Fp, _ = o.get_forces()
    assert np.abs(Fp).sum() > 1e-4
    assert np.all(np.abs(Fp.sum(1)) < 1e-15)


def test_newtonian_couette_steady_profile():
    """Plane Couette, eta_p = 0, from rest: the steady profile of half-way bounce-back
    with moving walls is u_x = -U + 2U (y + 1/2)/ny (exact for linear profiles; walls at
    y = -1/2 and ny - 1/2; Sec. 3.1 set-up)."""
    nx, ny, nz, U = 2, 16, 2, 0.01
    N = nx * ny * nz
    o = make(nx, ny, nz, 1, np.ones((1, N)))
    o.set_walls([-U, 0, 0], [U, 0, 0])
    assert o.step(6000) == 0
    _, u, _ = o.get_fields()
    _, Y, _ = coords(nx, ny, nz)
    exact = -U + 2 * U * (Y + 0.5) / ny
    assert np.max(np.abs(u[0] - exact)) < 1e-12
    assert np.max(np.abs(u[1:])) < 1e-14


@pytest.mark.parametrize("G", [0.0, 3.3])
def test_mass_conserved_per_species(G):
    """Collision conserves rho_s, streaming moves it, half-way bounce-back returns it to
    the same node and the moving-wall corrections of the +-c_x links cancel."""
    wl = workloads.droplet_shear(nx=20, ny=12, nz=16, R=4.0, G=G, polymer_phase="A", De=0.5,
                                 U=0.02)
    o = oracle.from_workload(wl)
    d0 = o.diagnostics()
    assert o.step(150) == 0
    d1 = o.diagnostics()
    for key in ("mass_A", "mass_B"):
        assert abs(d1[key] - d0[key]) < 1e-13 * d0[key]


@pytest.mark.parametrize("G", [0.0, 3.3])
def test_papers_scheme_conserves_mass_and_keeps_c_spd(G):
    """With the paper's scheme throughout (MRT collision, polymer stress in the
    equilibrium's second moment, Cholesky-log AB2 integrator with artificial diffusivity)
    the collision still conserves each species' mass exactly (the relaxed modes carry no
    mass), and C stays symmetric positive definite with tr C < L^2 at every node: the
    Cholesky scheme builds C from a factor with positive diagonal."""
    wl = workloads.droplet_shear(nx=20, ny=12, nz=16, R=4.0, G=G, polymer_phase="A", De=0.5,
                                 U=0.02, tau_A=0.7, tau_B=1.2, coupling="stress")
    wl["params"].update(collision="mrt", fene="cholesky_ab2", kappa=0.01)
    o = oracle.from_workload(wl)
    d0 = o.diagnostics()
    assert o.step(150) == 0
    d1 = o.diagnostics()
    for key in ("mass_A", "mass_B"):
        assert abs(d1[key] - d0[key]) < 1e-13 * d0[key]
    _, _, C = o.get_fields()
    xx, yy, zz, xy, xz, yz = C
    m2 = xx * yy - xy * xy
    m3 = xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz)
    assert xx.min() > 0 and m2.min() > 0 and m3.min() > 0
    assert (xx + yy + zz).max() < wl["params"]["L2"]
    # the droplet's polymer is stretched by the shear: the scheme is not idle
    assert np.abs(xy).max() > 1e-4


def test_two_components_at_zero_coupling_equal_one_component():
    """G = 0, equal tau, single-phase polymer: the sum of two components behaves as one
    fluid of density rho_A + rho_B (the model is linear in the populations except
    through rho and u, Sec. 3 intro: G = 0 gives two miscible ideal gases)."""
    nx, ny, nz = 6, 6, 5
    rho1, u, C = workloads.random_state(nx, ny, nz, 1, seed=5, amp_rho=0.02, amp_u=0.01, amp_C=0.05)
    rng = np.random.default_rng(9)
    share = rng.uniform(0.2, 0.8, rho1.shape[1])
    rho2 = np.stack([rho1[0] * share, rho1[0] * (1 - share)])
    kw = dict(tau_A=0.8, tau_B=0.8, G=0.0, polymer_phase="all", eta_p=0.05, tau_p=40.0, L2=30.0)
    o1 = make(nx, ny, nz, 1, rho1, u=u, C=C, **kw)
    o2 = make(nx, ny, nz, 2, rho2, u=u, C=C, **kw)
    for o in (o1, o2):
        o.set_walls([-0.01, 0, 0.003], [0.01, 0, -0.002])
        assert o.step(40) == 0
    r1, u1, C1 = o1.get_fields()
    r2, u2, C2 = o2.get_fields()
    assert np.allclose(r1[0], r2.sum(0), rtol=0, atol=1e-13)
    assert np.allclose(u1, u2, rtol=0, atol=1e-14)
    assert np.allclose(C1, C2, rtol=0, atol=1e-13)


@pytest.mark.parametrize("Grho,grows", [(2.5, True), (1.5, False)])
def test_shan_chen_critical_coupling(Grho, grows):
    """Linear stability of the bulk pressure P_b = c_s^2 (rho_A + rho_B + G rho_A rho_B)
    (Sec. 2, eq. PTexpanded) puts the spinodal of a symmetric mixture at G rho_tot = 2:
    composition noise grows above it and decays below it."""
    nx, ny, nz = 64, 3, 1
    rng = np.random.default_rng(21)
    noise = 0.01 * rng.uniform(-1, 1, nx)
    rho_tot = 1.0
    X, Y, Z = coords(nx, ny, nz)
    rho = np.zeros((2, X.size))
    rho[0] = 0.5 * rho_tot * (1 + noise[X.astype(int)])
    rho[1] = 0.5 * rho_tot * (1 - noise[X.astype(int)])
    o = make(nx, ny, nz, 2, rho, G=Grho / rho_tot)
    var0 = np.var(rho[0] - rho[1])
    assert o.step(600) == 0
    r, _, _ = o.get_fields()
    var1 = np.var(r[0] - r[1])
    assert (var1 > 10 * var0) if grows else (var1 < 0.5 * var0)


def test_shan_chen_flat_interface_bulk_densities():
    """G = 1.5 at total density 2.1 phase-separates into bulk densities about 2.0 / 0.1
    (Sec. 4.1 set-up paragraph; Appendix A ranges 1.9-2.15 and 0.05-0.2).  The
    symmetric mean-field binodal of P_b gives 1.978 / 0.122."""
    gold = GOLD["shan_chen_calibration"]
    nx, ny, nz = 64, 3, 1
    X, Y, Z = coords(nx, ny, nz)
    inside = (X >= 16) & (X < 48)
    rho = np.zeros((2, X.size))
    rho[0] = np.where(inside, 1.9, 0.2)
    rho[1] = np.where(inside, 0.2, 1.9)
    o = make(nx, ny, nz, 2, rho, G=gold["G"])
    assert o.step(8000) == 0
    r, u, _ = o.get_fields()
    rA_in = r[0][X == 32].mean()
    rB_in = r[1][X == 32].mean()
    lo, hi = GOLD["shan_chen_ranges"]["rho_A_bulk"]
    assert lo <= rA_in <= hi and abs(rA_in - gold["rho_A_bulk"]) < 0.1 * gold["rho_A_bulk"]
    lo, hi = GOLD["shan_chen_ranges"]["rho_B_bulk"]
    assert lo <= rB_in <= hi
    # symmetric profile, quiescent interface
    assert abs(r[0][X == 32].mean() - r[1][X == 0].mean()) < 1e-8
    assert np.max(np.abs(u)) < 1e-6
    # interface width (10 % - 90 % of the phi jump) is a few cells (Appendix A: 3-8)
    phi = ((r[0] - r[1]) / (r[0] + r[1]))[(Y == 0)]
    prof = phi[:32]
    lo_v, hi_v = prof.min(), prof.max()
    frac = (prof - lo_v) / (hi_v - lo_v)
    width = np.sum((frac > 0.1) & (frac < 0.9))
    assert 2 <= width <= 8


@pytest.mark.parametrize("a,b,ang", [(10.0, 6.0, 30.0), (9.0, 9.0, 0.0), (12.0, 5.0, -50.0)])
def test_droplet_diagnostics_ellipsoid(a, b, ang):
    """Deformation D = (a - b)/(a + b) and orientation theta of a synthetic ellipsoid
    indicator field (Sec. 4.1, definitions of D and theta), within voxelisation error."""
    nx, ny, nz = 48, 40, 24
    X, Y, Z = coords(nx, ny, nz)
    xc, yc, zc = (nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2
    t = math.radians(ang)
    dx, dy, dz = X - xc, Y - yc, Z - zc
    p = dx * math.cos(t) + dy * math.sin(t)
    q = -dx * math.sin(t) + dy * math.cos(t)
    inside = (p / a) ** 2 + (q / b) ** 2 + (dz / 6.0) ** 2 < 1
    rho = np.zeros((2, X.size))
    rho[0] = np.where(inside, 1.0, 0.04)
    rho[1] = np.where(inside, 0.04, 1.0)
    o = make(nx, ny, nz, 2, rho)
    d = o.diagnostics()
    assert abs(d["D"] - (a - b) / (a + b)) < 1e-2
    if a != b:
        assert abs(d["theta_deg"] - ang) < 1.0
    else:
        assert d["D"] < 1e-2
    assert abs(d["xc"] - xc) < 1e-9 and abs(d["yc"] - yc) < 1e-9


def test_conformation_wall_ghost_is_linear_extrapolation():
    """C is extrapolated linearly across the walls (Sec. 2, boundary condition of the
    conformation tensor): for C_xy = a + b y and C_xx = 1.2 - b' y, C_yy = 1 + b' y
    (uniform trace), the central divergence F_p,x = d_y T_yx = (eta_p/tau_p) f b and
    F_p,y = d_y T_yy = (eta_p/tau_p) f b' hold at every node, wall layers included."""
    nx, ny, nz = 2, 7, 2
    X, Y, Z = coords(nx, ny, nz)
    a, b, bp, L2 = 0.05, 0.01, 0.02, 40.0
    C = np.zeros((6, X.size))
    C[0] = 1.2 - bp * Y
    C[1] = 1.0 + bp * Y
    C[2] = 1.0
    C[3] = a + b * Y
    rho = np.ones((1, X.size))
    eta_p, tau_p = 0.4, 20.0
    o = make(nx, ny, nz, 1, rho, C=C, polymer_phase="all", eta_p=eta_p, tau_p=tau_p, L2=L2)
    _, Fp, _ = o.get_forces()
    fr = (L2 - 3) / (L2 - 3.2)
    assert np.allclose(Fp[0], eta_p / tau_p * fr * b, rtol=1e-12, atol=0)
    assert np.allclose(Fp[1], eta_p / tau_p * fr * bp, rtol=1e-12, atol=0)
    assert np.allclose(Fp[2], 0, atol=1e-18)


def test_upwind_advection_translates_and_stays_monotone():
    """Prescribed uniform velocity, no stretching (uniform u) and negligible relaxation:
    the first-order upwind step conserves sum_x C, moves the centroid of a bump at the
    flow speed in the flow direction, and creates no new extrema (CFL < 1)."""
    nx, ny, nz = 160, 3, 1
    X, Y, Z = coords(nx, ny, nz)
    for ux in (0.25, -0.25):
        o = oracle.Oracle(nx, ny, nz, 1)
        o.set_params(polymer_phase="none", tau_p=1e300, L2=1e300)
        o.set_walls([ux, 0, 0], [ux, 0, 0])
        u = np.zeros((3, X.size))
        u[0] = ux
        C = np.zeros((6, X.size))
        C[:3] = 1.0
        bump = np.exp(-0.5 * ((X - 80) / 3.0) ** 2)
        C[0] += bump
        C[3] = 0.5 * bump
        o.set_fields(np.ones((1, X.size)), u, C)
        steps = 40
        assert o.fenep_kinematic(u, steps) == 0
        Cn = o.get_C()
        for k in (0, 3):
            ex = Cn[k] - (1.0 if k == 0 else 0.0)
            assert abs(ex.sum() - (C[k] - (1.0 if k == 0 else 0.0)).sum()) < 1e-12
            cen0 = (X * (C[k] - (k == 0))).sum() / (C[k] - (k == 0)).sum()
            cen1 = (X * ex).sum() / ex.sum()
            assert abs(cen1 - cen0 - ux * steps) < 1e-9
            assert ex.max() <= (C[k] - (k == 0)).max() + 1e-15 and ex.min() >= -1e-15


@pytest.mark.parametrize("tau", [1.0, 0.8, 1.7])
def test_stress_coupling_first_step_closed_form(tau):
    """Stress coupling (Sec. 2, eq. MODEtransformation) from rest: one component at uniform
    density, C = I + a sin(k z) (e_x e_z + e_z e_x), so tr C = 3, f(r) = 1 and
    T_xz = (eta_p/tau_p) a sin(k z).  The collision moves the populations by
    -(9/tau) w c_x c_z T_xz toward the lowered equilibrium; streaming over the four
    (+-1, 0, +-1) links then gives exactly j_x(z) = (eta_p/tau_p) a sin(k) cos(k z) / tau,
    the central divergence of T divided by tau, with rho unchanged.  With the body-force
    coupling the same field gives the force (eta_p/tau_p) a sin(k) cos(k z) instead."""
    nx, ny, nz = 4, 5, 24
    k = 2 * np.pi / nz
    a, eta_p, tau_p = 0.1, 0.02, 50.0
    wl = workloads.couette_fenep(nx=nx, ny=ny, nz=nz, U=0.0, tau=tau, tau_p=tau_p, L2=100.0,
                                 noise=0.0, coupling="stress")
    wl["params"]["eta_p"] = eta_p
    N = nx * ny * nz
    Z = np.repeat(np.arange(nz), nx * ny)
    wl["u"] = np.zeros((3, N))
    wl["rho"] = np.ones((1, N))
    wl["C"][4] = a * np.sin(k * Z)
    o = oracle.from_workload(wl)
    assert o.step(1) == 0
    rho, u, _ = o.get_fields()
    expect = eta_p / tau_p * a * np.sin(k) * np.cos(k * Z) / tau
    assert np.allclose(rho[0], 1.0, rtol=0, atol=1e-15)
    assert np.allclose(u[0], expect, rtol=0, atol=1e-15)
    assert np.max(np.abs(u[1:])) < 1e-15
    # the body-force coupling sees the same divergence as a force
    wl["params"]["coupling"] = "force"
    o = oracle.from_workload(wl)
    _, Fp, _ = o.get_forces()
    assert np.allclose(Fp[0], eta_p / tau_p * a * np.sin(k) * np.cos(k * Z), rtol=0, atol=1e-16)


@pytest.mark.parametrize("phi", [-0.05, 0.05, 0.3])
def test_local_relaxation_time_from_shear_wave_decay(phi):
    """S7 (Sec. 2, eq. smoothingvisco, read as an interpolation of tau): a uniform miscible
    mixture (G = 0) at order parameter phi relaxes with tau = tau_B + (tau_A - tau_B) f+(phi),
    f+ = (1 + tanh(phi/Delta))/2, so a small shear wave u_x = a sin(k z) decays at the BGK
    kinematic viscosity nu = c_s^2 (tau - 1/2) (the transport coefficient of
    eq. TRANSPORTCOEFF at unit rates).  tau_A = 1.4 and tau_B = 0.7 give viscosities 60 %
    apart at phi = +-0.05, so the phase that receives tau_A, the tanh form and its width
    are each fixed; lattice corrections at k = 2 pi/64 stay below 0.3 %.  The wave is read
    at the centre row of a channel wide enough that the wall layers do not reach it."""
    nx, ny, nz = 1, 96, 64
    N = nx * ny * nz
    X, Y, Z = coords(nx, ny, nz)
    k = 2 * math.pi / nz
    tau_A, tau_B, delta = 1.4, 0.7, 0.1
    rho = np.stack([np.full(N, 0.5 * (1 + phi)), np.full(N, 0.5 * (1 - phi))])
    u = np.zeros((3, N))
    u[0] = 1e-3 * np.sin(k * Z)
    o = make(nx, ny, nz, 2, rho, u, tau_A=tau_A, tau_B=tau_B, G=0.0, delta=delta)
    row = Y == ny // 2

    def amp():
        _, uu, _ = o.get_fields()
        return 2.0 / nz * np.sum(uu[0][row] * np.sin(k * Z[row]))

    assert o.step(100) == 0
    a1 = amp()
    assert o.step(200) == 0
    a2 = amp()
    nu = -math.log(a2 / a1) / (k * k * 200)
    tau = tau_B + (tau_A - tau_B) * 0.5 * (1.0 + math.tanh(phi / delta))
    assert abs(nu - (tau - 0.5) / 3.0) < 3e-3 * (tau - 0.5) / 3.0, (nu, (tau - 0.5) / 3.0)


def _one_node_state(C6, nx=3, ny=3, nz=3, u=None):
    """Unit-density one-component lattice at rest whose centre node holds C6 (all others
    C = I)."""
    N = nx * ny * nz
    C = np.zeros((6, N))
    C[:3] = 1.0
    centre = ((nz // 2) * ny + ny // 2) * nx + nx // 2
    C[:, centre] = C6
    return np.ones((1, N)), (np.zeros((3, N)) if u is None else u), C


@pytest.mark.parametrize("C6,flag", [
    # leading minors 1, 1 and det = 0.19 - 0.81 < 0 (xz = yz = 0.9)
    ([1.0, 1.0, 1.0, 0.0, 0.9, 0.9], oracle.FLAG_NOT_SPD),
    # det < 0 with unequal couplings: 0.91 - 0.2 (0.2 + 0.285) + 0.95 (-0.06 - 0.95) = -0.147
    ([1.0, 1.0, 1.0, 0.2, 0.95, -0.3], oracle.FLAG_NOT_SPD),
    # second minor 1 - 1.44 < 0
    ([1.0, 1.0, 1.0, 1.2, 0.0, 0.0], oracle.FLAG_NOT_SPD),
    # second minor negative while the determinant (-0.44)(-1) is positive: only the second
    # minor shows it
    ([1.0, 1.0, -1.0, 1.2, 0.0, 0.0], oracle.FLAG_NOT_SPD),
    # SPD close to the boundary (det = 0.8236 - 0.81 = 0.0136 > 0): no flag
    ([1.0, 1.0, 1.0, 0.0, 0.9, 0.42], 0),
    # first minor negative
    ([-0.2, 1.0, 1.0, 0.0, 0.0, 0.0], oracle.FLAG_NOT_SPD),
    # tr C above L^2 = 100
    ([98.0, 1.5, 1.5, 0.0, 0.0, 0.0], oracle.FLAG_EXTENSIBILITY),
])
def test_fault_checks_raise_each_flag(C6, flag):
    """S11: a state with one node outside the admissible set raises exactly the flag of
    the violated condition after a step (the oracle never clips; flags: non-finite 1,
    tr C >= L^2 2, a leading principal minor <= 0 4).  tau_P = 1e6 leaves C almost unchanged
    over the step; the determinant of each SPD-violating case is checked against numpy's,
    so the expected flag follows from linear algebra, not from the oracle's own formula."""
    xx, yy, zz, xy, xz, yz = C6
    M = np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])
    spd = M[0, 0] > 0 and np.linalg.det(M[:2, :2]) > 0 and np.linalg.det(M) > 0
    assert spd == (flag != oracle.FLAG_NOT_SPD)
    rho, u, C = _one_node_state(C6)
    o = make(3, 3, 3, 1, rho, u, C, polymer_phase="none", tau_p=1e6, L2=100.0)
    assert o.step(1) == flag
    if flag:
        assert o.steps == 1 and o.diagnostics()["flags"] == flag


def test_fault_checks_non_finite_and_driven_extensibility():
    """S11 raised by the dynamics: a NaN in C flags non-finite; one step of strong shear
    takes tr C past L^2 = 10 (flag 2 alone: C stays finite and SPD); a
    relaxation time tau_P = 0.3 below one step makes forward Euler overshoot C = diag(3,
    0.3, 0.3) to a negative C_xx (flag 4 alone)."""
    rho, u, C = _one_node_state([np.nan, 1.0, 1.0, 0.0, 0.0, 0.0])
    o = make(3, 3, 3, 1, rho, u, C, polymer_phase="none", tau_p=100.0, L2=100.0)
    assert o.step(1) & oracle.FLAG_NONFINITE
    # FENE-P's f(r) diverges as tr C -> L^2, so a slow drive never crosses it; one step of
    # shear gdot = 0.625 on C_xy = 2 adds 2 gdot C_xy = 2.5 to C_xx: tr C 8 -> 10.5 > L^2 = 10,
    # while C stays SPD (second minor 8.5 - 2.625^2 = 1.61)
    nx, ny, nz = 3, 4, 3
    N = nx * ny * nz
    _, Y, _ = coords(nx, ny, nz)
    gdot = 0.625
    U = gdot * ny / 2
    u = np.zeros((3, N))
    u[0] = gdot * (Y - (ny - 1) / 2)
    C = np.zeros((6, N))
    C[0], C[1], C[2], C[3] = 6.0, 1.0, 1.0, 2.0
    o = oracle.Oracle(nx, ny, nz, 1)
    o.set_params(polymer_phase="none", tau_p=1e4, L2=10.0)
    o.set_walls([-U, 0, 0], [U, 0, 0])
    o.set_fields(np.ones((1, N)), u, C)
    assert o.step(5) == oracle.FLAG_EXTENSIBILITY and o.steps == 1
    rho, u, C = _one_node_state([3.0, 0.3, 0.3, 0.0, 0.0, 0.0])
    o = make(3, 3, 3, 1, rho, u, C, polymer_phase="none", tau_p=0.3, L2=100.0)
    assert o.step(1) == oracle.FLAG_NOT_SPD


def test_velocity_momentum_and_trace_diagnostics_on_known_fields():
    """Diagnostics on fields whose values are known by construction (no force acts: G = 0
    and no polymer feedback, so u is the u the populations were set from):
    max |u| is the largest speed put in, 0.05 at one node; the momentum is sum (rho_A +
    rho_B) u, here the total mass times a uniform drift plus that node's excess; the
    polymer-phase mean of tr C - 3 is the mean over the nodes of the polymer's phase
    (rho of the other species 1e-6, so f+-(phi) = 1 or 0 to 1e-8): 0.6 for phase A and 5.0
    for phase B."""
    nx, ny, nz = 8, 6, 4
    N = nx * ny * nz
    X, Y, Z = coords(nx, ny, nz)
    a_rich = X < 4
    rho = np.stack([np.where(a_rich, 1.0, 1e-6), np.where(a_rich, 1e-6, 0.8)])
    u = np.zeros((3, N))
    u[0] = 0.01
    spot = 17
    u[:, spot] = [0.03, -0.04, 0.0]
    C = np.zeros((6, N))
    C[:3] = 1.0
    C[0] = np.where(a_rich, 1.6, 6.0)  # tr C - 3 = 0.6 on the A side, 5.0 on the B side
    for phase, expect in (("A", 0.6), ("B", 5.0)):
        o = make(nx, ny, nz, 2, rho, u, C, G=0.0, polymer_phase=phase, eta_p=0.0, tau_p=1e6)
        d = o.diagnostics()
        assert abs(d["max_u"] - 0.05) < 1e-15
        mass = rho.sum()
        rs = rho.sum(0)[spot]
        assert abs(d["mom_x"] - (0.01 * mass + (0.03 - 0.01) * rs)) < 1e-12
        assert abs(d["mom_y"] - (-0.04 * rs)) < 1e-15 and abs(d["mom_z"]) < 1e-15
        assert abs(d["poly_trace_excess"] - expect) < 1e-6, (phase, d["poly_trace_excess"])
