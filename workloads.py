"""Seeded synthetic inputs for the hybrid LB/FD step.

This module is the ONLY code shared by the GPU library's tests/benchmark and the CPU
oracle.  It builds initial macroscopic fields (densities, velocity, conformation
tensor) and parameter sets from seeds; it performs none of the method's arithmetic
(no equilibrium, no forces, no collision, no FENE-P update).

Every workload is a dict::

    {"name": str,
     "grid":   {"nx", "ny", "nz", "ncomp"},              # y is the wall-normal axis
     "params": {"tau_A", "tau_B", "G", "delta", "rho0": [r0A, r0B],
                "polymer_phase": "none"|"A"|"B"|"all", "eta_p", "tau_p", "L2",
                "coupling": "force"|"stress"},
     "walls":  {"u_bottom": [ux, 0, uz], "u_top": [ux, 0, uz]},
     "rho": (ncomp, N) f64, "u": (3, N) f64, "C": (6, N) f64}

with host layout [field][z][y][x] flattened (x fastest) and C components ordered
(xx, yy, zz, xy, xz, yz).

Recipes (all lattice units, c_s^2 = 1/3, dt = dx = 1):

* ``couette_fenep`` -- single-component FENE-P plane Couette: 16x32x16, rho = 1, tau = 1
  (solvent viscosity eta_s = (tau - 1/2)/3 = 1/6), polymer concentration
  eta_p/(eta_s + eta_p) = 0.2 so eta_p = eta_s/4, tau_p = 1000, L^2 = 100, walls at
  u_x = -/+ 0.01 (bottom/top), linear Couette start u_x = gdot (y - (ny-1)/2) with
  gdot = 2U/ny, C = I + (N + N^T)/2 with N_ij ~ U(-1e-3, 1e-3) from
  ``numpy.random.default_rng(seed)`` drawn as one (N, 3, 3) array.
* ``droplet_shear`` -- two-component Shan-Chen droplet in confined shear: sharp sphere of
  radius R centred at ((nx-1)/2, (ny-1)/2, (nz-1)/2), rho_A = rho_in inside / rho_out
  outside (B reversed), Couette start, C = I.  Polymer in the droplet (A) or matrix (B).
  The wall speed follows from the capillary number, Ca = gdot R eta_M / sigma_AB with
  gdot = 2U/H; the polymer time from the Oldroyd-B Deborah number
  De = (tau_p/tau_em)(eta_p/eta_M), tau_em = R eta_M/sigma_AB.
"""
from __future__ import annotations

import math

import numpy as np

CS2 = 1.0 / 3.0

# Coupling at which a flat A/B interface coexists at bulk densities (1.0, 0.04): the
# symmetric mean-field binodal of the bulk pressure P_b = c_s^2 (rho_A + rho_B + G rho_A rho_B)
# gives ln(a/b) = G (a - b).
G_PHYSICS_1_004 = math.log(1.0 / 0.04) / (1.0 - 0.04)

# Interfacial tension used to convert Ca into a wall speed (lattice units): Laplace-law fit
# over resting droplets of radius 8-12 at G = G_PHYSICS_1_004, rho 1.0/0.04, measured with
# the FP64 oracle by tests/golden/sigma_calibration.py (result 0.07681, spread 0.0764-0.0773).
SIGMA_AB_1_004 = 0.0768


def _grid(nx, ny, nz, ncomp):
    return {"nx": int(nx), "ny": int(ny), "nz": int(nz), "ncomp": int(ncomp)}


def _coords(nx, ny, nz, x0=0, y0=0, z0=0, gx=None, gz=None):
    """Global node coordinates of a box, flattened [z][y][x]; x, z wrap periodically."""
    xs = np.arange(x0, x0 + nx)
    zs = np.arange(z0, z0 + nz)
    if gx is not None:
        xs = np.mod(xs, gx)
    if gz is not None:
        zs = np.mod(zs, gz)
    ys = np.arange(y0, y0 + ny)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return X.ravel().astype(np.float64), Y.ravel().astype(np.float64), Z.ravel().astype(np.float64)


def couette_profile(y, ny, U):
    """Linear plane-Couette start with walls at -U (bottom) and +U (top)."""
    gdot = 2.0 * U / ny
    return gdot * (y - (ny - 1) / 2.0)


def couette_fenep(nx=16, ny=32, nz=16, seed=0, U=0.01, tau=1.0, tau_p=1000.0, L2=100.0,
                  beta=0.2, noise=1e-3, coupling="force"):
    N = nx * ny * nz
    eta_s = (tau - 0.5) * CS2
    eta_p = eta_s * beta / (1.0 - beta)
    X, Y, Z = _coords(nx, ny, nz)
    u = np.zeros((3, N))
    u[0] = couette_profile(Y, ny, U)
    rng = np.random.default_rng(seed)
    Nm = rng.uniform(-noise, noise, size=(N, 3, 3))
    S = 0.5 * (Nm + np.transpose(Nm, (0, 2, 1)))
    C = np.zeros((6, N))
    C[0] = 1.0 + S[:, 0, 0]
    C[1] = 1.0 + S[:, 1, 1]
    C[2] = 1.0 + S[:, 2, 2]
    C[3] = S[:, 0, 1]
    C[4] = S[:, 0, 2]
    C[5] = S[:, 1, 2]
    rho = np.ones((1, N))
    return {
        "name": f"couette_fenep_{nx}x{ny}x{nz}",
        "grid": _grid(nx, ny, nz, 1),
        "params": {"tau_A": tau, "tau_B": tau, "G": 0.0, "delta": 0.1, "rho0": [1.0, 0.0],
                   "polymer_phase": "all", "eta_p": eta_p, "tau_p": tau_p, "L2": L2,
                   "coupling": coupling},
        "walls": {"u_bottom": [-U, 0.0, 0.0], "u_top": [U, 0.0, 0.0]},
        "rho": rho, "u": u, "C": C,
        "meta": {"U": U, "gdot": 2 * U / ny, "eta_s": eta_s, "Lambda": tau_p * 2 * U / ny},
    }


def droplet_fields(nx, ny, nz, R, rho_in, rho_out, U, box=None):
    """Sharp-sphere droplet + Couette start on the whole grid or on a sub-box.

    ``box`` = (x0, bx, z0, bz): a window of bx x ny x bz nodes starting at global
    (x0, 0, z0), with x and z wrapped periodically.
    """
    if box is None:
        X, Y, Z = _coords(nx, ny, nz)
    else:
        x0, bx, z0, bz = box
        X, Y, Z = _coords(bx, ny, bz, x0=x0, z0=z0, gx=nx, gz=nz)
    xc, yc, zc = (nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0
    inside = (X - xc) ** 2 + (Y - yc) ** 2 + (Z - zc) ** 2 < R * R
    M = X.size
    rho = np.empty((2, M))
    rho[0] = np.where(inside, rho_in, rho_out)
    rho[1] = np.where(inside, rho_out, rho_in)
    u = np.zeros((3, M))
    u[0] = couette_profile(Y, ny, U)
    C = np.zeros((6, M))
    C[0:3] = 1.0
    return rho, u, C


def droplet_shear(nx=128, ny=64, nz=128, R=16.0, rho_in=1.0, rho_out=0.04, G=0.9,
                  tau_A=1.0, tau_B=1.0, polymer_phase="A", L2=100.0, De=1.0, Ca=0.2,
                  concentration=0.4, sigma=None, U=None, box=None, name=None, coupling="force"):
    """Droplet-in-shear workload.  ``sigma`` (interfacial tension) sets U from Ca unless
    ``U`` is given; ``concentration`` = eta_p/(eta_s + eta_p) of the viscoelastic phase."""
    rho_tot = rho_in + rho_out
    eta_A = rho_tot * CS2 * (tau_A - 0.5)
    eta_B = rho_tot * CS2 * (tau_B - 0.5)
    eta_s_poly = eta_A if polymer_phase == "A" else eta_B
    eta_p = eta_s_poly * concentration / (1.0 - concentration) if polymer_phase != "none" else 0.0
    eta_M = eta_B + (eta_p if polymer_phase == "B" else 0.0)
    if sigma is None:
        sigma = SIGMA_AB_1_004
    if U is None:
        gdot = Ca * sigma / (R * eta_M)
        U = gdot * ny / 2.0
    tau_em = R * eta_M / sigma
    tau_p = De * tau_em * eta_M / eta_p if eta_p > 0 else 1000.0
    rho, u, C = droplet_fields(nx, ny, nz, R, rho_in, rho_out, U, box=box)
    # storage shift: initial mean density of each species over the full grid
    vol_frac = (4.0 / 3.0) * math.pi * R ** 3 / (nx * ny * nz)
    r0A = rho_out + vol_frac * (rho_in - rho_out)
    r0B = rho_in - vol_frac * (rho_in - rho_out)
    if box is None:
        r0A, r0B = float(rho[0].mean()), float(rho[1].mean())
    g = _grid(nx, ny, nz, 2) if box is None else _grid(box[1], ny, box[3], 2)
    return {
        "name": name or f"droplet_shear_{nx}x{ny}x{nz}_R{R:g}",
        "grid": g,
        "params": {"tau_A": tau_A, "tau_B": tau_B, "G": G, "delta": 0.1, "rho0": [r0A, r0B],
                   "polymer_phase": polymer_phase, "eta_p": eta_p, "tau_p": tau_p, "L2": L2,
                   "coupling": coupling},
        "walls": {"u_bottom": [-U, 0.0, 0.0], "u_top": [U, 0.0, 0.0]},
        "rho": rho, "u": u, "C": C,
        "meta": {"U": U, "gdot": 2 * U / ny, "eta_M": eta_M, "sigma": sigma, "Ca": Ca,
                 "De": De, "R": R, "global_grid": _grid(nx, ny, nz, 2)},
    }


def droplet_cfg1(De=1.0, variant="as_written", nx=128, ny=64, nz=128):
    """Two-component droplet, 128x64x128, R = 16 (2R/H = 0.5), polymer in the droplet,
    L^2 = 100.  ``as_written``: G = 0.9 (below the critical coupling 2/rho_tot, so the
    mixture is miscible); ``physics``: G at the mean-field binodal of 1.0/0.04."""
    G = 0.9 if variant == "as_written" else G_PHYSICS_1_004
    R = 16.0 * nx / 128.0 if nx != 128 else 16.0
    return droplet_shear(nx=nx, ny=ny, nz=nz, R=R, G=G, polymer_phase="A", L2=100.0, De=De,
                         Ca=0.2, name=f"droplet_cfg1_{variant}_De{De:g}_{nx}x{ny}x{nz}")


def droplet_cfg2(nx=1024, ny=256, nz=1024, box=None):
    """Large single-GPU run: 1024x256x1024, Newtonian droplet R = 64, viscoelastic matrix
    (L^2 = 400, De = 1), Ca = 0.2, G at the mean-field binodal of 1.0/0.04."""
    R = 64.0 * ny / 256.0
    return droplet_shear(nx=nx, ny=ny, nz=nz, R=R, G=G_PHYSICS_1_004, polymer_phase="B",
                         L2=400.0, De=1.0, Ca=0.2, box=box,
                         name=f"droplet_cfg2_{nx}x{ny}x{nz}")


def random_state(nx, ny, nz, ncomp, seed, amp_rho=0.05, amp_u=0.02, amp_C=0.2):
    """Smooth-free random fields for algebraic invariants (conservation, symmetry):
    rho_s = 1 + amp U(-1,1) per species, u ~ amp U(-1,1), C = I + A A^T amp/3 + small."""
    N = nx * ny * nz
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp_rho * rng.uniform(-1, 1, size=(ncomp, N))
    u = amp_u * rng.uniform(-1, 1, size=(3, N))
    A = rng.uniform(-1, 1, size=(N, 3, 3))
    S = np.einsum("nij,nkj->nik", A, A) * (amp_C / 3.0)
    C = np.zeros((6, N))
    C[0] = 1.0 + S[:, 0, 0]
    C[1] = 1.0 + S[:, 1, 1]
    C[2] = 1.0 + S[:, 2, 2]
    C[3] = S[:, 0, 1]
    C[4] = S[:, 0, 2]
    C[5] = S[:, 1, 2]
    return rho, u, C


def sweep_cases(n=64, seed=3, scale=1.0):
    """Droplet-in-shear sweep instances drawn with numpy.random.default_rng(seed):
    N_x = N_z in {64, 128, 192}, N_y in {32, 48, 64}, R ~ U{8..24} subject to 2R/H <= 0.75
    and 4R <= N_x, Ca ~ U[0.05, 0.4], De ~ logU[0.1, 2], viscosity ratio lambda ~
    logU[0.5, 2] (tau_A = 1/2 + lambda (tau_B - 1/2), tau_B = 1), L^2 in {50, 100, 400}, and
    the polymer in the droplet or the matrix by a coin flip.  ``scale`` shrinks every length
    (grid and radius) by the same factor."""
    rng = np.random.default_rng(seed)
    cases = []
    while len(cases) < n:
        nxz = int(round(int(rng.choice([64, 128, 192])) * scale))
        ny = int(round(int(rng.choice([32, 48, 64])) * scale))
        R = int(round(int(rng.integers(8, 25)) * scale))
        Ca = float(rng.uniform(0.05, 0.4))
        De = float(np.exp(rng.uniform(np.log(0.1), np.log(2.0))))
        lam = float(np.exp(rng.uniform(np.log(0.5), np.log(2.0))))
        L2 = float(rng.choice([50.0, 100.0, 400.0]))
        phase = "A" if rng.uniform() < 0.5 else "B"
        if 2 * R / ny > 0.75 or 4 * R > nxz:
            continue
        cases.append({"nx": nxz, "ny": ny, "nz": nxz, "R": float(R), "Ca": Ca, "De": De,
                      "lam": lam, "L2": L2, "polymer_phase": phase})
    return cases


def sweep_workload(case, sigma=None, G=None, tau_B=3.0, **kw):
    """Workload dict for one sweep case (see sweep_cases).  The matrix relaxation time
    tau_B = 3 keeps the wall speed of Ca up to 0.4 below 0.08 (at tau = 1 it would reach
    0.2); it corresponds to the paper's droplet viscosity 1.74 at total density 2.1."""
    tau_A = 0.5 + case["lam"] * (tau_B - 0.5)
    return droplet_shear(nx=case["nx"], ny=case["ny"], nz=case["nz"], R=case["R"],
                         G=G if G is not None else G_PHYSICS_1_004, tau_A=tau_A, tau_B=tau_B,
                         polymer_phase=case["polymer_phase"], L2=case["L2"], De=case["De"],
                         Ca=case["Ca"], sigma=sigma, name=f"sweep_{case['nx']}x{case['ny']}",
                         **kw)


def mlp_params(seed=0, scale=1.0):
    """Glorot-uniform weights and small random biases for the 5-128-128-3 surrogate,
    drawn with numpy.random.default_rng(seed), in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for fo, fi in ((128, 5), (128, 128), (3, 128)):
        a = math.sqrt(6.0 / (fo + fi)) * scale
        parts.append(rng.uniform(-a, a, size=fo * fi))
        parts.append(rng.uniform(-0.1, 0.1, size=fo))
    return np.concatenate(parts)


def mlp_batch(n, seed=0):
    """Standard-normal inputs (n, 5) and targets (n, 3) from a smooth function of them."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, 5))
    T = np.stack([np.tanh(X[:, 0] + 0.5 * X[:, 1]), np.sin(X[:, 2]) * X[:, 3], 0.3 * X[:, 4] ** 2 - 0.3], 1)
    return X, T
