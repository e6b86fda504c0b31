"""FENE-P pins of the oracle: the paper's closed forms for steady shear (Sec. 3.1), the
Oldroyd-B limit, shear thinning, zero second normal-stress difference, positivity and
extensibility, and stress relaxation after cessation of shear (Sec. 3.4)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads
from paper_closed_forms import (cessation_S_ratio, elongation_rate, lindner_N, lindner_S, saos_moduli,
                                steady_shear_conformation)

KEYS = ("xx", "yy", "zz", "xy", "xz", "yz")


def couette(ny, U, tau_p, L2, eta_p, nx=2, nz=2, coupling="force"):
    wl = workloads.couette_fenep(nx=nx, ny=ny, nz=nz, U=U, tau_p=tau_p, L2=L2, noise=0.0,
                                 coupling=coupling)
    wl["params"]["eta_p"] = eta_p
    return oracle.from_workload(wl), wl


@pytest.mark.parametrize("Lam,L2,tau_p,coupling", [(0.625, 100.0, 1000.0, "force"), (2.5, 100.0, 200.0, "force"),
                                                   (0.625, 1e8, 200.0, "force"), (2.5, 100.0, 200.0, "stress")])
def test_steady_shear_matches_lindner(Lam, L2, tau_p, coupling):
    """Full LB+FD run of plane Couette with feedback on; after 20 polymer times the
    conformation tensor equals the closed-form steady shear solution C = sigma_P/Z
    (eqs. EQNS, N2S, cubic, lindner, lindner2), with the stress acting as a body force or
    through the equilibrium (eq. MODEtransformation): a uniform stress moves no fluid."""
    ny = 16
    gdot = Lam / tau_p
    U = gdot * ny / 2.0
    o, wl = couette(ny, U, tau_p, L2, eta_p=1.0 / 24.0, coupling=coupling)
    assert o.step(int(20 * tau_p)) == 0
    _, u, C = o.get_fields()
    ref = steady_shear_conformation(Lam, L2)
    for k, key in enumerate(KEYS):
        assert np.allclose(C[k], ref[key], rtol=2e-6, atol=2e-8), key
    # zero second normal-stress difference: C_yy = C_zz, no out-of-plane shear
    assert np.allclose(C[1], C[2], rtol=0, atol=1e-12)
    assert np.max(np.abs(C[4:])) < 1e-12
    # sigma_P = f C recovers S and N directly
    tr = C[0] + C[1] + C[2]
    f = (L2 - 3) / (L2 - tr)
    assert np.allclose(f * C[3], lindner_S(Lam, L2), rtol=2e-6)
    assert np.allclose(f * C[0] - 1, lindner_N(Lam, L2), rtol=5e-6)
    if L2 > 1e6:  # Oldroyd-B limit: S = Lambda, N = 2 Lambda^2
        assert abs(f[0] * C[3, 0] - Lam) < 1e-6 * Lam
        assert abs(f[0] * C[0, 0] - 1 - 2 * Lam ** 2) < 1e-6 * Lam ** 2
    # the flow stays the linear Couette profile (uniform stress exerts no force)
    Y = np.repeat(np.arange(ny), 2)[None, :].repeat(2, 0).ravel()
    assert np.allclose(u[0], -U + 2 * U * (Y + 0.5) / ny, atol=1e-12)


def test_shear_thinning():
    """S/Lambda < 1 and decreasing in Lambda at finite L^2 (Sec. 3.1, end)."""
    r1 = lindner_S(0.625, 100.0) / 0.625
    r2 = lindner_S(2.5, 100.0) / 2.5
    assert r2 < r1 < 1.0
    assert abs(r1 - 0.99237) < 1e-5


def zero_d_recurrence(C6, gdot, tau_p, L2, n):
    """Uniform fields: advection and the stress divergence vanish and S10 reduces to
    C <- C + G^T C + C G - (f C - I)/tau_p with G_yx = gdot (u_x = gdot y)."""
    Cm = np.array([[C6[0], C6[3], C6[4]], [C6[3], C6[1], C6[5]], [C6[4], C6[5], C6[2]]])
    G = np.zeros((3, 3))
    G[1, 0] = gdot
    I = np.eye(3)
    for _ in range(n):
        f = (L2 - 3) / (L2 - np.trace(Cm))
        Cm = Cm + (G.T @ Cm + Cm @ G) - (f * Cm - I) / tau_p
    return np.array([Cm[0, 0], Cm[1, 1], Cm[2, 2], Cm[0, 1], Cm[0, 2], Cm[1, 2]])


def test_couette_fenep_workload_tracks_zero_d_recurrence():
    """The 16x32x16 FENE-P Couette workload (noise +-1e-3 on C) after 4000 steps: the
    node-average of C follows the uniform-field recurrence to noise level, the flow is
    the Couette profile, and C stays SPD with tr C < L^2."""
    wl = workloads.couette_fenep()
    o = oracle.from_workload(wl)
    C0 = wl["C"].mean(1)
    assert o.step(4000) == 0
    _, u, C = o.get_fields()
    p = wl["params"]
    ref = zero_d_recurrence(C0, wl["meta"]["gdot"], p["tau_p"], p["L2"], 4000)
    Cm = C.mean(1)
    dev = ref - np.array([1, 1, 1, 0, 0, 0])
    assert np.max(np.abs(Cm - ref)) < 1e-5 * np.max(np.abs(dev))
    d = o.diagnostics()
    assert d["min_minor"] > 0.9 and d["min_L2_minus_trC"] > 90
    # the 4000-step state is still short of the steady closed form (startup, 4 tau_p)
    S_ss = steady_shear_conformation(wl["meta"]["Lambda"], p["L2"])["xy"]
    assert Cm[3] < 0.99 * S_ss


def test_cessation_relaxation_follows_closed_forms():
    """Inception of shear at L^2 = 4.1 to steady state, then the flow is stopped: the
    trace excess T = tr sigma_P - 3 follows dT/d(t/tau_p) = T (L^2+T)^2/(L^2 (3-L^2))
    (eq. timeunclosed) and S/S0 follows eq. relax (Sec. 3.4).  Prescribed velocity,
    no feedback, as in the paper's benchmark."""
    nx, ny, nz = 1, 3, 1
    L2, tau_p, Lam = 4.1, 20000.0, 10.0
    gdot = Lam / tau_p
    U = gdot * ny / 2
    o = oracle.Oracle(nx, ny, nz, 1)
    o.set_params(polymer_phase="none", eta_p=0.0, tau_p=tau_p, L2=L2)
    o.set_walls([-U, 0, 0], [U, 0, 0])
    N = nx * ny * nz
    u = np.zeros((3, N))
    u[0] = gdot * (np.arange(ny) - (ny - 1) / 2)
    C = np.zeros((6, N))
    C[:3] = 1.0
    o.set_fields(np.ones((1, N)), u, C)
    assert o.fenep_kinematic(u, int(15 * tau_p)) == 0
    C = o.get_C()
    ref = steady_shear_conformation(Lam, L2)
    assert abs(C[3, 1] - ref["xy"]) < 1e-6 * ref["xy"]
    assert abs(C[0, 1] - ref["xx"]) < 1e-6 * ref["xx"]

    def sig(Cv):
        f = (L2 - 3) / (L2 - Cv[:3].sum())
        return f * (Cv[:3].sum()) - 3.0, f * Cv[3]

    T0, S0 = sig(C[:, 1])
    o.set_walls([0, 0, 0], [0, 0, 0])
    u0 = np.zeros((3, N))
    times, Ts, Ss = [], [], []
    for k in range(8):
        assert o.fenep_kinematic(u0, int(tau_p / 4)) == 0
        T, S = sig(o.get_C()[:, 1])
        times.append((k + 1) / 4.0)
        Ts.append(T)
        Ss.append(S)
    sol = solve_ivp(lambda t, T: T * (L2 + T) ** 2 / (L2 * (3 - L2)), (0, times[-1]), [T0],
                    t_eval=times, rtol=1e-11, atol=1e-13)
    # forward Euler with dt = 1: first-order error ~ rate*dt/2 with the initial decay rate
    # (L^2 + T0)^2 / (L^2 (L^2 - 3)) / tau_p ~ 3.4e-3 per step here
    assert np.allclose(Ts, sol.y[0], rtol=4e-3)
    pred = [S0 * cessation_S_ratio(T, T0, L2) for T in Ts]
    assert np.allclose(Ss, pred, rtol=4e-3)
    # relaxation of a FENE-P dumbbell is faster than the Oldroyd-B exponential at early times
    assert Ts[0] < T0 * math.exp(-0.25)


def centre_probe(u_of_xyz, tau_p, L2):
    """3x3x3 lattice in kinematic mode with a velocity field that vanishes at the centre node:
    there the upwind advection term is u . grad C = 0 exactly and the central differences of
    a linear field give its gradient exactly, so the centre follows the homogeneous FENE-P
    update (eq. FENE with uniform G) whatever the other nodes do."""
    n = 3
    Z, Y, X = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    X, Y, Z = X.ravel() - 1.0, Y.ravel() - 1.0, Z.ravel() - 1.0
    centre = int(np.argmax((X == 0) & (Y == 0) & (Z == 0)))
    o = oracle.Oracle(n, n, n, 1)
    o.set_params(polymer_phase="none", eta_p=0.0, tau_p=tau_p, L2=L2)
    o.set_walls([0, 0, 0], [0, 0, 0])
    C = np.zeros((6, X.size))
    C[:3] = 1.0
    u = u_of_xyz(X, Y, Z)
    o.set_fields(np.ones((1, X.size)), u, C)
    return o, centre, (X, Y, Z)


@pytest.mark.parametrize("Lam_e", [0.05, 0.4, 0.9, 1.5])
def test_uniaxial_elongation_matches_closed_form(Lam_e):
    """Steady uniaxial elongation u = edot (-x/2, -y/2, z) (Sec. 3.2): the stress difference
    D = sigma_zz - sigma_xx of the steady state satisfies the closed form of eqs. el8, el9,
    on the '+' branch below D = L^2 - 3 and on the '-' branch above it (here L^2 = 100, so
    Lambda_e = 0.9 and 1.5 lie on either side of the double root at Lambda_e = 0.97)."""
    L2, tau_p = 100.0, 50.0
    ed = Lam_e / tau_p

    def u_of(X, Y, Z):
        return np.stack([-0.5 * ed * X, -0.5 * ed * Y, ed * Z])

    o, c, (X, Y, Z) = centre_probe(u_of, tau_p, L2)
    assert o.fenep_kinematic(u_of(X, Y, Z), int(100 * tau_p)) == 0
    Cc = o.get_C()[:, c]
    f = (L2 - 3) / (L2 - Cc[:3].sum())
    D = f * (Cc[2] - Cc[0])
    branch = "+" if D < L2 - 3 else "-"
    assert (branch == "+") == (Lam_e < 0.97)
    assert abs(elongation_rate(D, L2, branch) - Lam_e) < 1e-6 * Lam_e
    # axisymmetry: C_xx = C_yy, no off-diagonal part
    assert abs(Cc[0] - Cc[1]) < 1e-12 and np.max(np.abs(Cc[3:])) < 1e-14


def test_elongational_viscosity_tends_to_three_at_small_rates():
    """Trouton limit (Sec. 3.2): eta_e / eta_P = D / Lambda_e -> 3 as Lambda_e -> 0."""
    L2, tau_p, Lam_e = 100.0, 50.0, 0.002
    ed = Lam_e / tau_p

    def u_of(X, Y, Z):
        return np.stack([-0.5 * ed * X, -0.5 * ed * Y, ed * Z])

    o, c, xyz = centre_probe(u_of, tau_p, L2)
    assert o.fenep_kinematic(u_of(*xyz), int(40 * tau_p)) == 0
    Cc = o.get_C()[:, c]
    f = (L2 - 3) / (L2 - Cc[:3].sum())
    assert abs(f * (Cc[2] - Cc[0]) / Lam_e - 3.0) < 0.01


@pytest.mark.parametrize("wt", [0.5, 2.0, 8.0])
def test_small_amplitude_oscillatory_shear_moduli(wt):
    """SAOS (Sec. 3.3): prescribed u_x = gamma0 omega cos(omega t) y in the Oldroyd-B limit
    (L^2 = 1e8).  After the transient, the shear conformation C_xy (= sigma_xy divided by
    eta_P/tau_P) oscillates as gamma0 (G' sin + G'' cos) with the moduli of eq. modulipred,
    up to the first-order error of the explicit update (relative O(omega + 1/tau_P)).  The
    same fit matches the exact periodic solution of that update,
    x_{n+1} = (1 - 1/tau_P) x_n + gamma0 omega cos(omega n), to the decayed transient."""
    tau_p, g0 = 2000.0, 0.01
    w = wt / tau_p

    def u_of(X, Y, Z, k=0):
        return np.stack([g0 * w * math.cos(w * k) * Y, 0 * Y, 0 * Y])

    o, c, xyz = centre_probe(u_of, tau_p, 1e8)
    n0 = int(14 * tau_p)
    n1 = n0 + int(3 * 2 * math.pi / w)
    ts, xs = [], []
    for k in range(n1):
        assert o.fenep_kinematic(u_of(*xyz, k=k), 1) == 0
        if k >= n0:
            Cc = o.get_C()[:, c]
            xs.append(Cc[3])
            ts.append(k + 1)
    ts = np.array(ts, dtype=np.float64)
    A = np.stack([np.sin(w * ts), np.cos(w * ts)], 1)
    (a, b), *_ = np.linalg.lstsq(A, np.array(xs), rcond=None)
    Gp, Gpp = saos_moduli(wt)
    err = 2.0 * (w + 1.0 / tau_p) * (Gp + Gpp)
    assert abs(a / g0 - Gp) < err and abs(b / g0 - Gpp) < err
    Z = g0 * w / (np.exp(1j * w) - (1.0 - 1.0 / tau_p))  # x_n = Re(Z e^{i w n})
    assert abs(a / g0 - (-Z.imag / g0)) < 1e-5 and abs(b / g0 - Z.real / g0) < 1e-5
    # no normal stress in y, z at first order; C_yy = C_zz = 1 exactly in simple shear
    Cc = o.get_C()[:, c]
    assert abs(Cc[1] - 1.0) < 1e-12 and abs(Cc[2] - 1.0) < 1e-12
