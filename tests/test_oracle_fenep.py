"""FENE-P pins of the oracle: the paper's closed forms for steady shear (Sec. 3.1), the
Oldroyd-B limit, shear thinning, zero second normal-stress difference, positivity and
extensibility, and stress relaxation after cessation of shear (Sec. 3.4)."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads
from paper_closed_forms import cessation_S_ratio, lindner_N, lindner_S, steady_shear_conformation

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
