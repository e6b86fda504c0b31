"""Pins of the oracle's second FENE-P integrator, the paper's own (Sec. 2, paragraph on the
FENE-P solver): sigma_P = f C evolved through its Cholesky factor L with ln l_ii,
second-order central differences in space, an artificial diffusivity, second-order
Adams-Bashforth in time.

Pinned: the node update (no rate leaves C unchanged; it is consistent to first order in
one step; whatever the rate, the result is SPD with tr C < L^2, where forward Euler is
not), the closed forms of Sec. 3 reached through it (uniaxial elongation on both branches,
steady shear on the full kinematic lattice), its second-order accuracy in time (SAOS
against the Oldroyd-B moduli to O(omega^2)) and in space (a translated bump converges
four-fold per halving of the spacing)."""
import math

import numpy as np
import pytest

import oracle
from paper_closed_forms import elongation_rate, saos_moduli, steady_shear_conformation


def sym6(M):
    return np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


def mat(c):
    return np.array([[c[0], c[3], c[4]], [c[3], c[1], c[5]], [c[4], c[5], c[2]]])


def model_rate(c, G, tau, L2):
    """dC/dt of eq. FENE for a uniform field: G^T C + C G - (f C - I)/tau_P."""
    C = mat(c)
    f = (L2 - 3) / (L2 - np.trace(C))
    return sym6(G.T @ C + C @ G - (f * C - np.eye(3)) / tau)


def run_0d(G_of, tau, L2, n):
    """Homogeneous (0-D) run through the oracle's node update."""
    c, yp, hist = np.array([1, 1, 1, 0, 0, 0.0]), None, []
    for k in range(n):
        c, yp, flag = oracle.cholesky_ab2(L2, c, model_rate(c, G_of(k), tau, L2), yp)
        assert flag == 0, k
        hist.append(c)
    return c, hist


def spd(c):
    C = mat(c)
    return C[0, 0] > 0 and np.linalg.det(C[:2, :2]) > 0 and np.linalg.det(C) > 0


def test_node_update_is_consistent_and_keeps_spd():
    rng = np.random.default_rng(11)
    L2 = 50.0
    for _ in range(20):
        Q = np.linalg.qr(rng.normal(size=(3, 3)))[0]
        C = Q @ np.diag(rng.uniform(0.2, 8.0, 3)) @ Q.T
        c = sym6(C)
        cn, _, flag = oracle.cholesky_ab2(L2, c, np.zeros(6))
        assert flag == 0 and np.max(np.abs(cn - c)) < 1e-13 * np.max(np.abs(c))
        R = sym6(rng.normal(size=(3, 3)) + rng.normal(size=(3, 3)).T)
        for eps in (1e-5, 1e-6):
            cn, _, flag = oracle.cholesky_ab2(L2, c, eps * R)
            assert flag == 0
            assert np.max(np.abs(cn - c - eps * R)) < 200 * eps * eps * np.max(np.abs(R))
        # a rate of order one per step, too large for an explicit step on C: still SPD
        # with tr C < L^2 (rates that squeeze an eigenvalue below 1e-12 of the largest
        # are SPD in exact arithmetic but not after rounding)
        cn, _, flag = oracle.cholesky_ab2(L2, c, 3.0 * R)
        assert flag == 0 and spd(cn) and cn[:3].sum() < L2
    # where forward Euler loses positive definiteness (strong compression along x)
    ed = 1.2
    G = np.diag([-ed, 0.0, ed])
    c = np.array([1, 1, 1, 0, 0, 0.0])
    R = model_rate(c, G, 50.0, 100.0)
    assert not spd(c + R)
    cn, _, flag = oracle.cholesky_ab2(100.0, c, R)
    assert flag == 0 and spd(cn) and cn[:3].sum() < 100.0


@pytest.mark.parametrize("Lam_e", [0.05, 0.4, 0.9, 1.5])
def test_uniaxial_elongation_through_the_cholesky_scheme(Lam_e):
    """Steady state of the homogeneous update = the closed form of eqs. el8, el9, on the
    branch that D = sigma_zz - sigma_xx selects (L^2 = 100)."""
    L2, tau = 100.0, 50.0
    ed = Lam_e / tau
    G = np.diag([-0.5 * ed, -0.5 * ed, ed])
    c, _ = run_0d(lambda k: G, tau, L2, int(100 * tau))
    f = (L2 - 3) / (L2 - c[:3].sum())
    D = f * (c[2] - c[0])
    assert abs(elongation_rate(D, L2, "+" if D < L2 - 3 else "-") - Lam_e) < 1e-9 * max(Lam_e, 1)


@pytest.mark.parametrize("wt", [0.5, 2.0, 8.0])
def test_saos_is_second_order_accurate(wt):
    """SAOS in the Oldroyd-B limit: the fitted moduli match eq. modulipred to
    O(omega^2 + 1/tau_P^2), far inside the O(omega + 1/tau_P) error of forward Euler."""
    tau, g0 = 2000.0, 0.01
    w = wt / tau

    def G_of(k):
        G = np.zeros((3, 3))
        G[1, 0] = g0 * w * math.cos(w * k)
        return G

    n0 = int(14 * tau)
    n1 = n0 + int(3 * 2 * math.pi / w)
    _, hist = run_0d(G_of, tau, 1e8, n1)
    ts = np.arange(n0, n1) + 1.0
    xs = np.array([h[3] for h in hist[n0:n1]])
    (a, b), *_ = np.linalg.lstsq(np.stack([np.sin(w * ts), np.cos(w * ts)], 1), xs, rcond=None)
    Gp, Gpp = saos_moduli(wt)
    tol = 2.0 * (w * w + 1.0 / tau ** 2) * (Gp + Gpp) + 1e-7
    assert abs(a / g0 - Gp) < tol and abs(b / g0 - Gpp) < tol
    assert tol < 0.05 * (w + 1.0 / tau) * (Gp + Gpp)  # the bound is beyond first order


@pytest.mark.parametrize("Lam,L2,tau_p", [(0.625, 100.0, 1000.0), (2.5, 100.0, 200.0)])
def test_kinematic_steady_shear_on_the_lattice(Lam, L2, tau_p):
    """Prescribed shear u_x = gdot (y - 1) on a 3x3x3 lattice run by the oracle's stepping
    with the Cholesky scheme: the centre node reaches the closed form of Sec. 3.1 (its
    central advection term vanishes with u), with C_yy = C_zz."""
    gd = Lam / tau_p
    n = 3
    Z, Y, X = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    Y = Y.ravel() - 1.0
    centre = int(np.argmax((X.ravel() == 1) & (Y == 0) & (Z.ravel() == 1)))
    o = oracle.Oracle(n, n, n, 1)
    o.set_params(polymer_phase="none", eta_p=0.0, tau_p=tau_p, L2=L2, fene="cholesky_ab2")
    o.set_walls([-gd * 1.5, 0, 0], [gd * 1.5, 0, 0])
    C = np.zeros((6, Y.size))
    C[:3] = 1.0
    u = np.stack([gd * Y, 0 * Y, 0 * Y])
    o.set_fields(np.ones((1, Y.size)), u, C)
    assert o.fenep_kinematic(u, int(30 * tau_p)) == 0
    Cc = o.get_C()[:, centre]
    ref = steady_shear_conformation(Lam, L2)
    for k, key in enumerate(("xx", "yy", "zz", "xy")):
        assert abs(Cc[k] - ref[key]) < 1e-9 * max(1.0, abs(ref[key])), key
    assert abs(Cc[1] - Cc[2]) < 1e-12


def test_central_advection_converges_at_second_order():
    """A bump in C_xx, C_xy carried by a uniform u_x = 0.1 (no stretching, no relaxation):
    halving the spacing (bump width 4 -> 8 cells, 200 -> 400 steps) cuts the error of the
    translated profile four-fold (first-order upwind would halve it)."""
    def err(nx, width, steps, u=0.1):
        o = oracle.Oracle(nx, 3, 1, 1)
        o.set_params(polymer_phase="none", tau_p=1e300, L2=1e300, fene="cholesky_ab2")
        o.set_walls([u, 0, 0], [u, 0, 0])
        X = np.tile(np.arange(nx), 3).astype(float)
        uu = np.zeros((3, X.size))
        uu[0] = u
        C = np.zeros((6, X.size))
        C[:3] = 1.0

        def bump(x):
            return np.exp(-0.5 * (x / width) ** 2)

        C[0] += 0.5 * bump(X - nx / 2)
        C[3] = 0.2 * bump(X - nx / 2)
        o.set_fields(np.ones((1, X.size)), uu, C)
        assert o.fenep_kinematic(uu, steps) == 0
        Cn = o.get_C()
        d = X - nx / 2 - u * steps
        return np.sqrt(np.mean((Cn[0] - 1 - 0.5 * bump(d)) ** 2))

    r = err(80, 4.0, 200) / err(160, 8.0, 400)
    assert 3.5 < r < 4.5
