"""Pins of the oracle's multiple-relaxation-time collision (Sec. 2: moments through an
orthogonal transformation, bulk and shear modes relaxed with tau_s = tau_b, species
momenta with tau_M = 1, the other modes with rate 1; eq. TRANSPORTCOEFF).

The basis is pinned by orthogonality and span, the collision by its moments (what each
mode does in one collision), and the whole scheme by the transport coefficients the paper
states: the shear viscosity c_s^2 (tau_s - 1/2) of a decaying shear wave and the mutual
diffusivity c_s^2 (tau_M - 1/2) = 1/6 of a two-component interdiffusion mode, independent
of tau_s (with BGK the same mode gives c_s^2 (tau - 1/2))."""
import math

import numpy as np
import pytest

import oracle

def velocities():
    c, w, _ = oracle.lattice()
    return np.asarray(c, dtype=np.float64), np.asarray(w, dtype=np.float64)


def test_basis_is_orthogonal_and_holds_the_hydrodynamic_moments():
    """19 mutually orthogonal rows (plain sum over the velocities); rows 0, 3, 5, 7 are 1
    and c; the rows relaxed at the shear rate (1, 9, 11, 13, 14, 15) together with row 0
    span exactly the second-order polynomials {1, c_i c_j}."""
    M = oracle.mrt_basis()
    c, _ = velocities()
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-12)
    assert np.linalg.matrix_rank(M) == 19
    assert np.array_equal(M[0], np.ones(19))
    for row, d in ((3, 0), (5, 1), (7, 2)):
        assert np.array_equal(M[row], c[:, d])
    quad = np.stack([np.ones(19)] + [c[:, i] * c[:, j] for i in range(3) for j in range(i, 3)])
    sub = M[[0, 1, 9, 11, 13, 14, 15]]
    assert np.linalg.matrix_rank(sub) == 7 and np.linalg.matrix_rank(np.vstack([sub, quad])) == 7


def node_state(seed=3):
    rng = np.random.default_rng(seed)
    rho, u = 1.07, np.array([0.03, -0.02, 0.015])
    f = oracle.equilibrium(rho, u) + rng.uniform(-2e-3, 2e-3, 19)
    f += (rho - f.sum()) / 19.0  # keep sum f = rho
    return f, rho, u


def test_unit_rates_reduce_to_bgk():
    """With tau = 1 every mode relaxes with rate 1, which is BGK at tau = 1 (the paper's
    remark that MRT and BGK coincide at unit rates, our reading Q1)."""
    f, rho, u = node_state()
    F = np.array([2e-4, -1e-4, 3e-4])
    a = oracle.collide_node(f, rho, u, F, 1.0, collision="mrt")
    b = oracle.collide_node(f, rho, u, F, 1.0)
    assert np.max(np.abs(a - b)) < 1e-15


@pytest.mark.parametrize("tau", [0.7, 1.6])
def test_each_mode_relaxes_at_its_rate(tau):
    """Unforced: mass kept; species momentum relaxed fully to rho u (tau_M = 1); the
    second-moment tensor's departure from equilibrium scaled by 1 - 1/tau; the third-order
    (q) and higher non-hydrodynamic moments fully relaxed.  Forced: the momentum after
    collision is rho u + F/2."""
    f, rho, u = node_state(7)
    c, _ = velocities()
    E = oracle.equilibrium(rho, u)
    out = oracle.collide_node(f, rho, u, np.zeros(3), tau, collision="mrt")
    assert abs(out.sum() - rho) < 1e-15
    assert np.allclose(c.T @ out, rho * u, atol=1e-15)
    for i in range(3):
        for j in range(i, 3):
            w = c[:, i] * c[:, j]
            assert abs(w @ (out - E) - (1 - 1 / tau) * (w @ (f - E))) < 1e-15
    M = oracle.mrt_basis()
    for row in (2, 4, 6, 8, 10, 12, 16, 17, 18):
        assert abs(M[row] @ (out - E)) < 1e-15
    F = np.array([2e-4, -1e-4, 3e-4])
    outF = oracle.collide_node(f, rho, u, F, tau, collision="mrt")
    assert np.allclose(c.T @ outF, rho * u + 0.5 * F, atol=1e-15)


def decay_rate(tau, collision, kind, nz=64, ny=96, t1=100, t2=300, amp=1e-3):
    """Decay rate / k^2 of a sine mode along z, read at the centre row y = ny/2 where the
    wall boundary layers (width ~ sqrt(nu t) << ny/2) have not arrived: a shear wave u_x(z)
    (one component) or an interdiffusion mode rho_A - rho_B (two components, G = 0)."""
    nx, N = 1, ny * nz
    Z, Y, _ = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    Z, Y = Z.ravel(), Y.ravel()
    k = 2 * math.pi / nz
    nc = 1 if kind == "shear" else 2
    o = oracle.Oracle(nx, ny, nz, nc)
    o.set_params(tau_A=tau, tau_B=tau, G=0.0, collision=collision)
    o.set_walls([0, 0, 0], [0, 0, 0])
    Cf = np.zeros((6, N))
    Cf[:3] = 1.0
    if kind == "shear":
        u = np.zeros((3, N))
        u[0] = amp * np.sin(k * Z)
        o.set_fields(np.ones((1, N)), u, Cf)
    else:
        o.set_fields(np.stack([0.5 + amp * np.sin(k * Z), 0.5 - amp * np.sin(k * Z)]), np.zeros((3, N)), Cf)
    row = Y == ny // 2

    def mode():
        r, uu, _ = o.get_fields()
        q = uu[0] if kind == "shear" else r[0] - r[1]
        return 2.0 / nz * np.sum(q[row] * np.sin(k * Z[row]))

    assert o.step(t1) == 0
    a1 = mode()
    assert o.step(t2 - t1) == 0
    a2 = mode()
    return -math.log(a2 / a1) / (k * k * (t2 - t1))


@pytest.mark.parametrize("tau", [0.8, 1.3])
def test_shear_viscosity_and_mobility_match_transport_coefficients(tau):
    """eq. TRANSPORTCOEFF: nu = c_s^2 (tau_s - 1/2) from the shear wave; the interdiffusion
    mode decays with c_s^2 (tau_M - 1/2) = 1/6 whatever tau_s is (BGK gives
    c_s^2 (tau - 1/2) for the same mode, a 40-60 % difference at these tau).  Lattice
    corrections at k = 2 pi / 64 are below 0.3 %."""
    nu = decay_rate(tau, "mrt", "shear")
    assert abs(nu - (tau - 0.5) / 3) < 3e-3 * (tau - 0.5) / 3
    D = decay_rate(tau, "mrt", "diff")
    assert abs(D - 1.0 / 6.0) < 3e-3 / 6.0
    Dbgk = decay_rate(tau, "bgk", "diff")
    assert abs(Dbgk - (tau - 0.5) / 3) < 3e-3 * (tau - 0.5) / 3
