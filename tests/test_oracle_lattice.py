"""Pins of the oracle's single-node formulas against textbook lattice identities and
the closed-form moments the paper's equilibrium and source must have (Sec. 2)."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_d3q19_weights_match_paper():
    c, w, opp = oracle.lattice()
    w0, w1, w2 = GOLD["d3q19_weights"]["value"]
    speed2 = (c ** 2).sum(1)
    assert np.allclose(w[speed2 == 0], w0, rtol=0, atol=1e-16)
    assert np.allclose(w[speed2 == 1], w1, rtol=0, atol=1e-16)
    assert np.allclose(w[speed2 == 2], w2, rtol=0, atol=1e-16)
    assert (speed2 == 1).sum() == 6 and (speed2 == 2).sum() == 12
    # the 19 velocities are distinct and opposite map is an involution with c_opp = -c
    assert len({tuple(v) for v in c}) == 19
    assert np.array_equal(c[opp], -c)
    assert np.array_equal(opp[opp], np.arange(19))


def test_lattice_isotropy():
    c, w, _ = oracle.lattice()
    cs2 = GOLD["cs2"]["value"]
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.allclose((w[:, None] * c).sum(0), 0, atol=1e-16)
    M2 = np.einsum("a,ai,aj->ij", w, c, c)
    assert np.allclose(M2, cs2 * np.eye(3), atol=1e-15)
    M3 = np.einsum("a,ai,aj,ak->ijk", w, c, c, c)
    assert np.allclose(M3, 0, atol=1e-16)
    M4 = np.einsum("a,ai,aj,ak,al->ijkl", w, c, c, c, c)
    d = np.eye(3)
    iso = (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d)
           + np.einsum("il,jk->ijkl", d, d)) * cs2 ** 2
    assert np.allclose(M4, iso, atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    """Sum E = rho, sum c E = rho u, sum c c E = rho (u u + c_s^2 I)."""
    c, w, _ = oracle.lattice()
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.02, 2.5)
    u = rng.uniform(-0.1, 0.1, 3)
    E = oracle.equilibrium(rho, u)
    assert abs(E.sum() - rho) < 1e-14 * rho
    assert np.allclose(E @ c, rho * u, atol=1e-15)
    P = np.einsum("a,ai,aj->ij", E, c, c)
    assert np.allclose(P, rho * (np.outer(u, u) + np.eye(3) / 3.0), atol=1e-14)
    # at rest it reduces to w rho
    assert np.allclose(oracle.equilibrium(rho, np.zeros(3)), w * rho, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_with_stress_moments(seed):
    """Stress coupling (Sec. 2, eq. MODEtransformation): the equilibrium keeps rho and
    rho u and its second moment is lowered by exactly the given symmetric tensor T_s."""
    c, _, _ = oracle.lattice()
    rng = np.random.default_rng(200 + seed)
    rho = rng.uniform(0.02, 2.5)
    u = rng.uniform(-0.1, 0.1, 3)
    A = rng.uniform(-1e-2, 1e-2, (3, 3))
    T = A + A.T
    Ts = np.array([T[0, 0], T[1, 1], T[2, 2], T[0, 1], T[0, 2], T[1, 2]])
    E = oracle.equilibrium_stress(rho, u, Ts)
    assert abs(E.sum() - rho) < 1e-14 * rho
    assert np.allclose(E @ c, rho * u, atol=1e-15)
    P = np.einsum("a,ai,aj->ij", E, c, c)
    assert np.allclose(P, rho * (np.outer(u, u) + np.eye(3) / 3.0) - T, atol=1e-14)
    # an isotropic stress shifts only the pressure: P = rho (uu + I/3) - t I
    E = oracle.equilibrium_stress(rho, u, [0.01, 0.01, 0.01, 0, 0, 0])
    P = np.einsum("a,ai,aj->ij", E, c, c)
    assert np.allclose(P, rho * (np.outer(u, u) + np.eye(3) / 3.0) - 0.01 * np.eye(3), atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_source_moments(seed):
    """Sum S = 0, sum c S = F, sum c c S = u F + F u (second-order forcing)."""
    c, _, _ = oracle.lattice()
    rng = np.random.default_rng(100 + seed)
    u = rng.uniform(-0.1, 0.1, 3)
    F = rng.uniform(-1e-3, 1e-3, 3)
    S = oracle.source(u, F)
    assert abs(S.sum()) < 1e-18
    assert np.allclose(S @ c, F, atol=1e-18)
    P = np.einsum("a,ai,aj->ij", S, c, c)
    assert np.allclose(P, np.outer(u, F) + np.outer(F, u), atol=1e-18)


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_collision_moments(tau):
    """BGK collision with the half-force velocity conserves mass and adds F to the
    momentum: with u = (j + F/2)/rho, sum c f* = j + F."""
    c, _, _ = oracle.lattice()
    rng = np.random.default_rng(7)
    rho = 1.3
    u_bare = rng.uniform(-0.05, 0.05, 3)
    f = oracle.equilibrium(rho, u_bare) + rng.uniform(-1e-3, 1e-3, 19) * 0.01
    f -= (f.sum() - rho) / 19.0  # keep density rho
    j = f @ c
    F = rng.uniform(-1e-3, 1e-3, 3)
    u = (j + 0.5 * F) / rho
    post = oracle.collide_node(f, rho, u, F, tau)
    assert abs(post.sum() - rho) < 1e-14
    assert np.allclose(post @ c, j + F, atol=1e-15)
    # the non-conserved second moment relaxes by 1/tau towards equilibrium (+ forcing)
    Pf = np.einsum("a,ai,aj->ij", f, c, c)
    Pe = rho * (np.outer(u, u) + np.eye(3) / 3.0)
    Ps = np.outer(u, F) + np.outer(F, u)
    Pp = np.einsum("a,ai,aj->ij", post, c, c)
    assert np.allclose(Pp, Pf - (Pf - Pe) / tau + (1 - 0.5 / tau) * Ps, atol=1e-14)
