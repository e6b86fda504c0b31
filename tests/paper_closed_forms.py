"""Closed-form results printed in arXiv:1406.2686, written out for use as pins.

These are the paper's analytic predictions, independent of any stepping scheme.
"""
import math

import numpy as np


def lindner_S(Lam, L2):
    """Steady-shear polymer shear stress S = sigma_P,xy (Sec. 3.1, eq. lindner)."""
    a = math.sqrt(L2 / 6.0)
    return 2.0 * a * math.sinh(math.asinh(Lam * L2 / 4.0 * (L2 / 6.0) ** -1.5) / 3.0)


def lindner_N(Lam, L2):
    """Steady-shear first normal-stress difference N = sigma_P,xx - 1 (Sec. 3.1, eq. lindner2)."""
    a = L2 / 6.0
    return 8.0 * a * math.sinh(math.asinh(Lam * L2 / 4.0 * a ** -1.5) / 3.0) ** 2


def steady_shear_conformation(Lam, L2):
    """Conformation tensor of steady homogeneous shear u_x = gdot y.

    sigma_P has xx = 1 + N, xy = S, yy = zz = 1 (Sec. 3.1, eqs. EQNS, N2S) and
    C = sigma_P / Z with Z = (L^2 - 3 + tr sigma_P)/L^2 (Sec. 3, FENErevised)."""
    S = lindner_S(Lam, L2)
    N = lindner_N(Lam, L2)
    Z = (L2 - 3.0 + (3.0 + N)) / L2
    return {"xx": (1 + N) / Z, "yy": 1.0 / Z, "zz": 1.0 / Z, "xy": S / Z, "xz": 0.0, "yz": 0.0,
            "S": S, "N": N, "Z": Z}


def elongation_rate(D, L2, branch):
    """Dimensionless elongation rate Lambda_e for a given D = sigma_zz - sigma_xx
    (Sec. 3.2, eqs. el8 and el9); branch '+' for small D, '-' beyond D = L^2 - 3."""
    P1 = 2.0 * D * L2
    P2 = -4.0 * D * D + (L2 - D - 3.0) * (D + 3.0)
    P3 = 2.0 * D ** 3 / L2 - (L2 - D - 3.0) * D
    rad = max(P2 * P2 - 4.0 * P1 * P3, 0.0)
    sgn = 1.0 if branch == "+" else -1.0
    return (-P2 + sgn * math.sqrt(rad)) / (2.0 * P1)


def cessation_S_ratio(T, T0, L2):
    """Shear-stress decay after cessation as a function of the trace excess
    T = tr sigma_P - 3 (Sec. 3.4, eq. relax)."""
    e = (L2 - 3.0) / L2
    return (T / T0) ** e * ((L2 + T) / (L2 + T0)) ** (1.0 - e)


def saos_moduli(wtp):
    """Oldroyd-B storage and loss moduli (Sec. 3.3, eq. modulipred)."""
    return wtp ** 2 / (1 + wtp ** 2), wtp / (1 + wtp ** 2)


def taylor_D(Ca, lam):
    """Unconfined small-deformation result (Sec. 4.1, eq. deformation)."""
    return (19 * lam + 16) / (16 * lam + 16) * Ca


def shapira_haber_D(Ca, lam, R_over_H, Csh=5.6996):
    """Confined correction (Sec. 4.1, Shapira-Haber)."""
    return taylor_D(Ca, lam) * (1 + Csh * (2.5 * lam + 1) / (lam + 1) * R_over_H ** 3)


def ellipsoid_D(a, b):
    return (a - b) / (a + b)
