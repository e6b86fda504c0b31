"""Interfacial tension of the two-component Shan-Chen mixture used by the droplet
workloads, measured with the FP64 oracle through the Laplace law.

Sec. 4.1 defines the capillary number with sigma_AB, and the bulk pressure of the model
is P_b = c_s^2 (rho_A + rho_B + G rho_A rho_B) (Sec. 2, eq. PTexpanded).  A resting droplet
of radius R has P_in - P_out = 2 sigma_AB / R, so a fit of the pressure jump against 1/R
over several radii gives sigma_AB.  Writes sigma_calibration.json next to this file.
Calls only the oracle and the seeded input generator.
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402

CS2 = 1.0 / 3.0


def laplace_run(R, G, n=40, steps=3000):
    wl = workloads.droplet_shear(nx=n, ny=n, nz=n, R=R, G=G, polymer_phase="none", U=0.0)
    o = oracle.from_workload(wl)
    assert o.step(steps) == 0
    rho, u, _ = o.get_fields()
    rA, rB = rho
    phi = (rA - rB) / (rA + rB)
    P = CS2 * (rA + rB + G * rA * rB)
    Z, Y, X = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((X.ravel() - (n - 1) / 2) ** 2 + (Y.ravel() - (n - 1) / 2) ** 2 + (Z.ravel() - (n - 1) / 2) ** 2)
    inside = r < R - 4
    outside = (r > R + 6) & (Y.ravel() > 2) & (Y.ravel() < n - 3)
    R_eff = (3.0 * np.count_nonzero(phi > 0) / (4.0 * math.pi)) ** (1.0 / 3.0)
    return {"R_init": R, "R_eff": float(R_eff), "P_in": float(P[inside].mean()), "P_out": float(P[outside].mean()),
            "rhoA_in": float(rA[inside].mean()), "rhoB_in": float(rB[inside].mean()),
            "rhoA_out": float(rA[outside].mean()), "rhoB_out": float(rB[outside].mean()),
            "max_u": float(np.abs(u).max()), "steps": steps}


def main():
    G = workloads.G_PHYSICS_1_004
    runs = [laplace_run(R, G) for R in (8.0, 10.0, 12.0)]
    x = np.array([2.0 / r["R_eff"] for r in runs])
    y = np.array([r["P_in"] - r["P_out"] for r in runs])
    sigma = float(np.dot(x, y) / np.dot(x, x))  # fit through the origin: dP = sigma * 2/R
    out = {"_about": "Laplace-law fit of sigma_AB with the FP64 oracle (tests/golden/sigma_calibration.py)",
           "G": G, "rho_in": 1.0, "rho_out": 0.04, "sigma_AB": sigma, "runs": runs}
    with open(os.path.join(HERE, "sigma_calibration.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
