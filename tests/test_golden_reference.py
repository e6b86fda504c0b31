"""CPU checks of the stored 20,000-step oracle reference of the 128x64x128 droplet
(tests/golden/droplet_long_De<De>.npz, written by tests/golden/droplet_long_reference.py):
the record is complete, and the reference obeys what the method conserves exactly (species
mass, Sec. 2: streaming and the collision move mass without creating it) and keeps C
symmetric positive definite with tr C < L^2 on the stored nodes (Sec. 2, FENE-P)."""
import json
import os

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
MARKS = ("1000", "2000", "5000", "10000", "20000")


@pytest.mark.parametrize("De", [0.1, 0.5, 1.0])
def test_stored_long_reference(De):
    path = os.path.join(HERE, "golden", f"droplet_long_De{De:g}.npz")
    if not os.path.exists(path):
        pytest.skip(f"no stored reference {os.path.basename(path)}")
    ref = np.load(path)
    assert int(ref["step"]) == 20000
    assert ref["rho"].shape == (2, 4096) and ref["u"].shape == (3, 4096) and ref["CmI"].shape == (6, 4096)
    diags = json.loads(str(ref["diags"]))
    assert tuple(diags) == MARKS
    wl = workloads.droplet_cfg1(De=De, variant="physics")
    m0 = wl["rho"].sum(axis=1)
    for k in MARKS:
        d = diags[k]
        assert d["flags"] == 0
        assert abs(d["mass_A"] - m0[0]) < 1e-9 * m0[0] and abs(d["mass_B"] - m0[1]) < 1e-9 * m0[1]
        assert 0.0 <= d["D"] < 1.0
    # C = I + CmI symmetric positive definite with tr C < L^2 on every stored node
    c = ref["CmI"].astype(np.float64) + np.array([1, 1, 1, 0, 0, 0.0])[:, None]
    M = np.empty((4096, 3, 3))
    M[:, 0, 0], M[:, 1, 1], M[:, 2, 2] = c[0], c[1], c[2]
    M[:, 0, 1] = M[:, 1, 0] = c[3]
    M[:, 0, 2] = M[:, 2, 0] = c[4]
    M[:, 1, 2] = M[:, 2, 1] = c[5]
    assert np.all(np.linalg.eigvalsh(M)[:, 0] > 0)
    assert np.all(c[0] + c[1] + c[2] < wl["params"]["L2"])
