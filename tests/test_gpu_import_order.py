"""The package binds the library to torch's HIP runtime whatever the import order: a fresh
process that imports the package before torch creates and steps a lattice on the GPU."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = """
import paper_1406_2686_amd as lb
import workloads
wl = workloads.droplet_shear(nx=16, ny=8, nz=12, R=3.0, G=workloads.G_PHYSICS_1_004, polymer_phase="A", U=0.01)
lat = lb.from_workload(wl, device="cuda:0")
lat.step(3)
print("step", lat.diagnostics()["step"])
lat.close()
"""


def test_package_before_torch_runs_on_the_gpu():
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "step 3" in r.stdout
