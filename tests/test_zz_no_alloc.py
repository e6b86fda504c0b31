"""lbfd_diagnostics_noalloc against lbfd_diagnostics, through the C ABI.

The no-allocation entry point reduces through a static per-device array that keeps the
last call's contents.  Two calls in a row, the second on a smaller lattice (fewer stage-1
partial records than the first left behind), must each return the record of the
context-buffer entry point.  Both run the same kernels in the same order, so the records
are compared for exact equality.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _lattice(nx, ny, nz, R, steps, phase):
    import paper_1406_2686_amd as lb

    wl = workloads.droplet_shear(nx=nx, ny=ny, nz=nz, R=R, G=workloads.G_PHYSICS_1_004,
                                 polymer_phase=phase, De=0.5, U=0.01)
    lat = lb.from_workload(wl, device="cuda:0")
    lat.step(steps)
    return lat


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert a[k] == b[k] or (np.isnan(a[k]) and np.isnan(b[k])), (k, a[k], b[k])


def test_noalloc_diagnostics_equal_buffer_diagnostics_on_two_calls():
    import torch

    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    # 96x40x80 = 307,200 nodes: the first stage uses all 1024 partial records
    big = _lattice(96, 40, 80, 10.0, 30, "A")
    # 24x12x20 = 5,760 nodes: 23 partial records; the rest of the array holds the big
    # lattice's records from the call before
    small = _lattice(24, 12, 20, 4.0, 30, "B")
    ref_big = big.diagnostics()
    ref_small = small.diagnostics()
    got_big = big.diagnostics_noalloc()
    got_small = small.diagnostics_noalloc()
    _same(got_big, ref_big)
    _same(got_small, ref_small)
    assert got_small["W"] != got_big["W"] and got_small["mass_A"] < got_big["mass_A"]
    # and once more in the opposite order after further steps
    small.step(7)
    big.step(5)
    got_small = small.diagnostics_noalloc()
    got_big = big.diagnostics_noalloc()
    _same(got_small, small.diagnostics())
    _same(got_big, big.diagnostics())
    big.close()
    small.close()


def test_noalloc_diagnostics_before_fields_is_estate():
    import paper_1406_2686_amd as lb
    import torch

    torch.cuda.set_device(0)
    lat = lb.Lattice(8, 6, 8, 1, lb.make_params(), device="cuda:0")
    with pytest.raises(lb.LbfdError) as e:
        lat.diagnostics_noalloc()
    assert e.value.status == lb.ESTATE
    lat.close()
