"""What the trained surrogate gains over the method without it.

A narrow droplet-in-shear family (only the capillary number varies) is solved to steady
deformation by the batched solver; the network is trained on the device on those solves
by the project's own kernels.  For held-out capillary numbers the network answers in a
fraction of a millisecond what the solver needs a batched run to the steady test for, and
its answers fall within |dD| <= 0.01 of the solver's steady D, the reference.  The warm start
built from its prediction keeps the droplet mass and leads the solver, used as fallback,
to the same steady D."""
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1406_2686_amd

    return paper_1406_2686_amd


def test_trained_surrogate_answers_held_out_cases_within_tolerance(lb):
    from paper_1406_2686_amd import surrogate as sg

    base = dict(nx=48, ny=24, nz=48, R=8.0, De=0.5, lam=1.0, L2=100.0, polymer_phase="B")
    train = [dict(base, Ca=float(c)) for c in np.linspace(0.08, 0.32, 13)]
    test = [dict(base, Ca=c) for c in (0.11, 0.17, 0.23, 0.29)]
    crit = dict(every=100, window=1000, tol=1e-4, max_steps=8000)
    gen = sg.solve(lb, [workloads.sweep_workload(c) for c in train], **crit)
    assert (gen["steady_step"] > 0).all(), gen["steady_step"]
    Y = np.stack([gen["D"], gen["theta"], gen["amp"]], 1)
    model = sg.Surrogate(lb, seed=1, max_train=64)
    model.fit(sg.features(train), Y, epochs=800, batch=13, lr=2e-3, seed=2)
    wtest = [workloads.sweep_workload(c) for c in test]
    cold = sg.solve(lb, wtest, **crit)
    assert (cold["steady_step"] > 0).all()
    t0 = time.perf_counter()
    pred = model.predict(sg.features(test))
    t_pred = time.perf_counter() - t0
    warm = sg.solve(lb, wtest, warm=[tuple(r) for r in pred], **crit)
    print("pred D", np.round(pred[:, 0], 4), "solver D", np.round(cold["D"], 4), "warm-start D",
          np.round(warm["D"], 4))
    print(f"answer time: network {t_pred * 1e3:.2f} ms, batched solve {cold['wall_s']:.2f} s; "
          f"steps cold {cold['steady_step']}, warm {warm['steady_step']}")
    # the gain: answers within the sweep tolerance at a small fraction of the solve time
    assert np.abs(pred[:, 0] - cold["D"]).max() <= 0.01
    assert t_pred < 0.05 * cold["wall_s"]
    # the fallback from the prediction reaches the solver's steady state
    assert (warm["steady_step"] > 0).all()
    assert np.abs(warm["D"] - cold["D"]).max() <= 0.01
