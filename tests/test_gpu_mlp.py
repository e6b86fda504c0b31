"""GPU parity of the surrogate network's hand-written kernels against the FP64 reference:
forward pass, loss and gradient of every parameter, one Adam update, BF16 inference on
the matrix cores, and on-device training that learns a smooth map."""
import numpy as np
import pytest

import workloads
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1406_2686_amd

    return paper_1406_2686_amd


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n", [1, 31, 200, 513])
def test_forward_matches_reference(lb, n):
    p = workloads.mlp_params(seed=5)
    X, _ = workloads.mlp_batch(n, seed=6)
    net = lb.MLP(max_batch=256, max_train=16)
    net.set_params(p)
    Y = net.forward(X)
    ref, _ = omlp.forward(p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    assert rel(Y, ref) < 2e-6
    net.close()


@pytest.mark.parametrize("n", [7, 256])
def test_loss_and_gradient_match_reference(lb, n):
    p = workloads.mlp_params(seed=7).astype(np.float32)
    X, T = workloads.mlp_batch(n, seed=8)
    X = X.astype(np.float32)
    T = T.astype(np.float32)
    net = lb.MLP(max_batch=256, max_train=16)
    net.set_params(p)
    L, g = net.loss_grad(X, T)
    Lr, gr = omlp.loss_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(L - Lr) < 1e-5 * Lr
    for lo, hi in ((0, 640), (640, 768), (768, 17152), (17152, 17280), (17280, 17664), (17664, 17667)):
        assert rel(g[lo:hi], gr[lo:hi]) < 1e-4, (lo, hi)
    # one Adam update from zero moments
    net.adam_step(lr=1e-3)
    q = net.get_params()
    qr, _, _ = omlp.adam(p.astype(np.float64), g.astype(np.float64), 0.0, 0.0, 1, lr=1e-3)
    assert np.max(np.abs(q - qr)) < 1e-6
    net.close()


def test_bf16_inference_on_matrix_cores(lb):
    """BF16 weights and activations with FP32 accumulation: within a few BF16 ulps of the
    FP64 reference; ragged sample counts exercise the padded tiles."""
    p = workloads.mlp_params(seed=9)
    net = lb.MLP(max_batch=512, max_train=16)
    net.set_params(p)
    for n in (1, 32, 77, 512, 1000):
        X, _ = workloads.mlp_batch(n, seed=10 + n)
        Y = net.infer_bf16(X)
        ref, _ = omlp.forward(p, X)
        assert rel(Y, ref) < 2e-2, n
        assert np.all(np.isfinite(Y))
    net.close()


def test_training_on_device_learns_a_smooth_map(lb):
    X, T = workloads.mlp_batch(2048, seed=11)
    Xv, Tv = workloads.mlp_batch(256, seed=12)
    net = lb.MLP(max_batch=256, max_train=2048, seed=3)
    before = omlp.loss(net.get_params(), Xv, Tv)
    last = net.train(X, T, epochs=150, batch=128, lr=3e-3, seed=1)
    after = omlp.loss(net.get_params(), Xv, Tv)
    print(f"mlp train: held-out loss {before:.4f} -> {after:.5f}, last minibatch {last:.5f}")
    assert after < 0.05 * before and after < 0.01
    # BF16 inference of the trained network agrees with the FP32 one
    assert rel(net.infer_bf16(Xv), net.forward(Xv)) < 2e-2
    net.close()
