"""Pins of the FP64 reference network used to check the GPU training kernels."""
import numpy as np
import pytest

from oracle import mlp as ref


def test_reference_gradient_by_finite_differences():
    """The FP64 reference backpropagation against central differences."""
    X, Y, _, _ = ref.dataset(64, seed=22)
    Xs = (X - X.mean(0)) / X.std(0)
    P = ref.init_params(seed=5)
    _, g = ref.loss_and_grad(P, Xs, Y)
    rng = np.random.default_rng(0)
    h = 1e-6
    for l in range(4):
        for k in range(2):
            arr = P[l][k]
            for _ in range(3):
                idx = tuple(rng.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = ref.loss_and_grad(P, Xs, Y)
                arr[idx] = old - h
                lm, _ = ref.loss_and_grad(P, Xs, Y)
                arr[idx] = old
                assert g[l][k][idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-5, abs=1e-9)


def test_dataset_targets_match_primitives():
    """Targets are log W and log(hW) of the sampled primitives, and the
    sampled magnetisation b^2/rho lies in the requested range."""
    X, Y, U, prims = ref.dataset(1000, seed=30)
    W = np.sqrt(1 + np.sum(prims[:, 1:4] ** 2, axis=1))
    assert np.allclose(np.exp(Y[:, 0]), W, rtol=1e-14)
    assert np.all((W >= 1.0) & (W <= 50.0 + 1e-9))
    v = prims[:, 1:4] / W[:, None]
    B = prims[:, 5:8]
    b2 = np.sum(B * B, axis=1) / W ** 2 + np.sum(B * v, axis=1) ** 2
    sig = b2 / prims[:, 0]
    assert np.all((sig > 1e-4 * 0.999) & (sig < 100 * 1.001))
    assert np.all(np.isfinite(X))
