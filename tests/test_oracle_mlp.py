"""Pins of the MLP oracle: parameter count, bf16 rounding, and the exact (unrounded) gradient
against central finite differences of the loss on a small network."""
import numpy as np

from oracle import mlp as M


def test_parameter_count():
    assert M.param_count() == 201475


def test_bf16_round_to_nearest_even():
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties go to the even one (1)
    assert M.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0
    assert M.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6
    assert M.bf16_round(np.float32(1.0 + 2.0 ** -8 + 2.0 ** -20)) == 1.0 + 2.0 ** -7
    assert M.bf16_round(np.float32(-3.0)) == -3.0
    x = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    r = M.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_gradient_matches_finite_differences():
    sizes = (12, 7, 6, 5, 4, 3)
    rng = np.random.default_rng(1)
    theta = M.init_params(3, sizes) + 0.1 * rng.standard_normal(M.param_count(sizes))
    X = rng.uniform(-1, 1, (9, 12))
    T = rng.standard_normal((9, 3)); T[:, 2] = rng.integers(0, 2, 9)
    mask = rng.integers(0, 2, 9)
    L, g = M.loss_grad(theta, X, T, mask, sizes, rounding=False)
    eps = 1e-6
    for i in rng.choice(theta.size, 60, replace=False):
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        fd = (M.loss_grad(tp, X, T, mask, sizes, rounding=False)[0] - M.loss_grad(tm, X, T, mask, sizes, rounding=False)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_topk_reference_ties_to_lower_index():
    s = np.array([1.0, 3.0, 3.0, np.nan, 2.0, 3.0, -np.inf], np.float32)
    assert list(M.topk_reference(s, 4)) == [1, 2, 5, 4]
