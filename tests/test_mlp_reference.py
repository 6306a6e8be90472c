"""Pins of the CPU reference network and of the smooth-part oracle used by the surrogate tests."""

import math

import numpy as np
import pytest
import torch

from oracle import method, mlp


def _queries(B, seed, near=True):
    rng = np.random.default_rng(seed)
    zmax = 0.6 if near else 1.0
    return np.column_stack([rng.uniform(-7, 7, B), rng.uniform(-7, 7, B), rng.uniform(-zmax, zmax, B),
                            rng.uniform(1, 10, B), rng.uniform(-0.5, 0.5, B), rng.uniform(-0.5, 0.5, B)])


def test_backward_matches_central_differences():
    """Every parameter block of the float64 backward pass against (L(p+h) - L(p-h)) / 2h."""
    p = mlp.init_params(0)
    q = _queries(48, 1)
    y = np.random.default_rng(2).normal(size=(48, 2))
    _, g = mlp.loss_and_grad(p, q, y)
    rng = np.random.default_rng(3)
    for off, shape in mlp.layout()[0]:
        for i in off + rng.choice(int(np.prod(shape)), min(3, int(np.prod(shape))), replace=False):
            h = 1e-5
            pp = p.copy()
            pp[i] += h
            lp, _ = mlp.loss_and_grad(pp, q, y)
            pp[i] -= 2 * h
            lm, _ = mlp.loss_and_grad(pp, q, y)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (off, i, fd, g[i])


def test_bf16_rounding_matches_torch():
    """Nearest-even rounding to bfloat16 against torch's own conversion, ties included."""
    rng = np.random.default_rng(4)
    v = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-6, 6, 4000),
                        1 + np.arange(-8, 9) * 2.0 ** -9, [0.0, -0.0, 1.0, -3.0]]).astype(np.float32)
    want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(v), want)
    assert mlp.bf16(np.float32(1 + 2.0 ** -8)) == 1.0                  # tie to even
    assert mlp.bf16(np.float32(1 + 3 * 2.0 ** -8)) == 1 + 2.0 ** -6    # tie to even (upwards)


def test_features_are_periodic_in_x1_x2_only():
    q = _queries(200, 5)
    F = mlp.features(q)
    for j in (0, 1):
        qs = q.copy()
        qs[:, j] += 2 * math.pi * 3
        assert np.max(np.abs(mlp.features(qs) - F)) < 1e-11
    qs = q.copy()
    qs[:, 2] *= 0.5
    assert np.max(np.abs(mlp.features(qs) - F)) > 0.1
    assert np.all(np.abs(F) <= 1.0 + 1e-12)


def test_bf16_forward_close_to_float64():
    """Rounding the matrix-core operands to bfloat16 moves the output by a few bf16 ulps."""
    p = mlp.init_params(6)
    q = _queries(256, 7)
    o64, _ = mlp.forward(p, q)
    o16, _ = mlp.forward(p, q, bf16_ops=True)
    err = np.max(np.abs(o16 - o64)) / np.max(np.abs(o64))
    assert 1e-4 < err < 3e-2


def test_smooth_part_plus_add_back_is_the_method():
    """G_d = e^{i alpha.x'} L_N + e^{i 2 pi alpha.n} psi (Algorithm 3.1 step 2e), with L_N from smooth_3d,
    reproduces evaluate_3d in the near region; far targets give NaN."""
    k, a1, a2 = 3.7, 0.2, 0.35
    st = method.prepare_3d(k, a1, a2, 8, 8, 8)
    rng = np.random.default_rng(8)
    x = np.column_stack([rng.uniform(-7, 7, 400), rng.uniform(-7, 7, 400), rng.uniform(-1, 1, 400)])
    x[:20, :2] = 2 * math.pi * rng.integers(-1, 2, (20, 2)) + rng.uniform(-0.05, 0.05, (20, 2))
    x[:20, 2] = rng.uniform(-0.05, 0.05, 20)
    L = method.smooth_3d(st, x)
    near = np.abs(x[:, 2]) <= 0.6
    assert np.all(np.isnan(L[~near])) and np.all(np.isfinite(L[near]))
    q = np.column_stack([x, np.full(400, k), np.full(400, a1), np.full(400, a2)])
    G = mlp.g_from_smooth(q, L)
    want = method.evaluate_3d(st, x)
    assert np.allclose(G[near], want[near], rtol=1e-13, atol=1e-13)
