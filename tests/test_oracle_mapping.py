"""Pins of the FP64 mapping-update oracle (Adam and the left-multiplied SE(3) pose step)
against closed forms and independent library routines."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle import mapping as om


def _twist(xi):
    T = np.zeros((4, 4))
    T[:3, :3] = om.hat(xi[3:])
    T[:3, 3] = xi[:3]
    return T


@pytest.mark.parametrize("scale", [1e-9, 1e-4, 0.3, 2.0, 3.1])
def test_exp_se3_matches_matrix_exponential_of_the_twist(scale):
    rng = np.random.default_rng(int(scale * 1e3) + 7)
    for _ in range(5):
        xi = rng.normal(size=6)
        xi[3:] *= scale / np.linalg.norm(xi[3:])
        R, t = om.exp_se3(xi)
        E = expm(_twist(xi))
        np.testing.assert_allclose(R, E[:3, :3], rtol=0, atol=1e-13)
        np.testing.assert_allclose(t, E[:3, 3], rtol=0, atol=1e-13)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-13)


def test_exp_se3_of_pure_translation_and_pure_rotation():
    R, t = om.exp_se3([0.3, -0.2, 0.5, 0, 0, 0])
    np.testing.assert_array_equal(R, np.eye(3))
    np.testing.assert_allclose(t, [0.3, -0.2, 0.5], atol=0)
    # a quarter turn about z maps x to y
    R, t = om.exp_se3([0, 0, 0, 0, 0, math.pi / 2])
    np.testing.assert_allclose(R @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    np.testing.assert_allclose(t, 0, atol=0)


def test_adam_first_step_closed_form():
    # zero moments: m_hat = g, v_hat = g^2, so the step is -lr g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = om.adam(np.ones(4), g, np.zeros(4), np.zeros(4), 0.1, 0.9, 0.999, 1e-8, 1)
    np.testing.assert_allclose(p, 1 - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_matches_torch_optimizer_over_steps():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    x0 = rng.normal(size=50)
    lr, b1, b2, eps = 0.01, 0.8, 0.95, 1e-6
    x = torch.tensor(x0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([x], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = x0.copy(), np.zeros(50), np.zeros(50)
    for k in range(1, 8):
        g = rng.normal(size=50)
        opt.zero_grad()
        x.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = om.adam(p, g, m, v, lr, b1, b2, eps, k)
        np.testing.assert_allclose(p, x.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_pose_step_moves_against_the_gradient_by_left_multiplication():
    rng = np.random.default_rng(4)
    R0, t0 = om.exp_se3(rng.normal(size=6) * 0.5)
    g = np.array([0.0, 0.0, 2.0, 0.0, -3.0, 0.0])
    R, t, m, v = om.pose_adam(R0, t0, g, np.zeros(6), np.zeros(6), 0.01, 0.02, 0.9, 0.999, 1e-8, 1)
    # first step: delta = -lr sign(g) (up to eps) per component
    d = np.array([0, 0, -0.01, 0, 0.02, 0]) * (np.abs(g) / (np.abs(g) + 1e-8) + (g == 0))
    E = expm(_twist(d))
    np.testing.assert_allclose(R, E[:3, :3] @ R0, atol=1e-14)
    np.testing.assert_allclose(t, E[:3, :3] @ t0 + E[:3, 3], atol=1e-14)
