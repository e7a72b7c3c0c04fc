"""Test infrastructure: FP64 reference of the mapping update that follows each back-propagation
(paper Sec. III-D): Adam on the Gaussian parameters and on every camera pose's tangent,
the pose then moved by a left-multiplied SE(3) exponential.

Only the tests import this module. Plain numpy in double precision; nothing here is shared
with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np


def adam(param, grad, m, v, lr, beta1, beta2, eps, step):
    """One step of Adam (Kingma and Ba 2015, Algorithm 1) with bias-corrected moments.

    Returns the new (param, m, v); step counts from 1. lr may be an array broadcast against
    param (one rate per component)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    p = np.asarray(param, np.float64) - np.asarray(lr, np.float64) * m_hat / (np.sqrt(v_hat) + eps)
    return p, m, v


def hat(w):
    """The skew matrix [w]x with [w]x u = w x u."""
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def exp_se3(xi):
    """Exp of the tangent xi = (rho, phi): the rigid motion (R, t) with R the rotation by the
    angle a = |phi| about phi (Rodrigues) and t = V rho, V = I + (1 - cos a) / a^2 [phi]x +
    (a - sin a) / a^3 [phi]x^2. 1 - cos a is formed as 2 sin^2(a/2), and (a - sin a) / a^3 as
    its Taylor series below a = 0.1, so that neither loses digits to cancellation."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    a = float(np.linalg.norm(phi))
    K = hat(phi)
    K2 = K @ K
    if a == 0.0:
        s, c, d = 1.0, 0.5, 1.0 / 6.0
    else:
        s = math.sin(a) / a
        c = 2.0 * math.sin(0.5 * a) ** 2 / (a * a)
        a2 = a * a
        d = (1.0 / 6.0 - a2 / 120.0 + a2 * a2 / 5040.0 - a2 ** 3 / 362880.0) if a < 0.1 else (a - math.sin(a)) / a ** 3
    R = np.eye(3) + s * K + c * K2
    V = np.eye(3) + c * K + d * K2
    return R, V @ rho


def pose_adam(R, t, grad, m, v, lr_rho, lr_phi, beta1, beta2, eps, step):
    """Adam on one view's pose tangent gradient (rho, phi), then T_cw <- Exp(delta) T_cw with
    delta the Adam step. Returns (R, t, m, v)."""
    lr = np.array([lr_rho] * 3 + [lr_phi] * 3, np.float64)
    zero = np.zeros(6)
    delta, m, v = adam(zero, grad, m, v, lr, beta1, beta2, eps, step)
    Rd, td = exp_se3(delta)
    R = np.asarray(R, np.float64).reshape(3, 3)
    t = np.asarray(t, np.float64).reshape(3)
    return Rd @ R, Rd @ t + td, m, v
