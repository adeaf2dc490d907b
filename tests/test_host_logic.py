"""CPU tests of the host-side pieces of the product: pose-update algebra of the optimiser and the
quaternion-gradient conversion of the autograd wrapper (torch on the CPU; no device needed)."""
import math

import numpy as np
import torch
from scipy.spatial.transform import Rotation

from paper_2510_26611_amd.autograd import _hamilton
from paper_2510_26611_amd.optim import quat_from_rotvec


def _to_scipy(q):
    return Rotation.from_quat(np.stack([q[:, 1], q[:, 2], q[:, 3], q[:, 0]], axis=1))


def test_quat_from_rotvec_matches_scipy():
    g = np.random.default_rng(0)
    w = g.normal(size=(50, 3)) * np.array([[1.0], [1e-9], [1e-14]] * 16 + [[2.0], [0.0]])
    q = quat_from_rotvec(torch.from_numpy(w)).numpy()
    assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-15)
    ref = Rotation.from_rotvec(w).as_matrix()
    assert np.allclose(_to_scipy(q).as_matrix(), ref, atol=1e-14)


def test_hamilton_product_composes_rotations():
    g = np.random.default_rng(1)
    a = g.normal(size=(20, 4))
    b = g.normal(size=(20, 4))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    ab = _hamilton(torch.from_numpy(a), torch.from_numpy(b)).numpy()
    ref = (_to_scipy(a) * _to_scipy(b)).as_matrix()
    assert np.allclose(_to_scipy(ab).as_matrix(), ref, atol=1e-14)


def test_tangent_gradient_reproduces_rotation_vector_gradient():
    """2 (0, g) q is tangent to the sphere and its inner product with (1/2)(0, e_j) q is g_j."""
    g = np.random.default_rng(2)
    q = g.normal(size=(10, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    gw = g.normal(size=(10, 3))
    qt = torch.from_numpy(q)
    pure = torch.cat([torch.zeros(10, 1, dtype=torch.float64), torch.from_numpy(gw)], dim=1)
    gq = (2.0 * _hamilton(pure, qt)).numpy()
    assert np.allclose(np.sum(gq * q, axis=1), 0.0, atol=1e-14)
    for j in range(3):
        e = torch.zeros(10, 4, dtype=torch.float64)
        e[:, 1 + j] = 1.0
        dq = (0.5 * _hamilton(e, qt)).numpy()
        assert np.allclose(np.sum(gq * dq, axis=1), gw[:, j], atol=1e-14)
    # and the rotation vector of a small left rotation moves q along that direction
    h = 1e-7
    w = np.zeros((10, 3))
    w[:, 0] = h
    q2 = _hamilton(quat_from_rotvec(torch.from_numpy(w)), qt).numpy()
    e = torch.zeros(10, 4, dtype=torch.float64)
    e[:, 1] = 1.0
    assert np.allclose((q2 - q) / h, (0.5 * _hamilton(e, qt)).numpy(), atol=1e-6)
    assert math.isfinite(float(np.sum(q2)))
