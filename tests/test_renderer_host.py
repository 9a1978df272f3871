"""Host-side checks of the Renderer's camera vectors (no GPU): the 6D
rotation parametrisation the paper's camera vector accepts (Sec. 4, citing
Zhou et al.) and the axis-angle form of Lst. 1."""
import numpy as np
import pytest
import torch

from paper_2004_07484_amd import _capi
from paper_2004_07484_amd.renderer import (axis_angle_to_matrix, camera_struct,
                                           rotation_6d_to_matrix, rotation_6d_to_matrix_torch)
from tests.oracle_helpers import random_rotation


def test_6d_rotation_is_a_rotation_and_recovers_its_columns():
    rng = np.random.default_rng(3)
    for _ in range(20):
        R = np.array(rotation_6d_to_matrix(rng.standard_normal(6))).reshape(3, 3)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-14)
        # a rotation's first two columns are its own 6D vector
        Q = random_rotation(rng)
        back = np.array(rotation_6d_to_matrix(np.concatenate([Q[:, 0], Q[:, 1]]))).reshape(3, 3)
        np.testing.assert_allclose(back, Q, atol=1e-14)


def test_6d_rotation_gram_schmidt_invariances():
    """Scaling a1 or a2, or adding a multiple of a1 to a2, leaves R unchanged."""
    rng = np.random.default_rng(4)
    a1, a2 = rng.standard_normal(3), rng.standard_normal(3)
    R = np.array(rotation_6d_to_matrix(np.concatenate([a1, a2])))
    for v in (np.concatenate([2.5 * a1, a2]), np.concatenate([a1, 0.3 * a2]),
              np.concatenate([a1, a2 - 1.7 * a1])):
        np.testing.assert_allclose(np.array(rotation_6d_to_matrix(v)), R, atol=1e-13)


def test_6d_rotation_torch_matches_host_and_has_a_gradient():
    r = torch.tensor(np.random.default_rng(5).standard_normal(6), requires_grad=True)
    Rt = rotation_6d_to_matrix_torch(r)
    np.testing.assert_allclose(Rt.detach().numpy().reshape(9),
                               np.array(rotation_6d_to_matrix(r.detach().numpy())), atol=1e-15)
    # the Jacobian against central differences of the host formula
    J = torch.autograd.functional.jacobian(lambda a: rotation_6d_to_matrix_torch(a).reshape(9),
                                           r.detach()).numpy()
    h = 1e-7
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        fd = (np.array(rotation_6d_to_matrix(r.detach().numpy() + e)) -
              np.array(rotation_6d_to_matrix(r.detach().numpy() - e))) / (2 * h)
        np.testing.assert_allclose(J[:, k], fd, atol=1e-7)


def test_camera_vectors_give_the_camera_struct():
    rng = np.random.default_rng(6)
    Q = random_rotation(rng)
    t = rng.standard_normal(3)
    v11 = np.concatenate([t, Q[:, 0], Q[:, 1], [1.3, 2.1]])
    c = camera_struct(v11, 40, 30, 1.0, 10.0)
    assert isinstance(c, _capi.pulsar_camera_t)
    np.testing.assert_allclose(np.array(c.R[:]), Q.reshape(9), atol=1e-6)
    np.testing.assert_allclose(np.array(c.t[:]), t, atol=1e-6)
    assert (c.focal, c.sensor_width, c.width, c.height) == pytest.approx((1.3, 2.1, 40, 30))
    aa = rng.standard_normal(3)
    c8 = camera_struct(np.concatenate([t, aa, [1.3, 2.1]]), 40, 30, 1.0, 10.0)
    np.testing.assert_allclose(np.array(c8.R[:]), np.array(axis_angle_to_matrix(aa)), atol=1e-6)
    with pytest.raises(ValueError):
        camera_struct(np.zeros(9), 40, 30, 1.0, 10.0)
