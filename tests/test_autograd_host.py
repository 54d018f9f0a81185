"""Host side of the autograd binding: the SE(3) right Jacobian that turns
the library's right-perturbation pose gradient into the gradient with
respect to xi, checked against central differences of the matrix
exponential of the twist (scipy's expm, independent of the closed form)."""
import numpy as np
import pytest
from scipy.linalg import expm

from paper_1709_03763_amd.autograd import perturbed_poses, se3_right_jacobian


def _hat(xi):
    M = np.zeros((4, 4))
    p = xi[3:]
    M[:3, :3] = [[0.0, -p[2], p[1]], [p[2], 0.0, -p[0]], [-p[1], p[0], 0.0]]
    M[:3, 3] = xi[:3]
    return M


@pytest.mark.parametrize("theta", [0.0, 1e-9, 1e-5, 1e-2, 0.3, 2.0, 3.0])
def test_right_jacobian_matches_expm_differences(theta):
    """Exp(xi)^-1 Exp(xi + h e_j) = Exp(h J_r(xi) e_j) + O(h^2): the central
    difference of the left side at h is the twist of column j of J_r."""
    rng = np.random.default_rng(int(theta * 1e3) + 7)
    xi = np.concatenate([rng.normal(0, 0.5, 3), rng.normal(0, 1, 3)])
    n = np.linalg.norm(xi[3:])
    xi[3:] *= theta / n
    Jr = se3_right_jacobian(xi)
    Ti = np.linalg.inv(expm(_hat(xi)))
    h = 1e-5
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        M = (Ti @ expm(_hat(xi + e)) - Ti @ expm(_hat(xi - e))) / (2 * h)
        np.testing.assert_allclose(M, _hat(Jr[:, j]), atol=1e-8)


def test_right_jacobian_is_identity_at_zero():
    np.testing.assert_array_equal(se3_right_jacobian(np.zeros(6)), np.eye(6))


def test_perturbed_poses_equal_expm():
    """T Exp(xi) from the closed-form exponential equals T expm(xi^)."""
    rng = np.random.default_rng(3)
    R = np.stack([expm(_hat(np.r_[0, 0, 0, rng.normal(0, 1, 3)]))[:3, :3] for _ in range(4)])
    t = rng.normal(0, 1, (4, 3))
    xi = rng.normal(0, 0.2, (4, 6))
    xi[1] = 0.0
    xi[2, 3:] = 1e-8
    Ro, to = perturbed_poses(R, t, xi)
    for k in range(4):
        T = np.eye(4)
        T[:3, :3], T[:3, 3] = R[k], t[k]
        E = T @ expm(_hat(xi[k]))
        np.testing.assert_allclose(Ro[k], E[:3, :3], atol=1e-13)
        np.testing.assert_allclose(to[k], E[:3, 3], atol=1e-13)
