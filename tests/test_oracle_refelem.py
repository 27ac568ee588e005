"""Pins of the edge maps and reference tensors (Sec. 3.6) by identities."""
import numpy as np
import pytest

from oracle.refelem import RefTensors, gamma, theta

NU_HAT = [np.array([1.0, 1.0]) / np.sqrt(2), np.array([-1.0, 0.0]), np.array([0.0, -1.0])]
LEN_HAT = [np.sqrt(2.0), 1.0, 1.0]


def test_gamma_endpoints_ccw():
    # edge n runs from vertex n+1 to vertex n+2 (counter-clockwise), opposite vertex n
    V = [np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.0, 1.0])]
    for n in range(3):
        a = np.array(gamma(n, 0.0), dtype=float)
        b = np.array(gamma(n, 1.0), dtype=float)
        np.testing.assert_allclose(a, V[(n + 1) % 3])
        np.testing.assert_allclose(b, V[(n + 2) % 3])


def test_theta_reverses_orientation():
    # theta_{n-n+}(gamma_{n-}(s)) = gamma_{n+}(1-s) for all nine maps (eq:mapEE)
    s = np.linspace(0, 1, 11)
    for nm in range(3):
        for npl in range(3):
            x1, x2 = gamma(nm, s)
            y = theta(nm, npl, x1, x2)
            z = gamma(npl, 1 - s)
            np.testing.assert_allclose(y[0], z[0], atol=1e-15)
            np.testing.assert_allclose(y[1], z[1], atol=1e-15)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5, 6])
def test_tensor_identities_exact_policy(p):
    r = RefTensors(p, "exact")
    N = r.N
    np.testing.assert_allclose(r.hatM, np.eye(N), atol=1e-13)
    # S_off(:,:,a,b) = S_off(:,:,b,a)^T
    for a in range(3):
        for b in range(3):
            np.testing.assert_allclose(r.hatSoff[:, :, a, b], r.hatSoff[:, :, b, a].T, atol=1e-12)
    # integration by parts on the reference triangle
    for m in range(2):
        bnd = sum(NU_HAT[n][m] * LEN_HAT[n] * r.hatSdiag[:, :, n] for n in range(3))
        np.testing.assert_allclose(r.hatH[:, :, m] + r.hatH[:, :, m].T, bnd, atol=1e-12)
        G = r.hatG[:, :, :, m]
        lhs = G + G.transpose(1, 0, 2) + G.transpose(1, 2, 0)
        bndR = sum(NU_HAT[n][m] * LEN_HAT[n] * r.hatRdiag[:, :, :, n] for n in range(3))
        np.testing.assert_allclose(lhs, bndR, atol=1e-11)
    # a constant coefficient d0 has D = (d0/sqrt2, 0, ...): contractions reduce to H and S
    Dc = np.zeros(N)
    Dc[0] = 3.0 / np.sqrt(2)
    for m in range(2):
        np.testing.assert_allclose(np.einsum("l,ijl->ij", Dc, r.hatG[:, :, :, m]),
                                   3.0 * r.hatH[:, :, m], atol=1e-12)
    for n in range(3):
        np.testing.assert_allclose(np.einsum("l,ijl->ij", Dc, r.hatRdiag[:, :, :, n]),
                                   3.0 * r.hatSdiag[:, :, n], atol=1e-12)
        for npl in range(3):
            np.testing.assert_allclose(np.einsum("l,ijl->ij", Dc, r.hatRoff[:, :, :, n, npl]),
                                       3.0 * r.hatSoff[:, :, n, npl], atol=1e-12)
    # phi_1 = sqrt2 is constant: R_off(0, j, l, a, b) = sqrt2 * S_diag(l, j, b)
    for a in range(3):
        for b in range(3):
            np.testing.assert_allclose(r.hatRoff[0, :, :, a, b], np.sqrt(2) * r.hatSdiag[:, :, b].T,
                                       atol=1e-12)


def test_paper_policy_under_integrates():
    # identical for p <= 1, the integration-by-parts identity fails for p >= 2
    for p in (0, 1):
        a, b = RefTensors(p, "exact"), RefTensors(p, "paper")
        assert np.abs(a.hatG - b.hatG).max() < 1e-13
        assert np.abs(a.hatRoff - b.hatRoff).max() < 1e-13
    r = RefTensors(2, "paper")
    G = r.hatG[:, :, :, 0]
    lhs = G + G.transpose(1, 0, 2) + G.transpose(1, 2, 0)
    bndR = sum(NU_HAT[n][0] * LEN_HAT[n] * r.hatRdiag[:, :, :, n] for n in range(3))
    assert np.abs(lhs - bndR).max() > 1e-2
    # the edge mass and H are exact under both policies
    e = RefTensors(3, "exact")
    q = RefTensors(3, "paper")
    assert np.abs(e.hatSoff - q.hatSoff).max() < 1e-12
    assert np.abs(e.hatH - q.hatH).max() < 1e-12
