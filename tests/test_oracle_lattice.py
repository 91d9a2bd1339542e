"""Pins of oracle.lattice against textbook facts of the D2Q9 MRT basis."""
import numpy as np

from oracle import lattice as lat
from oracle.step import feq_weights, meq_moments


def test_moment_rows_orthogonal():
    # Lallemand & Luo: rows of M are mutually orthogonal with these norms
    g = lat.M @ lat.M.T
    np.testing.assert_array_equal(g, np.diag([9, 36, 36, 6, 12, 6, 12, 4, 4]))


def test_inverse_is_scaled_transpose():
    d = np.diag(1.0 / np.array([9, 36, 36, 6, 12, 6, 12, 4, 4], dtype=float))
    np.testing.assert_allclose(lat.M_INV, lat.M.T @ d, atol=1e-15)
    np.testing.assert_allclose(lat.M_INV @ lat.M, np.eye(9), atol=1e-14)


def test_rows_match_velocity_polynomials():
    cx, cy = lat.CX.astype(float), lat.CY.astype(float)
    c2 = cx**2 + cy**2
    rows = [np.ones(9), 3 * c2 - 4, 4.5 * c2**2 - 10.5 * c2 + 4, cx, (3 * c2 - 5) * cx,
            cy, (3 * c2 - 5) * cy, cx**2 - cy**2, cx * cy]
    np.testing.assert_array_equal(lat.M, np.array(rows))


def test_weight_isotropy():
    w, cx, cy = lat.W_EQ, lat.CX, lat.CY
    assert abs(w.sum() - 1) < 1e-15
    assert abs((w * cx * cx).sum() - 1 / 3) < 1e-15
    assert abs((w * cx * cy).sum()) < 1e-15
    assert abs((w * cx**4).sum() - 1 / 3) < 1e-15
    assert abs((w * cx**2 * cy**2).sum() - 1 / 9) < 1e-15
    W = lat.W_INT
    assert abs((W * cx * cx).sum() - 1.0) < 1e-15  # gradient stencil normalisation
    assert abs((W * cx * cy).sum()) < 1e-15
    for i in range(9):
        assert lat.CX[lat.OPP[i]] == -lat.CX[i] and lat.CY[lat.OPP[i]] == -lat.CY[i]


def test_equilibrium_moments_match_weight_form():
    rng = np.random.default_rng(1)
    rho = rng.uniform(0.3, 7.0, (5, 6))
    ux = rng.uniform(-0.1, 0.1, (5, 6))
    uy = rng.uniform(-0.1, 0.1, (5, 6))
    m = np.tensordot(lat.M, feq_weights(rho, ux, uy), axes=(1, 0))
    np.testing.assert_allclose(m, meq_moments(rho, ux, uy), rtol=0, atol=1e-14)
