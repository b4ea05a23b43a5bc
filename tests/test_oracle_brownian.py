"""Pins for the oracle's Brownian displacement directions y = D^{1/2} z
(arXiv:1711.02976, Sec. 1: the random displacements of the Ermak-McCammon
step have covariance 2 D dt, and the library draws them as D^{1/2} z).
Expected values come from closed forms of the square root of small
mobility matrices, and from squaring the square root back onto the direct
matvec -- never from the eigen-route itself."""
import numpy as np
import pytest

PI = np.pi


def test_single_bead_closed_form(orc):
    a, eta = 0.7, 1.3
    z = np.array([[0.5, -1.25, 2.0]])
    y = orc.rpy_sqrt(np.array([[1.0, 2.0, 3.0]]), z, a, eta)
    assert np.allclose(y, z / np.sqrt(6 * PI * eta * a), rtol=1e-14, atol=0)


def _pair_sqrt(c0, m, u, v):
    # square root of [[c0, m], [m, c0]] applied to (u, v): eigenvalues c0 +- m
    # on (1, 1)/sqrt2 and (1, -1)/sqrt2
    p, q = np.sqrt(c0 + m), np.sqrt(c0 - m)
    return 0.5 * ((p + q) * u + (p - q) * v), 0.5 * ((p - q) * u + (p + q) * v)


@pytest.mark.parametrize("r_over_a", [0.6, 1.5, 2.0, 3.0, 8.0])
def test_two_beads_on_an_axis_closed_form(orc, r_over_a):
    # Two beads separated along x: D couples each Cartesian component only to
    # the same component of the other bead, with the classical pair
    # mobilities (relative to 1/(6 pi eta a)): along the line 3a/(2r) - a^3/r^3
    # (far) or 1 - 3r/(16a) (overlap), transverse 3a/(4r) + a^3/(2r^3) (far)
    # or 1 - 9r/(32a) (overlap).
    a, eta = 0.5, 1.0
    r = r_over_a * a
    mu0 = 1.0 / (6 * PI * eta * a)
    if r >= 2 * a:
        par, perp = mu0 * (1.5 * a / r - a ** 3 / r ** 3), mu0 * (0.75 * a / r + 0.5 * a ** 3 / r ** 3)
    else:
        par, perp = mu0 * (1 - 3 * r / (16 * a)), mu0 * (1 - 9 * r / (32 * a))
    pos = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    z = np.array([[0.3, -1.1, 0.7], [1.9, 0.4, -0.8]])
    y = orc.rpy_sqrt(pos, z, a, eta)
    for k, m in ((0, par), (1, perp), (2, perp)):
        y0, y1 = _pair_sqrt(mu0, m, z[0, k], z[1, k])
        assert np.isclose(y[0, k], y0, rtol=1e-13, atol=1e-16)
        assert np.isclose(y[1, k], y1, rtol=1e-13, atol=1e-16)


def test_square_root_squared_is_the_direct_matvec(orc):
    # D^{1/2}(D^{1/2} z) against the O(N^2) direct sum, on a cluster with
    # overlapping pairs (r < 2a) and coincident-free random positions
    g = np.random.default_rng(11)
    n, a, eta = 150, 0.5, 0.8
    pos = g.uniform(0.0, 5.0, size=(n, 3))
    z = g.standard_normal((2, n, 3))
    y = orc.rpy_sqrt(pos, orc.rpy_sqrt(pos, z, a, eta), a, eta)
    u = orc.rpy_direct(pos, z, a, eta)
    assert np.abs(y - u).max() <= 1e-12 * np.abs(u).max()


def test_dense_matrix_is_symmetric_with_the_direct_columns(orc):
    g = np.random.default_rng(3)
    n, a, eta = 40, 0.5, 1.0
    pos = g.uniform(0.0, 3.0, size=(n, 3))
    D = orc.rpy_dense(pos, a, eta)
    # symmetric up to the rounding order of B d_k d_l
    assert np.allclose(D, D.T, rtol=1e-15, atol=1e-18)
    e = np.zeros((1, n, 3))
    e[0, 7, 2] = 1.0
    col = orc.rpy_direct(pos, e, a, eta)[0].ravel()
    assert np.allclose(D[:, 3 * 7 + 2], col, rtol=1e-14, atol=1e-18)
