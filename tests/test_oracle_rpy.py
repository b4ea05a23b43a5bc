"""Pins for the oracle's RPY tensor and direct sum (arXiv:1711.02976, Sec. 1,
the three RPY block equations).  The expected values come from closed forms
written independently of the oracle (the classical a/r mobility functions),
from invariants, and from limits -- never from the oracle itself."""
import numpy as np
import pytest

PI = np.pi


def test_self_block_and_single_bead(orc):
    a, eta = 0.3, 1.7
    M = orc.rpy_block([0, 0, 0], a, eta)
    assert np.allclose(M, np.eye(3) / (6 * PI * eta * a), rtol=1e-15, atol=0)
    F = np.array([[[1.5, -2.0, 0.25]]])
    u = orc.rpy_direct(np.array([[0.3, 0.4, 0.5]]), F, a, eta)
    assert np.allclose(u[0, 0], F[0, 0] / (6 * PI * eta * a), rtol=1e-15)


@pytest.mark.parametrize("r_over_a", [2.0, 2.5, 3.7, 10.0, 123.0])
def test_two_bead_far_mobility_functions(orc, r_over_a):
    # Classical RPY pair mobilities in a/r form, relative to 1/(6 pi eta a):
    #   along the line of centres   3a/(2r) - a^3/r^3
    #   transverse                  3a/(4r) + a^3/(2r^3)
    a, eta = 0.4, 0.9
    r = r_over_a * a
    e = np.array([1.0, 2.0, -2.0]) / 3.0
    M = orc.rpy_block(r * e, a, eta)
    mu0 = 1.0 / (6 * PI * eta * a)
    par = mu0 * (1.5 * a / r - a ** 3 / r ** 3)
    perp = mu0 * (0.75 * a / r + 0.5 * a ** 3 / r ** 3)
    expect = perp * np.eye(3) + (par - perp) * np.outer(e, e)
    assert np.allclose(M, expect, rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("r_over_a", [1e-6, 0.3, 1.0, 1.9, 1.999999])
def test_two_bead_overlap_mobility_functions(orc, r_over_a):
    # Overlapping spheres (Rotne-Prager regularisation), relative to 1/(6 pi eta a):
    #   along the line of centres   1 - 3r/(16a)
    #   transverse                  1 - 9r/(32a)
    a, eta = 0.25, 2.0
    r = r_over_a * a
    e = np.array([0.0, 0.6, 0.8])
    M = orc.rpy_block(r * e, a, eta)
    mu0 = 1.0 / (6 * PI * eta * a)
    par = mu0 * (1 - 3 * r / (16 * a))
    perp = mu0 * (1 - 9 * r / (32 * a))
    expect = perp * np.eye(3) + (par - perp) * np.outer(e, e)
    assert np.allclose(M, expect, rtol=1e-13, atol=1e-16)


def test_continuity_at_contact_and_printed_form_fails(orc):
    a, eta = 0.5, 1.0
    e = np.array([0.48, -0.6, 0.64])
    lo = orc.rpy_block(2 * a * (1 - 1e-12) * e, a, eta)
    hi = orc.rpy_block(2 * a * e, a, eta)
    assert np.max(np.abs(lo - hi)) < 1e-11
    # The overlap block exactly as printed (prefactor 1/(6 pi eta r)) jumps.
    r = 2 * a
    printed = 1 / (6 * PI * eta * r) * ((1 - 9 * r / (32 * a)) * np.eye(3) + 3 / (32 * a) * np.outer(e, e))
    assert np.max(np.abs(printed - hi)) > 1e-3


def test_zero_separation_limit(orc):
    a, eta = 0.7, 1.3
    M0 = orc.rpy_block([0, 0, 0], a, eta)
    Me = orc.rpy_block([1e-13, -2e-13, 1e-13], a, eta)
    assert np.allclose(Me, M0, rtol=1e-11)


def test_oseen_limit(orc):
    # a -> 0 at fixed r: the Stokeslet (Oseen) tensor (I/r + d d^T/r^3)/(8 pi eta).
    eta = 1.0
    d = np.array([0.3, -1.2, 0.7])
    r = np.linalg.norm(d)
    M = orc.rpy_block(d, 1e-9, eta)
    oseen = (np.eye(3) / r + np.outer(d, d) / r ** 3) / (8 * PI * eta)
    assert np.allclose(M, oseen, rtol=1e-12)


def test_scaling(orc):
    d = np.array([0.9, 0.1, -0.4])
    for a in (0.2, 0.6):  # far and overlapping
        for lam in (0.5, 3.0):
            M = orc.rpy_block(d, a, 1.0)
            Ml = orc.rpy_block(lam * d, lam * a, 1.0)
            assert np.allclose(Ml, M / lam, rtol=1e-14)


def test_block_symmetry_and_evenness(orc):
    rng = np.random.default_rng(3)
    for _ in range(20):
        d = rng.normal(size=3)
        a = abs(rng.normal()) * 0.6
        M = orc.rpy_block(d, a, 1.0)
        assert np.allclose(M, M.T, rtol=0, atol=1e-15)
        assert np.allclose(M, orc.rpy_block(-d, a, 1.0), rtol=0, atol=0)


def _dense(orc, pos, a, eta):
    n = len(pos)
    D = np.zeros((3 * n, 3 * n))
    for i in range(n):
        for j in range(n):
            D[3 * i:3 * i + 3, 3 * j:3 * j + 3] = orc.rpy_block(pos[i] - pos[j], a, eta)
    return D


def test_spd_with_many_overlaps(orc):
    rng = np.random.default_rng(11)
    pos = rng.uniform(0, 1.0, size=(60, 3))
    a = 0.15
    D = _dense(orc, pos, a, 1.0)
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
    assert np.sum((d < 2 * a) & (d > 0)) > 200
    assert np.allclose(D, D.T, atol=1e-15)
    np.linalg.cholesky(D)  # raises if not positive definite


def test_printed_overlap_block_is_not_spd(orc):
    # The printed prefactor 1/(6 pi eta r) breaks positive definiteness.
    rng = np.random.default_rng(11)
    pos = rng.uniform(0, 1.0, size=(60, 3))
    a, eta = 0.15, 1.0
    D = _dense(orc, pos, a, eta)
    n = len(pos)
    for i in range(n):
        for j in range(n):
            dd = pos[i] - pos[j]
            r = np.linalg.norm(dd)
            if 0 < r < 2 * a:
                D[3 * i:3 * i + 3, 3 * j:3 * j + 3] = 1 / (6 * PI * eta * r) * (
                    (1 - 9 * r / (32 * a)) * np.eye(3) + 3 / (32 * a) * np.outer(dd, dd) / r ** 2)
    assert np.linalg.eigvalsh(D).min() < 0


def test_direct_matches_dense_and_invariants(orc):
    rng = np.random.default_rng(5)
    n = 80
    pos = rng.uniform(0, 2.0, size=(n, 3))
    a, eta = 0.1, 0.8
    F = rng.normal(size=(2, n, 3))
    u = orc.rpy_direct(pos, F, a, eta)
    D = _dense(orc, pos, a, eta)
    for r in range(2):
        assert np.allclose(u[r].ravel(), D @ F[r].ravel(), rtol=1e-13, atol=1e-14)
    # linearity, translation invariance, symmetry G.(MF) = F.(MG), F.MF > 0
    u2 = orc.rpy_direct(pos + np.array([10.0, -3.0, 7.0]), F, a, eta)
    assert np.allclose(u2, u, rtol=1e-12, atol=1e-13)
    ul = orc.rpy_direct(pos, 2.0 * F[0] - 0.5 * F[1], a, eta)
    assert np.allclose(ul, 2.0 * u[0] - 0.5 * u[1], rtol=1e-12, atol=1e-13)
    assert abs(np.sum(F[1] * u[0]) - np.sum(F[0] * u[1])) < 1e-12 * np.sum(np.abs(F[0] * u[1]))
    assert np.sum(F[0] * u[0]) > 0


def test_direct_targets_subset(orc):
    rng = np.random.default_rng(9)
    pos = rng.uniform(0, 1, size=(300, 3))
    F = rng.normal(size=(300, 3))
    full = orc.rpy_direct(pos, F, 0.02, 1.0)
    tg = np.array([0, 17, 299, 5])
    sub = orc.rpy_direct(pos, F, 0.02, 1.0, targets=tg)
    assert np.array_equal(sub, full[tg])
