"""Pins for the four-Laplace decomposition (arXiv:1711.02976, Sec. 2:
L1..L4, L_C and eq. (2.8)) and for the spherical-harmonic machinery of the
oracle's FMM (Sec. 2: expansion forms, Y_n^m normalisation, Theorems 1-2).

Expected values come from an independent library (scipy), from closed-form
derivatives of 1/r, from exactness of polynomial translations, or from the
direct RPY sum."""
import numpy as np
import pytest
from scipy.special import assoc_legendre_p, sph_harm_y


def test_legendre_matches_scipy_with_cs_phase(orc):
    P = 30
    for x in (-0.93, -0.2, 0.0, 0.41, 0.999):
        got = orc.legendre(P, x)
        for n in range(P + 1):
            for m in range(n + 1):
                ref = float(np.squeeze(assoc_legendre_p(n, m, x)))
                assert abs(got[n * (n + 1) // 2 + m] - ref) <= 1e-12 * max(1.0, abs(ref)), (n, m, x)


def test_ynm_normalisation_matches_scipy(orc):
    # Paper: Y_n^m = sqrt((n-|m|)!/(n+|m|)!) P_n^|m| e^{im phi}; scipy's
    # orthonormal harmonic carries an extra sqrt((2n+1)/(4 pi)).
    P = 20
    th, ph = 1.1, 2.3
    got = orc.ynm(P, th, ph)
    for n in range(P + 1):
        for m in range(n + 1):
            ref = sph_harm_y(n, m, th, ph) * np.sqrt(4 * np.pi / (2 * n + 1))
            assert abs(got[n * (n + 1) // 2 + m] - ref) < 1e-13


def _laplace_exact(src, q, x):
    d = x[None, :] - src
    r = np.linalg.norm(d, axis=1)
    val = np.sum(q / r)
    grad = -np.sum(q[:, None] * d / r[:, None] ** 3, axis=0)
    hess = np.zeros((3, 3))
    for k in range(len(q)):
        hess += q[k] * (3 * np.outer(d[k], d[k]) - r[k] ** 2 * np.eye(3)) / r[k] ** 5
    return val, grad, hess


def test_multipole_theorem1_against_closed_form(orc):
    # Sources near the centre, target far: truncation ~ (0.1)^p.
    rng = np.random.default_rng(2)
    src = rng.uniform(-0.05, 0.05, size=(6, 3))
    q = rng.normal(size=6)
    p = 18
    M = orc.p2m(p, src, q, np.zeros(3))
    for x in (np.array([0.8, -0.3, 0.5]), np.array([0.0, 0.0, -0.9]), np.array([0.0, 0.7, 0.0])):
        v, g, h = orc.eval_expansion(p, "M", M, x)
        ve, ge, he = _laplace_exact(src, q, x)
        assert abs(v - ve) < 1e-13 * abs(ve) + 1e-15
        assert np.allclose(g, ge, rtol=1e-12, atol=1e-14)
        assert np.allclose(h, he, rtol=1e-11, atol=1e-13)


def test_local_theorem2_against_closed_form(orc):
    # Target near the centre, sources far.  A wrong sign in s6 or a dropped
    # s1 term would break the gradient/Hessian comparison.
    rng = np.random.default_rng(4)
    src = rng.uniform(-1, 1, size=(7, 3))
    src = src / np.linalg.norm(src, axis=1, keepdims=True) * 1.2
    q = rng.normal(size=7)
    p = 20
    c = np.array([0.01, -0.02, 0.015])
    L = orc.p2l(p, src, q, c)
    for v in (np.array([0.05, 0.03, -0.06]), np.array([0.0, 0.0, 0.08]), np.zeros(3)):
        val, g, h = orc.eval_expansion(p, "L", L, v)
        ve, ge, he = _laplace_exact(src, q, c + v)
        assert abs(val - ve) < 1e-13 * abs(ve) + 1e-15
        assert np.allclose(g, ge, rtol=1e-12, atol=1e-14)
        assert np.allclose(h, he, rtol=1e-11, atol=1e-13)


def test_m2m_is_exact(orc):
    rng = np.random.default_rng(6)
    src = rng.uniform(-0.25, 0.25, size=(9, 3))
    q = rng.normal(size=9)
    p = 12
    c0 = np.zeros(3)
    c1 = np.array([0.25, -0.25, 0.25])
    Mt = orc.translate(p, "m2m", orc.p2m(p, src, q, c0), c0, c1)
    Md = orc.p2m(p, src, q, c1)
    assert np.max(np.abs(Mt - Md)) < 1e-13 * np.max(np.abs(Md))


def test_l2l_is_exact(orc):
    rng = np.random.default_rng(7)
    src = rng.uniform(3, 4, size=(5, 3))
    q = rng.normal(size=5)
    p = 12
    c0 = np.zeros(3)
    c1 = np.array([-0.2, 0.1, 0.3])
    L0 = orc.p2l(p, src, q, c0)
    L1 = orc.translate(p, "l2l", L0, c0, c1)
    x = np.array([0.1, 0.2, -0.1])
    a = orc.eval_expansion(p, "L", L0, x - c0)
    b = orc.eval_expansion(p, "L", L1, x - c1)
    assert abs(a[0] - b[0]) < 1e-13 * abs(a[0])
    assert np.allclose(a[1], b[1], rtol=1e-12)
    assert np.allclose(a[2], b[2], rtol=1e-11)


def test_m2l_converges_to_p2l_and_exact(orc):
    rng = np.random.default_rng(8)
    src = rng.uniform(-0.5, 0.5, size=(8, 3))
    q = rng.normal(size=8)
    ct = np.array([2.0, 1.0, -2.0])  # a V-list-like separation for unit boxes
    x = ct + np.array([0.3, -0.4, 0.2])
    ve = _laplace_exact(src, q, x)[0]
    prev = np.inf
    for p in (4, 8, 12, 16, 20):
        L = orc.translate(p, "m2l", orc.p2m(p, src, q, np.zeros(3)), np.zeros(3), ct)
        err = abs(orc.eval_expansion(p, "L", L, x - ct)[0] - ve) / abs(ve)
        assert err < prev
        prev = err
    assert prev < 1e-9


def test_four_laplace_identity_vs_direct(orc):
    # With no overlapping pairs, direct - self = far field of eq. (2.8).
    rng = np.random.default_rng(12)
    n = 400
    pos = rng.uniform(0, 5.0, size=(n, 3))
    F = rng.normal(size=(n, 3))
    a, eta = 0.004, 1.3
    d = np.linalg.norm(pos[:, None] - pos[None], axis=-1) + 1e9 * np.eye(n)
    assert d.min() >= 2 * a
    direct = orc.rpy_direct(pos, F, a, eta)
    far = orc.far_four_laplace(pos, F, a, eta)
    near = direct - F / (6 * np.pi * eta * a)
    assert orc.rel_l2(far, near) < 1e-12


def test_four_laplace_with_overlaps_and_box_centring(orc):
    rng = np.random.default_rng(13)
    n = 300
    pos = rng.uniform(0, 1.0, size=(n, 3)) + 200.0  # far from the origin
    F = rng.normal(size=(n, 3))
    a, eta = 0.05, 1.0
    direct = orc.rpy_direct(pos, F, a, eta)
    corr = np.zeros((n, 3))
    for i in range(n):
        for j in range(n):
            dd = pos[i] - pos[j]
            if np.linalg.norm(dd) < 2 * a:
                corr[i] += orc.rpy_block(dd, a, eta) @ F[j]
    # box-centred fourth charge (any per-target centre) is an exact rewrite
    centres = np.floor(pos * 4) / 4 + 0.125
    far_c = orc.far_four_laplace(pos, F, a, eta, centers=centres)
    assert orc.rel_l2(far_c + corr, direct) < 1e-12
    # the global-origin form is the same sum, but loses digits to cancellation
    far_g = orc.far_four_laplace(pos, F, a, eta)
    assert orc.rel_l2(far_g + corr, direct) < 1e-8
