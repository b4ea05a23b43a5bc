"""Pins for the oracle's second evaluation approach (Sec. 2, the paragraph
after Theorem 2): each velocity component of eq. (2.8) pre-assembled into one
polynomial per leaf, then evaluated.

  * the monomial form of r^n P_n^m(cos t) e^{i m phi} (written out from
    Rodrigues' formula) equals scipy's associated Legendre function (with the
    Condon-Shortley phase) at random points;
  * those polynomials are harmonic (their Laplacian vanishes identically);
  * the oracle FMM with the second approach equals the first approach
    (Theorem 2's derivative series, a different route) to rounding, on
    trees with W, X and O lists, and converges to the direct sum."""
import numpy as np
import pytest
from scipy.special import lpmv

import workloads as W


def _eval_poly(C, v):
    P = C.shape[0] - 1
    s = 0.0
    for a in range(P + 1):
        for b in range(P + 1 - a):
            for c in range(P + 1 - a - b):
                s = s + C[a, b, c] * v[0] ** a * v[1] ** b * v[2] ** c
    return s


@pytest.mark.parametrize("n,m", [(0, 0), (1, 0), (1, 1), (2, 1), (5, 0), (5, 3), (8, 8), (9, 4), (12, 7)])
def test_solid_monomials_match_legendre(orc, n, m):
    P = 12
    C = orc.solid_monomials(P, n, m)
    g = np.random.default_rng(100 + 13 * n + m)
    for _ in range(5):
        v = g.uniform(-1.0, 1.0, 3)
        r = np.linalg.norm(v)
        th, ph = np.arccos(v[2] / r), np.arctan2(v[1], v[0])
        ref = r ** n * lpmv(m, n, np.cos(th)) * np.exp(1j * m * ph)
        got = _eval_poly(C, v)
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref))
    # only degree-n monomials appear
    deg = np.add.outer(np.add.outer(np.arange(P + 1), np.arange(P + 1)), np.arange(P + 1))
    assert np.all(C[deg != n] == 0)


@pytest.mark.parametrize("n,m", [(3, 2), (7, 1), (10, 6)])
def test_solid_monomials_are_harmonic(orc, n, m):
    P = 12
    C = orc.solid_monomials(P, n, m)
    lap = np.zeros_like(C)
    for a in range(P + 1):
        for b in range(P + 1):
            for c in range(P + 1):
                if a >= 2:
                    lap[a - 2, b, c] += a * (a - 1) * C[a, b, c]
                if b >= 2:
                    lap[a, b - 2, c] += b * (b - 1) * C[a, b, c]
                if c >= 2:
                    lap[a, b, c - 2] += c * (c - 1) * C[a, b, c]
    assert np.abs(lap).max() <= 1e-9 * max(1.0, np.abs(C).max())


@pytest.mark.parametrize("case", ["uniform-p8", "clustered-p7-WXO", "nrhs2-p10"])
def test_second_approach_equals_first(orc, case):
    if case == "uniform-p8":
        w, p, s, wd = W.uniform_cube(2500, 1.0, 0.01, seed=141), 8, 30, 90
    elif case == "clustered-p7-WXO":
        w, p, s, wd = W.clustered(2500, 8, 8.0, 0.6, 0.3, 1, seed=142), 7, 20, 40
    else:
        w, p, s, wd = W.uniform_cube(2000, 1.0, 0.01, nrhs=2, seed=143), 10, 40, -1
    t = orc.Tree(w.pos, s, 14, w.a)
    if case.startswith("clustered"):
        assert all(len(t.lists[L][1]) > 0 for L in "WXO")
    u1 = orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, wd, eval_mode=0)
    u2 = orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, wd, eval_mode=1)
    assert orc.rel_l2(u2, u1) <= 1e-12
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    assert orc.rel_l2(u2, ref) <= 1e-3


def test_second_approach_converges(orc):
    w = W.clustered(2000, 10, 10.0, 1.0, 0.05, 1, seed=144)
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    errs = [orc.rel_l2(orc.fmm(w.pos, w.forces, w.a, w.eta, p, 25, -1, eval_mode=1), ref) for p in (2, 5, 8)]
    assert errs[1] < 0.3 * errs[0] and errs[2] < 0.3 * errs[1], errs
