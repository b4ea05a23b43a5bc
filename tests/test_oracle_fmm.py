"""Pins for the oracle's four-Laplace FMM (O4): it must converge to the direct
RPY sum (O1) as the order p grows, reduce to it exactly with a single leaf,
and be linear in the forces, on uniform, clustered (W/X lists) and
small-leaf (O list) trees.  The order for a requested accuracy eps is the
calibration reading taken for the paper's unstated accuracy-to-order map."""
import numpy as np
import pytest

import workloads as W


def test_single_leaf_is_direct(orc):
    w = W.uniform_cube(500, 1.0, 0.03, nrhs=2, seed=31)
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    u = orc.fmm(w.pos, w.forces, w.a, w.eta, 4, 10_000)
    assert orc.rel_l2(u, ref) < 1e-14


@pytest.mark.parametrize("case", ["uniform", "clustered", "overlap"])
def test_geometric_convergence(orc, case):
    if case == "uniform":
        w = W.uniform_cube(2500, 1.0, 0.01, seed=32)
        s = 30
    elif case == "clustered":
        w = W.clustered(2500, 15, 15.0, 1.0, 0.05, 1, seed=33)
        s = 25
    else:
        w = W.uniform_cube(2000, 1.0, 0.07, seed=34)
        s = 12
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    errs = [orc.rel_l2(orc.fmm(w.pos, w.forces, w.a, w.eta, p, s), ref) for p in (2, 6, 10, 14)]
    assert all(e1 < 0.5 * e0 for e0, e1 in zip(errs, errs[1:])), errs
    assert errs[-1] < 3e-5, errs


def test_multi_rhs_equals_separate_calls_and_linearity(orc):
    w = W.uniform_cube(1200, 1.0, 0.02, nrhs=3, seed=35)
    u = orc.fmm(w.pos, w.forces, w.a, w.eta, 6, 20)
    for r in range(3):
        ur = orc.fmm(w.pos, w.forces[r], w.a, w.eta, 6, 20)
        assert np.array_equal(ur, u[r])
    ul = orc.fmm(w.pos, 2.0 * w.forces[0] - w.forces[2], w.a, w.eta, 6, 20)
    assert np.allclose(ul, 2.0 * u[0] - u[2], rtol=1e-12, atol=1e-13)


def test_translation_far_from_origin(orc):
    # Box-centred fourth charge: shifting all beads by a large offset
    # changes nothing but rounding.
    w = W.uniform_cube(1500, 1.0, 0.01, seed=36)
    u0 = orc.fmm(w.pos, w.forces, w.a, w.eta, 8, 25)
    u1 = orc.fmm(w.pos + 1000.0, w.forces, w.a, w.eta, 8, 25)
    assert orc.rel_l2(u1, u0) < 1e-11


def test_invalid_arguments(orc):
    pos = np.zeros((3, 3))
    F = np.zeros((3, 3))
    with pytest.raises(ValueError):
        orc.fmm(pos, F, -1.0, 1.0, 4, 10)
    with pytest.raises(ValueError):
        orc.fmm(pos, F, 1.0, 1.0, 99, 10)
