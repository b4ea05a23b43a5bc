"""Pins for the oracle's four-Laplace FMM (O4): it must converge to the direct
RPY sum (O1) as the order p grows, reduce to it exactly with a single leaf,
and be linear in the forces, on uniform, clustered (W/X lists) and
small-leaf (O list) trees.  The order for a requested accuracy eps is the
calibration reading taken for the paper's unstated accuracy-to-order map.
W-list boxes may be evaluated through their multipoles (Theorem 1) or summed
directly with the far formula that the multipole approximates; both
branches are pinned against the direct sum, including a threshold that
splits the W boxes of one tree between them."""
import numpy as np
import pytest

import workloads as W


def test_single_leaf_is_direct(orc):
    w = W.uniform_cube(500, 1.0, 0.03, nrhs=2, seed=31)
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    u = orc.fmm(w.pos, w.forces, w.a, w.eta, 4, 10_000, -1)
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
    errs = [orc.rel_l2(orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, -1), ref) for p in (2, 6, 10, 14)]
    assert all(e1 < 0.5 * e0 for e0, e1 in zip(errs, errs[1:])), errs
    assert errs[-1] < 3e-5, errs


def test_multi_rhs_equals_separate_calls_and_linearity(orc):
    w = W.uniform_cube(1200, 1.0, 0.02, nrhs=3, seed=35)
    u = orc.fmm(w.pos, w.forces, w.a, w.eta, 6, 20, 40)
    for r in range(3):
        ur = orc.fmm(w.pos, w.forces[r], w.a, w.eta, 6, 20, 40)
        assert np.array_equal(ur, u[r])
    ul = orc.fmm(w.pos, 2.0 * w.forces[0] - w.forces[2], w.a, w.eta, 6, 20, 40)
    assert np.allclose(ul, 2.0 * u[0] - u[2], rtol=1e-12, atol=1e-13)


def test_translation_far_from_origin(orc):
    # Box-centred fourth charge: shifting all beads by a large offset
    # changes nothing but rounding.
    w = W.uniform_cube(1500, 1.0, 0.01, seed=36)
    u0 = orc.fmm(w.pos, w.forces, w.a, w.eta, 8, 25, 90)
    u1 = orc.fmm(w.pos + 1000.0, w.forces, w.a, w.eta, 8, 25, 90)
    assert orc.rel_l2(u1, u0) < 1e-11


def test_invalid_arguments(orc):
    pos = np.zeros((3, 3))
    F = np.zeros((3, 3))
    with pytest.raises(ValueError):
        orc.fmm(pos, F, -1.0, 1.0, 4, 10, -1)
    with pytest.raises(ValueError):
        orc.fmm(pos, F, 1.0, 1.0, 99, 10, -1)


def test_w_list_branches_converge_to_direct(orc):
    """Every W box through its multipole (w_direct = -1), every W box summed
    directly (w_direct huge), and a threshold at the median W-box size (the
    tree's W boxes split between the branches): all converge to the direct
    sum as p grows, and neither direct variant is worse than the
    all-multipole one."""
    w = W.clustered(3000, 12, 12.0, 1.0, 0.05, 1, seed=37)
    s = 20
    t = orc.Tree(w.pos, s, 14, w.a)
    wo, we = t.lists["W"]
    sizes = t.boxes[we, 5] - t.boxes[we, 4]
    assert len(sizes) > 20
    mid = int(np.median(sizes))
    assert (sizes <= mid).any() and (sizes > mid).any()
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    prev = None
    for p in (3, 7, 11):
        e_m = orc.rel_l2(orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, -1), ref)
        e_d = orc.rel_l2(orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, 10**9), ref)
        e_s = orc.rel_l2(orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, mid), ref)
        # summing a W box directly removes its truncation error
        assert e_d <= 1.05 * e_m and e_s <= 1.05 * e_m
        if prev is not None:
            assert e_m < 0.5 * prev[0] and e_d < 0.5 * prev[1] and e_s < 0.5 * prev[2]
        prev = (e_m, e_d, e_s)
    assert max(prev) < 1e-4

