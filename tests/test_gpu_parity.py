"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

  * tree, permutation and U/V/W/X/O lists: bit-exact (integers);
  * a single-leaf plan is the direct sum:           rel-L2 <= 1e-12 vs O1;
  * FP64 FMM vs the oracle FMM of the same order:  rel-L2 <= 1e-12 vs O4;
  * FP64 FMM at eps vs the direct sum:             rel-L2 <= eps   vs O1;
  * several right-hand sides equal separate calls, and the edge cases.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import gpu_matvec, log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _tree_cases():
    return [
        ("uniform", W.uniform_cube(2500, 1.0, 0.01, seed=21).pos, 30, 14, 0.01),
        ("clustered", W.clustered(3000, 12, 10.0, 0.7, 0.05, 1, seed=22).pos, 20, 14, 0.05),
        ("deep-overlap", W.clustered(2000, 4, 50.0, 0.3, 0.5, 1, seed=23).pos, 8, 14, 0.5),
        ("depth-capped", W.uniform_cube(1500, 1.0, 0.01, seed=24).pos, 3, 2, 0.01),
        ("ragged-20k", W.clustered(20_011, 40, 30.0, 1.0, 0.05, 1, seed=25).pos, 33, 14, 0.05),
    ]


@pytest.mark.parametrize("case", _tree_cases(), ids=lambda c: c[0])
def test_tree_and_lists_bit_exact(orc, case):
    import paper_1711_02976_amd as R
    name, pos, s, md, a = case
    log(f"tree case {name} n={len(pos)} s={s} max_depth={md}")
    ref = orc.Tree(pos, s, md, a)
    P = R.Plan(to_dev(pos), a, 1.0, 1e-3, leaf_size=s, max_depth=md)
    try:
        got = P.export()
        st = P.stats()
    finally:
        P.free()
    assert st["nbox"] == ref.nbox
    assert np.array_equal(got["keys"], ref.keys)
    assert np.array_equal(got["perm"], ref.perm)
    assert np.array_equal(got["boxes"], ref.boxes)
    for L in "UVWXO":
        assert np.array_equal(got["lists"][L][0], ref.lists[L][0]), L
        assert np.array_equal(got["lists"][L][1], ref.lists[L][1]), L


def test_batched_tree_matches_per_system(orc):
    import paper_1711_02976_amd as R
    w = W.multi_system(5, 200, 3000, 0.1, 0.5, 1, seed=41)
    log(f"batched tree counts={w.counts}")
    P = R.Plan(to_dev(w.pos), 0.5, 1.0, 1e-3, leaf_size=40, counts=w.counts)
    try:
        got = P.export()
    finally:
        P.free()
    boxes = got["boxes"]
    off = np.concatenate([[0], np.cumsum(w.counts)])
    # per-system renumbering: GPU machines are ordered by (level, system, key)
    for s in range(len(w.counts)):
        ref = orc.Tree(w.pos[off[s]:off[s + 1]], 40, 14, 0.5)
        mine = np.where((boxes[:, 4] >= off[s]) & (boxes[:, 5] <= off[s + 1]) & (boxes[:, 5] > boxes[:, 4]))[0]
        # roots of other systems can be empty only if count is 0 (not the case here)
        assert len(mine) == ref.nbox
        gid2loc = {int(g): i for i, g in enumerate(mine)}
        b = boxes[mine].copy()
        b[:, 4:6] -= off[s]
        b[:, 6] = [gid2loc.get(int(x), -1) for x in b[:, 6]]
        b[:, 7] = [gid2loc.get(int(x), -1) for x in b[:, 7]]
        assert np.array_equal(b, ref.boxes)
        assert np.array_equal(got["perm"][off[s]:off[s + 1]] - off[s], ref.perm)
        for L in "UVWXO":
            goff, gent = got["lists"][L]
            roff, rent = ref.lists[L]
            for i, g in enumerate(mine):
                e = [gid2loc[int(x)] for x in gent[goff[g]:goff[g + 1]]]
                assert e == list(rent[roff[i]:roff[i + 1]]), (s, L, i)


def test_single_leaf_is_direct(orc):
    w = W.uniform_cube(3000, 1.0, 0.02, nrhs=2, seed=51)
    log("single leaf n=3000")
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, leaf_size=10_000)
    assert st["nleaf"] == 1
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    assert orc.rel_l2(u, ref) <= 1e-12


def _fmm_cases():
    # (name, workload, order, leaf size, W-direct threshold given to both sides)
    return [
        ("uniform-p8", W.uniform_cube(6000, 1.0, 0.005, nrhs=1, seed=61), 8, 30, 90),
        ("uniform-p16-ragged", W.uniform_cube(4999, 1.0, 0.005, nrhs=1, seed=62), 16, 40, 306),
        ("clustered-p10-WX", W.clustered(5000, 15, 15.0, 1.0, 0.05, 1, seed=63), 10, 25, 132),
        ("clustered-p10-W-multipoles", W.clustered(5000, 15, 15.0, 1.0, 0.05, 1, seed=63), 10, 25, -1),
        ("clustered-p10-W-direct", W.clustered(5000, 15, 15.0, 1.0, 0.05, 1, seed=63), 10, 25, 10**6),
        ("overlap-p6-O", W.uniform_cube(3000, 1.0, 0.07, nrhs=2, seed=64), 6, 12, 56),
        ("far-origin-nrhs3", W.uniform_cube(3000, 1.0, 0.01, nrhs=3, seed=65), 9, 30, 110),
        ("nrhs5-chunks", W.clustered(2500, 8, 8.0, 0.8, 0.05, 5, seed=66), 7, 20, 72),
    ]


def assert_close(u, ref, rel, per_target, orc, what=""):
    """rel-L2 bound and a per-target bound: max_i |u_i - ref_i| <=
    per_target * max_i |ref_i| (3-vector norms, every right-hand side)."""
    err = orc.rel_l2(u, ref)
    d = np.linalg.norm(np.asarray(u) - np.asarray(ref), axis=-1).max()
    m = np.linalg.norm(np.asarray(ref), axis=-1).max()
    log(f"  {what} rel-L2 = {err:.3e}, max target error / max |ref| = {d / m:.3e}")
    assert err <= rel
    assert d <= per_target * m


@pytest.mark.parametrize("case", _fmm_cases(), ids=lambda c: c[0])
def test_fmm_fp64_matches_oracle_fmm(orc, case):
    name, w, p, s, wd = case
    pos = w.pos + (500.0 if name.startswith("far") else 0.0)
    log(f"fmm parity {name} n={w.n} nrhs={w.nrhs} p={p} s={s} w_direct={wd}")
    u, st = gpu_matvec(pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=s, w_direct=wd)
    ref = orc.fmm(pos, w.forces, w.a, w.eta, p, s, wd)
    log(f"  lists {st['list_len']}")
    assert_close(u, ref, 1e-12, 1e-11, orc, "vs oracle FMM")


# Leaves of several hundred beads, as the library's own leaf-size choice
# makes them on the benchmark workloads: P2P tiles of 128 beads and
# evaluation tiles of 64 beads span several tiles per leaf, the M->L runs in
# batches of 64 columns with the deepest level on its own stream, and on
# clustered beads the W, X and O lists are non-empty and some boxes' S->L
# work is split over several work items.
def _large_leaf_cases():
    return [
        ("uniform-s324-p16-nrhs1", W.uniform_cube(20_000, 2.0, 0.01, nrhs=1, seed=111), 16, 324, 306, False),
        ("uniform-s729-p21-nrhs4", W.uniform_cube(24_000, 2.0, 0.01, nrhs=4, seed=112), 21, 729, 506, False),
        ("clustered-s324-p16-nrhs4", W.clustered(40_000, 20, 30.0, 1.0, 0.5, 4, seed=113), 16, 324, 306, True),
        ("clustered-s729-p21-nrhs1", W.clustered(40_000, 20, 30.0, 1.0, 0.5, 1, seed=114), 21, 729, 506, True),
    ]


_large_ref = {}


@pytest.mark.parametrize("case", _large_leaf_cases(), ids=lambda c: c[0])
def test_large_leaves_match_oracle_fmm(orc, case):
    name, w, p, s, wd, adaptive = case
    log(f"large-leaf parity {name} n={w.n} nrhs={w.nrhs} p={p} s={s}")
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=s, w_direct=wd)
    L = st["list_len"]
    log(f"  depth={st['depth']} nleaf={st['nleaf']} lists {L} p2l items={st['p2l_items']} "
        f"split boxes={st['p2l_split_boxes']}")
    assert L["V"] > 0
    if adaptive:
        assert L["W"] > 0 and L["X"] > 0 and L["O"] > 0
        assert st["p2l_split_boxes"] > 0
    ref = orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, wd)
    _large_ref[name] = ref
    assert_close(u, ref, 1e-12, 1e-11, orc, "FP64 vs oracle FMM")
    # the mixed form on the same plan: FP32 pair sums and M->L against the
    # FP64 GPU result, within half the accuracy setting (1e-6)
    um, _ = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=s, w_direct=wd, precision="mixed")
    assert_close(um, u, 5e-7, 1e-5, orc, "mixed vs FP64")


# 16 right-hand sides per near-field group: the P2P runs on the matrix cores
# (9 16x16x4 products per 4-source step, pair blocks formed per lane); the
# right-hand sides past 16 form groups of 8, 4, 2 or 1 on the vector units.
# A single leaf is the direct sum: every tile of 128 targets (the last one
# ragged, so some waves hold fewer than 16 targets and some none), with self
# terms and overlapping pairs.  In the FP64 form 16 + x right-hand sides take
# x = 1, 2, 4 or 8 of them on the vector units of the matrix-core launch, and
# 26 and 40 run 16 + 8 then 2, and 16 then 16 + 8; the mixed form runs 16 on
# the matrix cores and the rest in the vector kernel.
@pytest.mark.parametrize("nrhs", [16, 17, 18, 20, 24, 26, 40])
def test_matrix_core_p2p_single_leaf_is_direct(orc, nrhs):
    w = W.uniform_cube(3000, 1.0, 0.02, nrhs=nrhs, seed=52)
    log(f"single leaf n=3000 nrhs={nrhs} (matrix-core P2P)")
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, leaf_size=10_000)
    assert st["nleaf"] == 1
    assert_close(u, ref, 1e-12, 1e-11, orc, "FP64 vs direct")
    um, _ = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, leaf_size=10_000, precision="mixed")
    assert_close(um, ref, 1e-6, 1e-5, orc, "mixed vs direct")


# The whole FMM with a near-field group of 16 right-hand sides against the
# oracle FMM: large uniform leaves (20 rhs: groups of 16 and 4), and a
# clustered set with overlapping pairs outside U, W and X lists and 16 rhs
# (overlap and direct W sums then run as two launches of 8).
def _matrix_core_cases():
    return [
        ("uniform-s324-p12-nrhs20", W.uniform_cube(12_000, 2.0, 0.01, nrhs=20, seed=115), 12, 324, False),
        ("clustered-s200-p10-nrhs16", W.clustered(20_000, 20, 30.0, 1.0, 0.5, 16, seed=116), 10, 200, True),
    ]


@pytest.mark.parametrize("case", _matrix_core_cases(), ids=lambda c: c[0])
def test_matrix_core_p2p_fmm_matches_oracle_fmm(orc, case):
    name, w, p, s, adaptive = case
    wd = (p + 1) * (p + 2)
    log(f"matrix-core P2P parity {name} n={w.n} nrhs={w.nrhs} p={p} s={s}")
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=s, w_direct=wd)
    L = st["list_len"]
    log(f"  depth={st['depth']} nleaf={st['nleaf']} lists {L}")
    if adaptive:
        assert L["W"] > 0 and L["X"] > 0 and L["O"] > 0
    ref = orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, wd)
    assert_close(u, ref, 1e-12, 1e-11, orc, "FP64 vs oracle FMM")
    um, _ = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=s, w_direct=wd, precision="mixed")
    assert_close(um, u, 5e-7, 1e-5, orc, "mixed vs FP64")


def test_fp64_matvec_is_bitwise_reproducible(orc):
    """FP64 matvecs on an adaptive tree with split S->L work are bitwise
    equal from call to call and from plan to plan (the split shares are
    added in a fixed order)."""
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    w = W.clustered(40_000, 20, 30.0, 1.0, 0.5, 2, seed=113)
    log("bitwise reproducibility n=40000 s=324 p=16")
    F = to_dev(w.forces)
    outs = []
    for _ in range(2):
        P = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, leaf_size=324, order=16)
        try:
            assert P.stats()["p2l_split_boxes"] > 0
            for _ in range(2):
                outs.append(P.matvec(F).cpu().numpy())
        finally:
            P.free()
    torch.cuda.synchronize()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


# (order, rhs) pairs that reach every particle-to-expansion schedule: 8 steps
# per wave and pass over 1..4 passes (one or two right-hand sides per pass)
# and, with four right-hand sides per pass, 8 steps over 1..2 passes or 16
# steps over 2; above order 21 (the 9-digit setting) one right-hand side per
# pass over 5..7 passes; the tree has W and X lists.
@pytest.mark.parametrize("p,nrhs", [(1, 3), (7, 4), (14, 3), (15, 4), (18, 2), (19, 1), (21, 4), (24, 2), (27, 3)],
                         ids=lambda v: str(v))
def test_schedules_match_oracle_fmm(orc, p, nrhs):
    w = W.clustered(1500, 8, 10.0, 0.8, 0.05, nrhs, seed=80 + p)
    wd = (p + 1) * (p + 2)
    log(f"schedule parity n={w.n} nrhs={nrhs} p={p} s=20 w_direct={wd}")
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=20, w_direct=wd)
    assert st["list_len"]["X"] > 0 and st["list_len"]["W"] > 0
    ref = orc.fmm(w.pos, w.forces, w.a, w.eta, p, 20, wd)
    err = orc.rel_l2(u, ref)
    log(f"  rel-L2 vs oracle FMM = {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_fmm_fp64_accuracy_vs_direct(orc, eps):
    w = W.uniform_cube(20_000, 2.0, 0.01, nrhs=1, seed=71)
    log(f"accuracy n=20000 eps={eps}")
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, eps, leaf_size=60)
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    err = orc.rel_l2(u, ref)
    log(f"  p={st['order']} rel-L2 vs direct = {err:.3e}")
    assert err <= eps


@pytest.mark.parametrize("precision,bound,a", [("fp64", 1e-12, 1e-9), ("mixed", 1e-6, 1e-9),
                                              ("fp64", 1e-12, 1e-10), ("mixed", 1e-6, 1e-10)])
def test_si_units_small_beads(orc, precision, bound, a):
    # SI-like units (a = 1 nm or 1 Angstrom, positions over 20 a, water
    # viscosity): the pair kernels scale lengths so that 2a is of order one,
    # and their floor on r^2 must leak neither into the far pairs, the self
    # term nor the overlap branch; one leaf, so the matvec is the exact pair
    # sum
    g = np.random.default_rng(17)
    n, eta = 300, 1e-3
    pos = g.uniform(0.0, 20 * a, size=(n, 3))
    F = g.standard_normal((1, n, 3)) * 1e-12
    log(f"SI units n={n} a={a} {precision}")
    u, st = gpu_matvec(pos, F, a, eta, 1e-6, leaf_size=1000, precision=precision)
    ref = orc.rpy_direct(pos, F, a, eta)
    assert_close(u, ref, bound, 10 * bound, orc, "vs direct")


def test_si_units_fmm_matches_oracle_fmm(orc):
    # the same scale through the whole FMM (tree, expansions, overlap list)
    # (4000 beads in a cube of side 12a: leaves of 8 beads at depth 3 have
    # side 1.5a < 2a, so non-adjacent leaves can hold overlapping pairs)
    g = np.random.default_rng(18)
    n, a, eta = 4000, 1e-10, 1e-3
    pos = g.uniform(0.0, 12 * a, size=(n, 3))
    F = g.standard_normal((1, n, 3)) * 1e-12
    log(f"SI units FMM n={n} a={a}")
    u, st = gpu_matvec(pos, F, a, eta, 1e-6, leaf_size=10, order=10, w_direct=132)
    assert st["list_len"]["O"] > 0
    ref = orc.fmm(pos, F, a, eta, 10, 10, 132)
    assert_close(u, ref, 1e-12, 1e-11, orc, "vs oracle FMM")


@pytest.mark.parametrize("case", [(115, 20_000, 40, True), (117, 40_000, 60, False)],
                         ids=["n20000-s40", "n40000-s60"])
def test_deep_overlap_mixed_against_fp64(orc, case):
    """Leaves much smaller than the bead radius (dense clusters): many
    overlapping pairs fall in the O list, whose correction the mixed form
    evaluates in FP32 in a factored form free of cancellation.  The terms it
    removes are up to tens of self mobilities, so its FP32 rounding adds to
    that of the FP32 M->L on the same large terms: the mixed form is held to
    its accuracy target, eps against the FP64 direct sum (and eps against the
    FP64 FMM), target by target as well."""
    seed, n, s, fmm = case
    w = W.clustered(n, 4, 40.0, 0.4, 0.5, 2, seed=seed)
    log(f"deep overlap n={n} s={s}, order 12: mixed vs fp64")
    ud, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, leaf_size=s, order=12, w_direct=182)
    um, _ = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, leaf_size=s, order=12, w_direct=182,
                       precision="mixed")
    log(f"  depth={st['depth']} O={st['list_len']['O']}")
    assert st["list_len"]["O"] > 0
    assert_close(um, ud, 1e-6, 1e-5, orc, "mixed vs FP64")
    if fmm:
        ref = orc.fmm(w.pos, w.forces, w.a, w.eta, 12, s, 182)
        assert_close(ud, ref, 1e-12, 1e-11, orc, "FP64 vs oracle FMM")
    # the plan the library chooses for eps = 1e-6 (leaf size and order), both
    # forms against the direct sum
    direct = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    for prec in ("fp64", "mixed"):
        u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, precision=prec)
        log(f"  {prec} p={st['order']} s={st['leaf_size']} O={st['list_len']['O']}")
        assert_close(u, direct, 1e-6, 2e-5, orc, f"{prec} vs direct")


def test_nine_digit_setting_vs_direct(orc):
    # eps below 1e-8 selects the highest order built (27): the paper's 9-digit
    # setting, FP64, on uniform beads (level-uniform tree) and clustered beads
    # (adaptive tree, W and X lists)
    w = W.uniform_cube(20_000, 2.0, 0.01, nrhs=1, seed=71)
    log("9-digit setting n=20000 uniform eps=1e-9")
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-9, leaf_size=60)
    err = orc.rel_l2(u, orc.rpy_direct(w.pos, w.forces, w.a, w.eta))
    log(f"  p={st['order']} rel-L2 vs direct = {err:.3e}")
    assert st["order"] == 27 and err <= 3.5e-9
    w = W.clustered(20_000, 30, 30.0, 1.0, 0.5, 2, seed=72)
    log("9-digit setting n=20000 clustered eps=1e-9, 2 rhs")
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-9, leaf_size=40)
    err = orc.rel_l2(u, orc.rpy_direct(w.pos, w.forces, w.a, w.eta))
    log(f"  p={st['order']} W={st['list_len']['W']} rel-L2 vs direct = {err:.3e}")
    assert st["order"] == 27 and st["list_len"]["W"] > 0 and err <= 1e-8


def test_clustered_accuracy_vs_direct(orc):
    w = W.clustered(20_000, 30, 30.0, 1.0, 0.5, 1, seed=72)
    log("clustered accuracy n=20000 eps=1e-6 (O list active)")
    u, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, leaf_size=40)
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    err = orc.rel_l2(u, ref)
    log(f"  p={st['order']} lists={st['list_len']} rel-L2 = {err:.3e}")
    assert st["list_len"]["O"] > 0
    assert err <= 1e-6


def test_multi_rhs_equals_separate_calls(orc):
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    # 11 right-hand sides: near-field groups of 8, 2 and 1, far-field passes
    # of 4, 4, 2 and 1
    w = W.uniform_cube(4000, 1.0, 0.01, nrhs=11, seed=81)
    log("nrhs=11 vs 11 single calls")
    P = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, leaf_size=40)
    try:
        F = to_dev(w.forces)
        U = P.matvec(F).cpu().numpy()
        for r in range(11):
            ur = P.matvec(F[r]).cpu().numpy()
            assert orc.rel_l2(ur, U[r]) <= 1e-14
        torch.cuda.synchronize()
    finally:
        P.free()


def test_twenty_rhs_equal_separate_calls(orc):
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    # 20 right-hand sides: near-field groups of 16 (matrix cores) and 4;
    # single calls run the vector kernels, so the sums differ in order only
    w = W.uniform_cube(4000, 1.0, 0.01, nrhs=20, seed=82)
    log("nrhs=20 vs 20 single calls")
    P = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, leaf_size=40)
    try:
        F = to_dev(w.forces)
        U = P.matvec(F).cpu().numpy()
        for r in range(20):
            ur = P.matvec(F[r]).cpu().numpy()
            assert orc.rel_l2(ur, U[r]) <= 1e-13
        torch.cuda.synchronize()
    finally:
        P.free()


def test_repeated_and_overlapping_plans_agree(orc):
    # later plans reuse the cached translation tables: a plan built again on
    # the same beads gives the same
    # velocities (up to the order of atomic FP64 sums in the adaptive
    # S->L pass), also while plans of other orders are alive
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    w = W.uniform_cube(6000, 1.0, 0.01, nrhs=2, seed=83)
    log("repeated and overlapping plans")
    F = to_dev(w.forces)
    pos = to_dev(w.pos)

    def once(order):
        P = R.Plan(pos, w.a, w.eta, 1e-6, leaf_size=60, order=order)
        try:
            u = P.matvec(F)
            torch.cuda.synchronize()
            return u.cpu().numpy()
        finally:
            P.free()

    first = {o: once(o) for o in (9, 16)}
    alive = [R.Plan(pos, w.a, w.eta, 1e-6, leaf_size=60, order=o) for o in (16, 9, 16)]
    try:
        outs = [P.matvec(F) for P in alive]
        torch.cuda.synchronize()
        for o, u in zip((16, 9, 16), outs):
            assert orc.rel_l2(u.cpu().numpy(), first[o]) <= 1e-14
    finally:
        for P in alive:
            P.free()
    for o in (16, 9):
        assert orc.rel_l2(once(o), first[o]) <= 1e-14
    assert orc.rel_l2(first[16], orc.rpy_direct(w.pos, w.forces, w.a, w.eta)) <= 1e-6


def test_edge_cases(orc):
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    log("edge cases")
    # n = 0: valid, no-op
    P = R.Plan(torch.zeros((0, 3), dtype=torch.float64, device="cuda"), 0.5)
    P.matvec(torch.zeros((1, 0, 3), dtype=torch.float64, device="cuda"))
    P.free()
    # n = 1: F / (6 pi eta a)
    u, _ = gpu_matvec(np.array([[0.3, -2.0, 5.0]]), np.array([[[1.0, 2.0, -3.0]]]), 0.25, 2.0)
    assert np.allclose(u[0, 0], np.array([1.0, 2.0, -3.0]) / (6 * np.pi * 2.0 * 0.25), rtol=1e-14)
    # coincident beads and a max-depth leaf holding many of them
    pos = np.repeat(np.array([[0.5, 0.5, 0.5], [0.1, 0.9, 0.3], [0.7, 0.2, 0.8]]), [300, 7, 1], axis=0)
    F = np.random.default_rng(3).normal(size=(1, len(pos), 3))
    u, st = gpu_matvec(pos, F, 0.05, 1.0, 1e-6, leaf_size=4)
    ref = orc.rpy_direct(pos, F, 0.05, 1.0)
    assert orc.rel_l2(u, ref) <= 1e-6
    # non-finite position
    bad = np.zeros((5, 3))
    bad[2, 1] = np.nan
    with pytest.raises(R.RpyError) as ei:
        R.Plan(to_dev(bad), 0.5)
    assert ei.value.status == R.RPY_ENONFINITE
    with pytest.raises(R.RpyError):
        R.Plan(to_dev(np.zeros((5, 3))), -0.5)


@pytest.mark.parametrize("phase", ["p2p", "m2l", "l2l", "unpermute"])
def test_failed_phase_makes_the_plan_sticky(orc, phase):
    """A HIP error reported at a phase (forced from the host; no kernel
    fails) stops the pass there, rpy_matvec returns RPY_EDEVICE, and the
    plan stays in the error state; other plans are unaffected."""
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    w = W.uniform_cube(3000, 1.0, 0.01, nrhs=1, seed=121)
    log(f"injected failure at {phase}")
    P = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, leaf_size=40)
    Q = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, leaf_size=40)
    try:
        F = to_dev(w.forces)
        good = P.matvec(F).cpu().numpy()
        with pytest.raises(ValueError):
            P.inject_error(99)
        P.inject_error(phase)
        with pytest.raises(R.RpyError) as ei:
            P.matvec(F)
        assert ei.value.status == R.RPY_EDEVICE
        with pytest.raises(R.RpyError) as ei:
            P.matvec(F)
        assert ei.value.status == R.RPY_EDEVICE
        torch.cuda.synchronize()
        assert np.array_equal(Q.matvec(F).cpu().numpy(), good)
    finally:
        P.free()
        Q.free()


def test_failed_workspace_allocation_leaves_the_plan_usable(orc):
    """An allocation failure of the matvec workspace (forced from the host,
    half-way through its arrays) returns RPY_ENOMEM before any work is
    issued and leaves the velocities unwritten; the plan stays usable and
    its next call gives what a plan that never failed gives.  A call that
    needs no new workspace leaves the injection pending."""
    import ctypes as C
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    w = W.uniform_cube(3000, 1.0, 0.01, nrhs=4, seed=122)
    log("injected workspace allocation failure")
    P = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, leaf_size=40)
    Q = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, leaf_size=40)
    try:
        F = to_dev(w.forces)

        def raw(nrhs, U):
            return R.lib().rpy_matvec(P.handle, nrhs, C.c_void_p(F.data_ptr()), C.c_void_p(U.data_ptr()))

        U1 = torch.empty_like(F[:1])
        assert raw(1, U1) == R.RPY_OK  # workspace for one right-hand side
        P.inject_error("alloc")
        assert raw(1, U1) == R.RPY_OK  # no new workspace needed: still pending
        U4 = torch.full_like(F, float("nan"))
        assert raw(4, U4) == R.RPY_ENOMEM
        assert b"workspace" in R.lib().rpy_last_error()
        torch.cuda.synchronize()
        assert torch.isnan(U4).all()
        assert raw(4, U4) == R.RPY_OK
        torch.cuda.synchronize()
        assert np.array_equal(U4.cpu().numpy(), Q.matvec(F).cpu().numpy())
        # one right-hand side alone runs other kernels than a pass of four
        assert orc.rel_l2(U1.cpu().numpy(), U4[:1].cpu().numpy()) <= 1e-13
    finally:
        P.free()
        Q.free()


def test_fullsize_cube_1M_sampled(orc):
    """1,000,000 beads, cube side 100, a = 0.5: FP64 FMM at eps = 1e-6 against
    the direct sum on 2,000 sampled targets."""
    torch = torch_cuda()
    w = W.config(2, nsample=2000)
    log(f"full size {w.name} n={w.n} eps=1e-6")
    import paper_1711_02976_amd as R
    P = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6)
    try:
        u = P.matvec(to_dev(w.forces)).cpu().numpy()
        st = P.stats()
    finally:
        P.free()
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta, targets=w.sample)
    err = orc.rel_l2(u[:, w.sample], ref)
    log(f"  p={st['order']} s={st['leaf_size']} nbox={st['nbox']} rel-L2 (2000 targets) = {err:.3e}")
    assert err <= 1e-6


@pytest.mark.parametrize("p", [4, 13, 21, 27])
def test_m2l_rotation_matches_dense(orc, p):
    """The rotation-based M->L and the dense O(p^4) M->L compute the same
    truncated operator; both match the oracle FMM."""
    w = W.clustered(4000, 10, 10.0, 0.8, 0.05, 2, seed=91)
    log(f"m2l modes p={p}")
    ud, _ = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=30, m2l="dense")
    ur, _ = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=30, m2l="rotation")
    err = orc.rel_l2(ur, ud)
    log(f"  rotation vs dense rel-L2 = {err:.3e}")
    assert err <= 1e-12
    if p <= 13:
        ref = orc.fmm(w.pos, w.forces, w.a, w.eta, p, 30, (p + 1) * (p + 2))
        assert orc.rel_l2(ur, ref) <= 1e-12


@pytest.mark.parametrize("case", ["uniform-p16-offset", "uniform-p7-offset", "clustered-p20", "nrhs5"])
def test_mixed_precision_accuracy(orc, case):
    """Mixed form (FP32 near field and M->L, FP64 expansions and sums):
    error against the FP64 direct sum within the requested eps, and close to
    the FP64 FMM of the same plan."""
    if case == "uniform-p16-offset":
        w, eps, s = W.uniform_cube(20_000, 2.0, 0.01, nrhs=1, seed=101), 1e-6, 60
    elif case == "uniform-p7-offset":
        w, eps, s = W.uniform_cube(20_000, 2.0, 0.01, nrhs=2, seed=102), 1e-3, 60
    elif case == "clustered-p20":
        w, eps, s = W.clustered(20_000, 30, 30.0, 1.0, 0.5, 1, seed=103), 1e-6, 40
    else:
        w, eps, s = W.uniform_cube(8_000, 1.5, 0.01, nrhs=5, seed=104), 1e-6, 50
    log(f"mixed {case} n={w.n} nrhs={w.nrhs} eps={eps}")
    um, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, eps, leaf_size=s, precision="mixed")
    ud, _ = gpu_matvec(w.pos, w.forces, w.a, w.eta, eps, leaf_size=s, precision="fp64")
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    e_mix, e_fp64, e_rel = orc.rel_l2(um, ref), orc.rel_l2(ud, ref), orc.rel_l2(um, ud)
    log(f"  p={st['order']} mixed vs direct {e_mix:.3e}, fp64 vs direct {e_fp64:.3e}, mixed vs fp64 {e_rel:.3e}")
    assert e_mix <= eps
    assert e_rel <= max(3e-7, 0.5 * eps)


# The two evaluation approaches of Sec. 2 (after Theorem 2): derivative sets
# per Laplace expansion (first) and one pre-assembled polynomial per velocity
# component and leaf (second), each against the oracle FMM with the same
# approach and against each other on the same plan.
@pytest.mark.parametrize("case", [("uniform-p7", 7, 60, False), ("clustered-p12-WXO", 12, 40, True),
                                  ("large-leaf-p16", 16, 324, True), ("clustered-p21-nrhs4", 21, 200, True)],
                         ids=lambda c: c[0])
def test_evaluation_approaches_match_oracle(orc, case):
    name, p, s, clustered = case
    if name == "uniform-p7":
        w = W.uniform_cube(20_000, 2.0, 0.01, nrhs=2, seed=151)
    elif name == "clustered-p12-WXO":
        w = W.clustered(20_000, 12, 25.0, 1.0, 0.5, 1, seed=152)
    elif name == "large-leaf-p16":
        w = W.clustered(40_000, 20, 30.0, 1.0, 0.5, 1, seed=153)
    else:
        w = W.clustered(10_000, 8, 15.0, 0.8, 0.5, 4, seed=154)
    wd = (p + 1) * (p + 2)
    log(f"evaluation approaches {name} n={w.n} nrhs={w.nrhs} p={p} s={s}")
    up, st = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=s, w_direct=wd, eval_mode="poly")
    us, st2 = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=s, w_direct=wd, eval_mode="sets")
    assert st["eval_mode"] == "poly" and st2["eval_mode"] == "sets"
    if clustered:
        assert all(st["list_len"][L] > 0 for L in "WXO")
    ref2 = orc.fmm(w.pos, w.forces, w.a, w.eta, p, s, wd, eval_mode=1)
    assert_close(up, ref2, 1e-12, 1e-11, orc, "polynomial evaluation vs oracle (second approach)")
    assert_close(us, ref2, 1e-12, 1e-11, orc, "set evaluation vs oracle (second approach)")
    assert_close(up, us, 1e-12, 1e-11, orc, "polynomial vs set evaluation")
    um, _ = gpu_matvec(w.pos, w.forces, w.a, w.eta, 1e-6, order=p, leaf_size=s, w_direct=wd, eval_mode="poly",
                       precision="mixed")
    assert_close(um, up, 5e-7, 1e-5, orc, "mixed vs FP64 (polynomial evaluation)")


def test_polynomial_evaluation_limits(orc):
    import paper_1711_02976_amd as R
    torch_cuda()
    w = W.uniform_cube(2000, 1.0, 0.01, seed=155)
    with pytest.raises(R.RpyError) as ei:
        R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, order=24, eval_mode="poly")
    assert ei.value.status == R.RPY_EUNSUPPORTED
    P = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-3, leaf_size=40)
    try:
        st = P.stats()
        assert st["eval_mode"] == ("poly" if st["order"] <= 10 else "sets")
    finally:
        P.free()


def test_autotuner_measures_gates_and_caches(orc):
    """tune = 1: the plan's leaf size, order and evaluation approach are
    chosen by timing candidate plans, each gated on its measured error
    against an FP64 direct sum at sampled targets (eps / 2); the tuned plan
    meets eps against the oracle's direct sum, and a second plan of the same
    class is served from the cache with the same choices."""
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    w = W.uniform_cube(30_000, 3.0, 0.02, nrhs=2, seed=161)
    log("autotuner n=30000 eps=1e-6 nrhs=2")
    F = to_dev(w.forces)
    P = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, tune=1, nrhs=2)
    try:
        st = P.stats()
        u = P.matvec(F).cpu().numpy()
    finally:
        P.free()
    log(f"  tuned: s={st['leaf_size']} p={st['order']} eval={st['eval_mode']} measured err={st['tune_err']:.2e} "
        f"plan {st['plan_ms']:.0f} ms")
    assert st["tuned"] == "measured" and 0 < st["tune_err"] <= 0.5e-6
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
    err = orc.rel_l2(u, ref)
    log(f"  rel-L2 vs oracle direct = {err:.3e}")
    assert err <= 1e-6
    P2 = R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, tune=1, nrhs=2)
    try:
        st2 = P2.stats()
    finally:
        P2.free()
    assert st2["tuned"] == "cached"
    assert (st2["leaf_size"], st2["order"], st2["eval_mode"]) == (st["leaf_size"], st["order"], st["eval_mode"])
    assert st2["plan_ms"] < st["plan_ms"]
    torch.cuda.synchronize()


def test_batched_matvec_equals_per_system_matvecs(orc):
    """One plan over several independent systems (uneven sizes, one of a
    single bead) gives each system's velocities as its own plan does, to
    1e-14 in FP64: the systems share launches but no interactions."""
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    g = np.random.default_rng(171)
    counts = [3000, 500, 8000, 1, 2000]
    parts = [g.uniform(0.0, (c / 0.5) ** (1 / 3), size=(c, 3)) for c in counts]
    pos = np.concatenate(parts)
    F = g.standard_normal((3, len(pos), 3))
    log(f"batched vs per-system matvecs counts={counts} nrhs=3")
    P = R.Plan(to_dev(pos), 0.5, 1.0, 1e-6, leaf_size=40, order=10, counts=counts)
    try:
        ub = P.matvec(to_dev(F)).cpu().numpy()
    finally:
        P.free()
    off = np.concatenate([[0], np.cumsum(counts)])
    for s in range(len(counts)):
        Ps = R.Plan(to_dev(parts[s]), 0.5, 1.0, 1e-6, leaf_size=40, order=10)
        try:
            us = Ps.matvec(to_dev(F[:, off[s]:off[s + 1]])).cpu().numpy()
        finally:
            Ps.free()
        err = orc.rel_l2(ub[:, off[s]:off[s + 1]], us)
        log(f"  system {s} ({counts[s]} beads): rel-L2 batched vs own plan = {err:.3e}")
        assert err <= 1e-14
    torch.cuda.synchronize()
