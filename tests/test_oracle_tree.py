"""Pins for the oracle's adaptive octree (arXiv:1711.02976, Sec. 4.2: leaves
hold at most `threshold` beads) and the adaptive-FMM interaction lists.

The strongest pin is the coverage theorem of the adaptive FMM: for every
target leaf B, every source bead is reached exactly once through U(B), W(B),
or V(A) / X(A) of some A on the path from B to the root.  A wrong list
definition (a dropped or doubled box) fails it."""
import numpy as np
import pytest

import workloads as W


def _trees():
    out = []
    w = W.uniform_cube(2500, 1.0, 0.01, seed=21)
    out.append(("uniform", w.pos, 30, 14, w.a))
    w = W.clustered(3000, 12, 10.0, 0.7, 0.05, 1, seed=22)
    out.append(("clustered", w.pos, 20, 14, w.a))
    w = W.clustered(2000, 4, 50.0, 0.3, 0.5, 1, seed=23)
    out.append(("deep-overlap", w.pos, 8, 14, w.a))
    w = W.uniform_cube(1500, 1.0, 0.01, seed=24)
    out.append(("depth-capped", w.pos, 3, 2, w.a))
    return out


TREES = _trees()


@pytest.fixture(scope="module", params=range(len(TREES)), ids=[t[0] for t in TREES])
def tree(request, orc):
    name, pos, s, md, a = TREES[request.param]
    return name, pos, s, md, a, orc.Tree(pos, s, md, a)


def _adjacent(t, A, B):
    L = max(t.level[A], t.level[B])
    sa, sb = L - t.level[A], L - t.level[B]
    alo = t.anchor[A] << sa
    ahi = (t.anchor[A] + 1) << sa
    blo = t.anchor[B] << sb
    bhi = (t.anchor[B] + 1) << sb
    return bool(np.all(alo <= bhi) and np.all(blo <= ahi))


def test_partition_and_refinement(tree):
    name, pos, s, md, a, t = tree
    n = len(pos)
    assert sorted(t.perm.tolist()) == list(range(n))
    assert np.all(np.diff(t.keys.astype(np.uint64).view(np.int64)) >= 0) or np.all(t.keys[1:] >= t.keys[:-1])
    leaves = np.where(t.is_leaf())[0]
    cover = np.zeros(n, dtype=int)
    for b in leaves:
        cover[t.begin[b]:t.end[b]] += 1
        assert t.end[b] > t.begin[b]
        assert t.end[b] - t.begin[b] <= s or t.level[b] == md
    assert np.all(cover == 1)
    for b in np.where(~t.is_leaf())[0]:
        assert t.end[b] - t.begin[b] > s and t.level[b] < md
        kids = np.where(t.parent == b)[0]
        assert kids[0] == t.child_begin[b] and np.all(np.diff(kids) == 1)
        assert t.begin[kids[0]] == t.begin[b] and t.end[kids[-1]] == t.end[b]
        assert np.all(t.end[kids[:-1]] == t.begin[kids[1:]])
        assert np.all(t.level[kids] == t.level[b] + 1)
        assert np.all((t.anchor[kids] >> 1) == t.anchor[b])
    # boxes numbered by (level, Morton order of anchors)
    assert np.all(np.diff(t.level) >= 0)


def test_beads_lie_in_their_box(tree):
    name, pos, s, md, a, t = tree
    scale = 2.0 ** 21 / t.side
    q = np.minimum(np.floor((pos[t.perm] - t.lo) * scale), 2 ** 21 - 1).astype(np.int64)
    for b in range(t.nbox):
        sh = 21 - t.level[b]
        assert np.all((q[t.begin[b]:t.end[b]] >> sh) == t.anchor[b])


def test_list_definitions(tree):
    name, pos, s, md, a, t = tree
    leaf = t.is_leaf()
    for L in "UVWXO":
        off, ent = t.lists[L]
        for b in range(t.nbox):
            e = ent[off[b]:off[b + 1]]
            assert np.all(np.diff(e) > 0), "entries sorted by box id"
            for c in e:
                adj = _adjacent(t, b, c)
                if L == "U":
                    assert leaf[b] and leaf[c] and adj
                elif L == "V":
                    assert t.level[c] == t.level[b] and not adj
                    assert _adjacent(t, t.parent[b], t.parent[c])
                elif L == "W":
                    assert leaf[b] and t.level[c] > t.level[b] and not adj
                    assert _adjacent(t, t.parent[c], b)
                elif L == "X":
                    assert leaf[c] and t.level[c] < t.level[b] and not adj
                elif L == "O":
                    assert leaf[b] and leaf[c] and not adj
    # X is the transpose of W; U, V, O are symmetric
    def pairs(L):
        off, ent = t.lists[L]
        return {(b, int(c)) for b in range(t.nbox) for c in ent[off[b]:off[b + 1]]}
    assert pairs("X") == {(c, b) for (b, c) in pairs("W")}
    for L in "UVO":
        P = pairs(L)
        assert P == {(c, b) for (b, c) in P}


def test_coverage_exactly_once(tree):
    name, pos, s, md, a, t = tree
    n = len(pos)
    U, V, Wl, X = (t.lists[k] for k in "UVWX")
    for b in np.where(t.is_leaf())[0]:
        cnt = np.zeros(n, dtype=int)
        for c in U[1][U[0][b]:U[0][b + 1]]:
            cnt[t.begin[c]:t.end[c]] += 1
        for c in Wl[1][Wl[0][b]:Wl[0][b + 1]]:
            cnt[t.begin[c]:t.end[c]] += 1
        A = b
        while A >= 0:
            for c in V[1][V[0][A]:V[0][A + 1]]:
                cnt[t.begin[c]:t.end[c]] += 1
            for c in X[1][X[0][A]:X[0][A + 1]]:
                cnt[t.begin[c]:t.end[c]] += 1
            A = t.parent[A]
        assert np.all(cnt == 1), (name, b, np.unique(cnt))


def test_o_list_covers_every_overlap_outside_u(tree):
    name, pos, s, md, a, t = tree
    n = len(pos)
    leaf_of = np.empty(n, dtype=np.int64)
    for b in np.where(t.is_leaf())[0]:
        leaf_of[t.begin[b]:t.end[b]] = b
    sp = pos[t.perm]
    U = {(b, int(c)) for b in range(t.nbox) for c in t.lists["U"][1][t.lists["U"][0][b]:t.lists["U"][0][b + 1]]}
    O = {(b, int(c)) for b in range(t.nbox) for c in t.lists["O"][1][t.lists["O"][0][b]:t.lists["O"][0][b + 1]]}
    d = np.linalg.norm(sp[:, None] - sp[None], axis=-1) if n <= 3000 else None
    ii, jj = np.where(d < 2 * a)
    for i, j in zip(ii, jj):
        key = (int(leaf_of[i]), int(leaf_of[j]))
        assert key in U or key in O
    assert U.isdisjoint(O)


def test_coincident_beads_and_depth_cap(orc):
    pos = np.repeat(np.array([[0.5, 0.5, 0.5], [0.1, 0.9, 0.3]]), [50, 7], axis=0)
    t = orc.Tree(pos, 4, 14, 0.01)
    leaves = np.where(t.is_leaf())[0]
    assert sum(t.end[b] - t.begin[b] for b in leaves) == 57
    assert max(t.end[b] - t.begin[b] for b in leaves) == 50
    assert t.level.max() == 14
