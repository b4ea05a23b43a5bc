"""The seeded input generators (no GPU): shapes, determinism and the
structure each named workload promises (bead counts, geometry, density,
sampled targets)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import workloads as W  # noqa: E402


@pytest.mark.parametrize("cid", [1, 2, 3, 4, 5, 6])
def test_named_workloads_are_seeded_and_shaped(cid):
    w = W.config(cid, scale=1e-3 if cid != 1 else 1.0)
    v = W.config(cid, scale=1e-3 if cid != 1 else 1.0)
    assert np.array_equal(w.pos, v.pos) and np.array_equal(w.forces, v.forces)
    assert np.array_equal(w.sample, v.sample)
    assert w.pos.shape == (w.n, 3) and w.forces.shape == (w.nrhs, w.n, 3)
    assert np.isfinite(w.pos).all() and np.isfinite(w.forces).all()
    assert sum(w.counts) == w.n
    s = np.asarray(w.sample)
    assert s.min() >= 0 and s.max() < w.n and len(np.unique(s)) == len(s)
    assert w.nrhs == {1: 1, 2: 1, 3: 4, 4: 16, 5: 20, 6: 1}[cid]
    other = W.config(cid, scale=1e-3 if cid != 1 else 1.0, seed=7)
    assert not np.array_equal(other.pos, w.pos)


def test_cube_is_uniform_in_its_side():
    w = W.uniform_cube(200_000, 2.0, 0.01, seed=3)
    assert w.pos.min() >= 0.0 and w.pos.max() < 2.0
    # each octant holds about an eighth of the beads
    oct_ = (w.pos >= 1.0).astype(int) @ np.array([1, 2, 4])
    frac = np.bincount(oct_, minlength=8) / w.n
    assert np.abs(frac - 0.125).max() < 0.005


def test_sphere_beads_lie_on_the_surface_at_unit_density():
    w = W.config(6, scale=1e-3)
    r = np.sqrt(w.n / (4.0 * np.pi))
    d = np.linalg.norm(w.pos - r, axis=1)
    assert np.allclose(d, r, rtol=1e-12)
    # no hemisphere is favoured
    assert abs(np.mean(w.pos[:, 2] > r) - 0.5) < 0.05


def test_blob_counts_follow_zipf_and_sum_to_n():
    n, nb, seed = 10_000, 20, 4
    w = W.clustered(n, nb, 1000.0, 1.0, 0.5, 1, seed=seed)
    assert w.n == n
    # the centres are the generator's first draw; beads go to the nearest one
    centres = np.random.Generator(np.random.PCG64(seed)).uniform(0.0, 1000.0, size=(nb, 3))
    d2 = ((w.pos[:, None, :] - centres[None, :, :]) ** 2).sum(-1)
    got = np.bincount(d2.argmin(1), minlength=nb)
    # Zipf(1) shares n / (k H_nb), rounded by largest remainder
    raw = (1.0 / np.arange(1, nb + 1)) / (1.0 / np.arange(1, nb + 1)).sum() * n
    want = np.floor(raw).astype(int)
    want[np.argsort(-(raw - want), kind="stable")[: n - want.sum()]] += 1
    assert np.array_equal(got, want)
    # sigma = 1 around each centre
    r = np.sqrt(d2.min(1))
    assert abs(np.sqrt(np.mean(r ** 2) / 3.0) - 1.0) < 0.03


def test_batched_counts_are_log_uniform_in_range_and_systems_at_density():
    w = W.multi_system(64, 1000, 200_000, 0.1, 0.5, 2, seed=5)
    c = np.asarray(w.counts)
    assert len(c) == 64 and c.min() >= 1000 and c.max() <= 200_000 and c.sum() == w.n
    off = np.concatenate([[0], np.cumsum(c)])
    for k in range(64):
        p = w.pos[off[k]:off[k + 1]]
        side = (c[k] / 0.1) ** (1.0 / 3.0)
        assert p.min() >= 0.0 and p.max() < side
    # at most min(n_s, 500) sampled targets per system, each inside its system
    for k in range(64):
        s = w.sample[(w.sample >= off[k]) & (w.sample < off[k + 1])]
        assert len(s) == min(c[k], 500)
