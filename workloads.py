"""Seeded synthetic inputs for the RPY mobility matvec.

Shared by the tests, the benchmark and the smoke check; it holds none of the
method's arithmetic (no RPY tensor, no expansions), only random inputs.
The paper's workloads are synthetic (arXiv:1711.02976, Sec. 4.3: uniform beads
in a cube, uniform on a sphere surface); the five named configurations restate
the cube workload and add clustered, multi-system and multi-right-hand-side
variants at the sizes the benchmark uses.

RNG: ``numpy.random.Generator(PCG64(seed))``, default seed 1000 + config id.
Draw order: positions, then forces ``standard_normal((nrhs, N, 3))``, then the
sampled target indices ``choice(N, k, replace=False)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    pos: np.ndarray            # [N, 3] float64 (systems concatenated)
    forces: np.ndarray         # [nrhs, N, 3] float64
    a: float
    eta: float
    eps: float
    sample: np.ndarray         # target indices used for error checks
    counts: list = field(default_factory=list)  # per-system bead counts
    max_depth: int = 14

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def nrhs(self) -> int:
        return int(self.forces.shape[0])


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_cube(n, side, a, nrhs=1, eps=1e-6, seed=0, nsample=None, name="cube", eta=1.0):
    g = _rng(seed)
    pos = g.uniform(0.0, side, size=(n, 3))
    F = g.standard_normal((nrhs, n, 3))
    k = n if nsample is None else min(n, nsample)
    sample = np.arange(n) if k == n else np.sort(g.choice(n, k, replace=False))
    return Workload(name, pos, F, a, eta, eps, sample, [n])


def sphere_surface(n, radius, a, nrhs=1, eps=1e-6, seed=0, nsample=None, name="sphere"):
    g = _rng(seed)
    v = g.standard_normal((n, 3))
    pos = radius * v / np.linalg.norm(v, axis=1, keepdims=True) + radius
    F = g.standard_normal((nrhs, n, 3))
    k = n if nsample is None else min(n, nsample)
    sample = np.arange(n) if k == n else np.sort(g.choice(n, k, replace=False))
    return Workload(name, pos, F, a, 1.0, eps, sample, [n])


def clustered(n, nblobs, side, sigma, a, nrhs, eps=1e-6, seed=0, nsample=None, name="blobs"):
    """Gaussian blobs with Zipf (exponent 1) counts scaled to n by largest
    remainder; beads are centre + N(0, sigma^2) per axis, globally shuffled."""
    g = _rng(seed)
    centres = g.uniform(0.0, side, size=(nblobs, 3))
    w = 1.0 / np.arange(1, nblobs + 1)
    raw = w / w.sum() * n
    cnt = np.floor(raw).astype(np.int64)
    rem = n - int(cnt.sum())
    order = np.argsort(-(raw - cnt), kind="stable")
    cnt[order[:rem]] += 1
    pos = np.repeat(centres, cnt, axis=0) + sigma * g.standard_normal((n, 3))
    pos = pos[g.permutation(n)]
    F = g.standard_normal((nrhs, n, 3))
    k = n if nsample is None else min(n, nsample)
    sample = np.arange(n) if k == n else np.sort(g.choice(n, k, replace=False))
    return Workload(name, pos, F, a, 1.0, eps, sample, [n])


def multi_system(nsys, nmin, nmax, density, a, nrhs, eps=1e-6, seed=0, per_sys_sample=500,
                 name="batched"):
    """Independent systems with log-uniform bead counts, each uniform in its
    own cube of the given bead density; positions concatenated."""
    g = _rng(seed)
    counts = np.round(np.exp(g.uniform(np.log(nmin), np.log(nmax), size=nsys))).astype(np.int64)
    parts = []
    for c in counts:
        side = (c / density) ** (1.0 / 3.0)
        parts.append(g.uniform(0.0, side, size=(int(c), 3)))
    pos = np.concatenate(parts)
    n = pos.shape[0]
    F = g.standard_normal((nrhs, n, 3))
    samp = []
    off = 0
    for c in counts:
        k = int(min(c, per_sys_sample))
        samp.append(off + np.sort(g.choice(int(c), k, replace=False)))
        off += int(c)
    return Workload(name, pos, F, a, 1.0, eps, np.concatenate(samp), [int(c) for c in counts])


def config(cid: int, scale: float = 1.0, seed=None, nsample=None):
    """The named workloads (1-5, and 6: 8M beads on a sphere surface);
    `scale` < 1 shrinks the bead count while keeping the bead density (cube
    sides shrink by scale^(1/3))."""
    s = 1000 + cid if seed is None else seed
    c3 = scale ** (1.0 / 3.0)
    if cid == 1:
        n = max(1, int(round(2000 * scale)))
        return uniform_cube(n, 1.0 * c3, 0.01, 1, 1e-6, s, nsample, "cube-2k")
    if cid == 2:
        n = max(1, int(round(1_000_000 * scale)))
        return uniform_cube(n, 100.0 * c3, 0.5, 1, 1e-6, s, 10_000 if nsample is None else nsample,
                            "cube-1M")
    if cid == 3:
        n = max(1, int(round(4_000_000 * scale)))
        nb = max(1, int(round(2000 * scale)))
        return clustered(n, nb, 500.0 * c3, 1.0, 0.5, 4, 1e-6, s,
                         10_000 if nsample is None else nsample, "blobs-4M")
    if cid == 4:
        return multi_system(64, max(2, int(1000 * scale)), max(3, int(200_000 * scale)), 0.1,
                            0.5, 16, 1e-6, s, 500 if nsample is None else nsample, "batched-64")
    if cid == 5:
        n = max(1, int(round(15_000_000 * scale)))
        return uniform_cube(n, 2000.0 * c3, 0.5, 20, 1e-6, s, 10_000 if nsample is None else nsample,
                            "cube-15M")
    if cid == 6:
        # uniform on a sphere surface (the paper's second workload), one bead
        # per unit area: radius sqrt(n / (4 pi))
        n = max(1, int(round(8_000_000 * scale)))
        return sphere_surface(n, float(np.sqrt(n / (4.0 * np.pi))), 0.5, 1, 1e-6, s,
                              10_000 if nsample is None else nsample, "sphere-8M")
    raise ValueError(f"unknown config {cid}")
