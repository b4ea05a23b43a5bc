"""Full-size workloads on the GPU, checked on sampled targets against the FP64
direct sum of the oracle (each sampled target summed over every source of
its system), in the configuration the benchmark uses (library-chosen leaf
size and order, both precision forms).

  * cube-1M:    1,000,000 uniform beads, one rhs, at both accuracy settings
                (eps 1e-3 and 1e-6), on 10,000 sampled targets;
  * blobs-4M:   4,000,000 clustered beads (2,000 Gaussian blobs), 4 rhs,
                adaptive tree with W/X lists and overlapping pairs outside U,
                on 2,000 sampled targets;
  * batched-64: 64 independent systems of 1e3 .. 2e5 beads, 16 rhs, one plan,
                min(n_s, 500) sampled targets per system;
  * cube-15M:   15,000,000 uniform beads, 20 rhs, on 2,000 sampled targets;
  * sphere-8M:  8,000,000 beads uniform on a sphere surface (adaptive tree),
                on 2,000 sampled targets.
Every case checks the rel-L2 error over all sampled targets and right-hand
sides against eps, and each target's error against 20 eps times the largest
reference velocity.  The direct-sum references are computed once per
workload and shared by the two precision forms.
"""
import numpy as np
import pytest

import workloads as W
from gpu_common import log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _run(w, precision, counts=None):
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    P = R.Plan(to_dev(w.pos), w.a, w.eta, w.eps, precision=precision, max_depth=w.max_depth, counts=counts,
               nrhs=w.forces.shape[0])
    try:
        F = to_dev(w.forces)
        U = P.matvec(F)
        idx = torch.as_tensor(w.sample, device=U.device)
        u = U[:, idx].cpu().numpy()
        st = P.stats()
        del F, U
    finally:
        P.free()
        torch.cuda.empty_cache()
    return u, st


def _direct_by_system(orc, w):
    """Direct sum for the sampled targets, system by system."""
    out = np.zeros((w.nrhs, len(w.sample), 3))
    bounds = np.concatenate([[0], np.cumsum(w.counts)])
    for s in range(len(w.counts)):
        b0, b1 = bounds[s], bounds[s + 1]
        sel = np.where((w.sample >= b0) & (w.sample < b1))[0]
        if len(sel) == 0:
            continue
        out[:, sel] = orc.rpy_direct(w.pos[b0:b1], w.forces[:, b0:b1], w.a, w.eta, targets=w.sample[sel] - b0)
    return out


_refs = {}


def _check(orc, key, w, u, st, direct=None):
    if key not in _refs:
        _refs[key] = (direct or (lambda: orc.rpy_direct(w.pos, w.forces, w.a, w.eta, targets=w.sample)))()
    ref = _refs[key]
    err = orc.rel_l2(u, ref)
    d = np.linalg.norm(u - ref, axis=-1).max() / np.linalg.norm(ref, axis=-1).max()
    log(f"  p={st['order']} s={st['leaf_size']} depth={st['depth']} nbox={st['nbox']} lists={st['list_len']} "
        f"rel-L2 = {err:.3e}, max target error / max |ref| = {d:.3e} ({len(w.sample)} targets)")
    assert err <= w.eps
    assert d <= 20 * w.eps
    return err


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_blobs_4M(orc, precision):
    w = W.config(3, nsample=2000)
    log(f"{w.name} n={w.n} nrhs={w.nrhs} {precision}")
    u, st = _run(w, precision)
    assert st["list_len"]["O"] > 0, "the clustered workload is expected to need the overlap correction"
    _check(orc, "blobs", w, u, st)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_64(orc, precision):
    w = W.config(4, nsample=500)
    log(f"{w.name} systems={len(w.counts)} n={w.n} nrhs={w.nrhs} {precision}")
    u, st = _run(w, precision, counts=w.counts)
    assert st["nsys"] == 64
    assert len(w.sample) == sum(min(c, 500) for c in w.counts)
    _check(orc, "batched", w, u, st, direct=lambda: _direct_by_system(orc, w))


@pytest.mark.parametrize("precision,eps", [("fp64", 1e-3), ("mixed", 1e-3), ("fp64", 1e-6), ("mixed", 1e-6)])
def test_cube_1M(orc, precision, eps):
    import dataclasses
    w = dataclasses.replace(W.config(2), eps=eps)  # 10,000 sampled targets
    log(f"{w.name} n={w.n} eps={eps} {precision}")
    u, st = _run(w, precision)
    assert len(w.sample) == 10_000
    _check(orc, "cube1M", w, u, st)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cube_15M(orc, precision):
    w = W.config(5, nsample=2000)
    log(f"{w.name} n={w.n} nrhs={w.nrhs} {precision}")
    u, st = _run(w, precision)
    _check(orc, "cube15M", w, u, st)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sphere_8M(orc, precision):
    w = W.config(6, nsample=2000)
    log(f"{w.name} n={w.n} nrhs={w.nrhs} {precision}")
    u, st = _run(w, precision)
    _check(orc, "sphere8M", w, u, st)
