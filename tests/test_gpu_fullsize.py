"""Full-size workloads on the GPU, checked on sampled targets against the FP64
direct sum of the oracle (each sampled target summed over every source of
its system), in the configuration the benchmark uses (library-chosen leaf
size and order, both precision forms).

  * cube-1M:    1,000,000 uniform beads, one rhs, at both accuracy settings
                (eps 1e-3 and 1e-6), on 10,000 sampled targets;
  * blobs-4M:   4,000,000 clustered beads (2,000 Gaussian blobs), 4 rhs,
                adaptive tree with W/X lists and overlapping pairs outside U;
  * batched-64: 64 independent systems of 1e3 .. 2e5 beads, 16 rhs, one plan;
  * cube-15M:   15,000,000 uniform beads, 20 rhs;
  * sphere-8M:  8,000,000 beads uniform on a sphere surface (adaptive tree).
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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_blobs_4M(orc, precision):
    w = W.config(3, nsample=400)
    log(f"{w.name} n={w.n} nrhs={w.nrhs} {precision}")
    u, st = _run(w, precision)
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta, targets=w.sample)
    err = orc.rel_l2(u, ref)
    log(f"  p={st['order']} s={st['leaf_size']} depth={st['depth']} nbox={st['nbox']} "
        f"W={st['list_len']['W']} X={st['list_len']['X']} O={st['list_len']['O']} rel-L2 = {err:.3e}")
    assert st["list_len"]["O"] > 0, "the clustered workload is expected to need the overlap correction"
    assert err <= w.eps


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_64(orc, precision):
    w = W.config(4, nsample=60)
    log(f"{w.name} systems={len(w.counts)} n={w.n} nrhs={w.nrhs} {precision}")
    u, st = _run(w, precision, counts=w.counts)
    ref = _direct_by_system(orc, w)
    err = orc.rel_l2(u, ref)
    log(f"  p={st['order']} s={st['leaf_size']} nbox={st['nbox']} rel-L2 = {err:.3e}")
    assert st["nsys"] == 64
    assert err <= w.eps


_cube_ref = {}


@pytest.mark.parametrize("precision,eps", [("fp64", 1e-3), ("mixed", 1e-3), ("fp64", 1e-6), ("mixed", 1e-6)])
def test_cube_1M(orc, precision, eps):
    import dataclasses
    w = dataclasses.replace(W.config(2), eps=eps)  # 10,000 sampled targets
    log(f"{w.name} n={w.n} eps={eps} {precision}")
    u, st = _run(w, precision)
    if "ref" not in _cube_ref:
        _cube_ref["ref"] = orc.rpy_direct(w.pos, w.forces, w.a, w.eta, targets=w.sample)
    err = orc.rel_l2(u, _cube_ref["ref"])
    log(f"  p={st['order']} s={st['leaf_size']} depth={st['depth']} rel-L2 = {err:.3e}")
    assert len(w.sample) == 10_000
    assert err <= eps


def test_cube_15M_mixed(orc):
    w = W.config(5, nsample=150)
    log(f"{w.name} n={w.n} nrhs={w.nrhs} mixed")
    u, st = _run(w, "mixed")
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta, targets=w.sample)
    err = orc.rel_l2(u, ref)
    log(f"  p={st['order']} s={st['leaf_size']} depth={st['depth']} nbox={st['nbox']} rel-L2 = {err:.3e}")
    assert err <= w.eps


def test_sphere_8M_mixed(orc):
    w = W.config(6, nsample=200)
    log(f"{w.name} n={w.n} nrhs={w.nrhs} mixed")
    u, st = _run(w, "mixed")
    ref = orc.rpy_direct(w.pos, w.forces, w.a, w.eta, targets=w.sample)
    err = orc.rel_l2(u, ref)
    log(f"  p={st['order']} s={st['leaf_size']} depth={st['depth']} nbox={st['nbox']} "
        f"W={st['list_len']['W']} O={st['list_len']['O']} rel-L2 = {err:.3e}")
    assert err <= w.eps
