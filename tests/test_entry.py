"""The CPU side of __graft_entry__.smoke(): the oracle references it checks
the GPU against are computed with the arguments smoke() passes (no GPU)."""
import numpy as np

import workloads as W


def test_smoke_oracle_references():
    import __graft_entry__ as entry
    w = W.config(1)
    direct, fmm, pos3, z, sq = entry._oracle_refs(w, (8 + 1) * (8 + 2))
    assert direct.shape == w.forces.shape and fmm.shape == w.forces.shape
    assert np.all(np.isfinite(direct)) and np.all(np.isfinite(fmm)) and np.all(np.isfinite(sq))
    assert sq.shape == z.shape and pos3.shape == (300, 3)
    # order 8 with leaves of at most 40 beads is a few digits from the direct sum
    import oracle
    assert oracle.rel_l2(fmm, direct) < 1e-3
