"""rpy_matvec_noalloc (workspace in the library's fixed device scratch, no
allocation) against rpy_matvec on the same plans, through the C ABI: two
calls in a row, the second on a smaller plan with fewer right-hand sides,
then the first plan again; FP64 results agree to the parity bar (rel-L2
<= 1e-12 and per target), and are bitwise equal where both calls carry the
same right-hand sides per pass.  A plan whose workspace exceeds the scratch
is refused with RPY_ENOMEM and nothing written."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_common import log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(R, w, **kw):
    return R.Plan(to_dev(w.pos), w.a, w.eta, 1e-6, **kw)


def _noalloc(R, P, F, U):
    R.rpy_matvec_noalloc(P.handle, F.shape[0], F.data_ptr(), U.data_ptr())


def _close(a, b, orc):
    err = orc.rel_l2(a, b)
    d = np.linalg.norm(a - b, axis=-1).max() / np.linalg.norm(b, axis=-1).max()
    log(f"  noalloc vs matvec rel-L2 = {err:.3e}, max target error / max |ref| = {d:.3e}")
    assert err <= 1e-12 and d <= 1e-11


def test_noalloc_matches_matvec(orc):
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    big = W.clustered(30_000, 12, 25.0, 1.0, 0.5, 3, seed=131)
    small = W.uniform_cube(5_000, 1.0, 0.01, nrhs=1, seed=132)
    log(f"noalloc: plan A n={big.n} nrhs={big.nrhs}, plan B n={small.n} nrhs={small.nrhs}")
    PA = _plan(R, big, leaf_size=200, order=12)
    PB = _plan(R, small, leaf_size=40, order=9, precision="mixed")
    try:
        stA = PA.stats()
        assert stA["list_len"]["W"] > 0 and stA["list_len"]["O"] > 0
        FA, FB = to_dev(big.forces), to_dev(small.forces)
        refA = PA.matvec(FA).cpu().numpy()
        refB = PB.matvec(FB).cpu().numpy()
        UA = torch.full_like(FA, float("nan"))
        UB = torch.full_like(FB, float("nan"))
        torch.cuda.synchronize()
        _noalloc(R, PA, FA, UA)   # first call: larger plan, 3 right-hand sides
        _noalloc(R, PB, FB, UB)   # second call: smaller plan, 1 right-hand side
        torch.cuda.synchronize()
        a, b = UA.cpu().numpy(), UB.cpu().numpy()
        _close(a, refA, orc)
        assert np.array_equal(a, refA)
        assert orc.rel_l2(b, refB) <= 1e-12 and np.array_equal(b, refB)
        # the first plan again after the smaller one left its contents
        UA.fill_(float("nan"))
        _noalloc(R, PA, FA, UA)
        torch.cuda.synchronize()
        assert np.array_equal(UA.cpu().numpy(), refA)
        # and against the oracle FMM of the same tree and order
        _close(UA.cpu().numpy(), orc.fmm(big.pos, big.forces, big.a, big.eta, 12, 200, stA["w_direct"]), orc)
    finally:
        PA.free()
        PB.free()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_matrix_core_group(orc, precision):
    # 20 right-hand sides: in the mixed form a near-field group of 16 on the
    # matrix cores and one of 4 on the vector units, in the FP64 form one
    # launch of 16 + 4, from the scratch; the workspace fits, so the grouping
    # and the results equal rpy_matvec's
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    w = W.uniform_cube(6_000, 1.0, 0.01, nrhs=20, seed=134)
    log(f"noalloc: n={w.n} nrhs={w.nrhs} {precision}")
    P = _plan(R, w, leaf_size=200, order=16, precision=precision)
    try:
        F = to_dev(w.forces)
        ref = P.matvec(F).cpu().numpy()
        U = torch.full_like(F, float("nan"))
        torch.cuda.synchronize()
        _noalloc(R, P, F, U)
        torch.cuda.synchronize()
        assert np.array_equal(U.cpu().numpy(), ref)
        assert orc.rel_l2(ref, orc.rpy_direct(w.pos, w.forces, w.a, w.eta)) <= 1e-6
    finally:
        P.free()


def test_noalloc_refuses_oversized_plan(orc):
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    w = W.uniform_cube(1_000_000, 100.0, 0.5, nrhs=1, seed=133)
    log("noalloc: 1M-bead plan exceeds the scratch")
    P = _plan(R, w, leaf_size=64, order=16)
    try:
        F = to_dev(w.forces)
        U = torch.zeros_like(F)
        st = R.lib().rpy_matvec_noalloc(P.handle, 1, C.c_void_p(F.data_ptr()), C.c_void_p(U.data_ptr()))
        assert st == R.RPY_ENOMEM
        assert b"scratch" in R.lib().rpy_last_error()
        torch.cuda.synchronize()
        assert float(U.abs().max()) == 0.0
        # the plan is still usable
        u = P.matvec(F)
        assert torch.isfinite(u).all()
    finally:
        P.free()
