"""GPU parity of rpy_sqrt_matvec (Brownian displacement directions
y = D^{1/2} z by the Lanczos approximation over the Krylov space {D^k z},
arXiv:1711.02976 Sec. 1) against the oracle's dense eigen-decomposition."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_common import log, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _cloud(n, side, seed):
    g = np.random.default_rng(seed)
    return g.uniform(0.0, side, size=(n, 3)), g


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_single_leaf_matches_dense_square_root(orc):
    # one leaf holds every bead, so every matvec is the exact FP64 pair sum;
    # the Lanczos result then differs from D^{1/2} z only by its tolerance
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    pos, g = _cloud(500, 30.0, 5)
    z = g.standard_normal((1, 500, 3))
    log("sqrt_matvec single leaf n=500")
    P = R.Plan(to_dev(pos), 0.5, 1.0, 1e-6, leaf_size=1000)
    try:
        y, info = P.sqrt_matvec(to_dev(z), tol=1e-11, max_iter=100)
        torch.cuda.synchronize()
        ref = orc.rpy_sqrt(pos, z, 0.5, 1.0)
        err = _rel(y.cpu().numpy(), ref)
        log(f"  iterations {info['iterations']} change {info['rel_change']:.2e} rel err {err:.2e}")
        assert info["converged"] and info["iterations"] < 100
        assert info["min_ritz"] > 0.0
        assert err <= 1e-9
    finally:
        P.free()


@pytest.mark.parametrize("precision,eps,bound", [("fp64", 1e-8, 1e-7), ("mixed", 1e-6, 2e-6)])
def test_multilevel_tree_matches_dense_square_root(orc, precision, eps, bound):
    # a multi-level tree: D is applied by the FMM to eps, so y carries the
    # far-field error as well as the Lanczos tolerance
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    pos, g = _cloud(1200, 40.0, 9)
    z = g.standard_normal((2, 1200, 3))
    log(f"sqrt_matvec multilevel n=1200 {precision}")
    P = R.Plan(to_dev(pos), 0.5, 1.0, eps, precision=precision, leaf_size=40)
    try:
        assert P.stats()["depth"] >= 2
        y, info = P.sqrt_matvec(to_dev(z), tol=1e-9, max_iter=100)
        torch.cuda.synchronize()
        ref = orc.rpy_sqrt(pos, z, 0.5, 1.0)
        y = y.cpu().numpy()
        errs = [_rel(y[r], ref[r]) for r in range(2)]
        log(f"  iterations {info['iterations']} change {info['rel_change']:.2e} rel errs {errs}")
        assert info["converged"]
        assert max(errs) <= bound
    finally:
        P.free()


def test_one_step_and_zero_vector(orc):
    # after one step the approximation is beta_0 sqrt(alpha_0) v_0
    # = sqrt(z.Dz / z.z) z; a zero right-hand side gives y = 0
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    pos, g = _cloud(300, 20.0, 2)
    z = g.standard_normal((3, 300, 3))
    z[1] = 0.0
    log("sqrt_matvec one step, zero rhs")
    P = R.Plan(to_dev(pos), 0.5, 1.0, 1e-6, leaf_size=1000)
    try:
        y, info = P.sqrt_matvec(to_dev(z), tol=1e-6, max_iter=1)
        torch.cuda.synchronize()
        y = y.cpu().numpy()
        assert info["iterations"] == 1 and not info["converged"]
        Dz = orc.rpy_direct(pos, z, 0.5, 1.0)
        for r in (0, 2):
            expect = np.sqrt(np.sum(z[r] * Dz[r]) / np.sum(z[r] * z[r])) * z[r]
            assert _rel(y[r], expect) <= 1e-12
        assert np.all(y[1] == 0.0)
        # the same right-hand sides one at a time give the same vectors
        y0, _ = P.sqrt_matvec(to_dev(z[0]), tol=1e-6, max_iter=1)
        torch.cuda.synchronize()
        assert _rel(y0.cpu().numpy(), y[0]) <= 1e-14
    finally:
        P.free()


def test_batched_rhs_agree_with_single(orc):
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    pos, g = _cloud(800, 25.0, 4)
    z = g.standard_normal((4, 800, 3))
    log("sqrt_matvec 4 rhs vs one at a time")
    P = R.Plan(to_dev(pos), 0.5, 1.0, 1e-8, leaf_size=60)
    try:
        y, info = P.sqrt_matvec(to_dev(z), tol=1e-10, max_iter=100)
        torch.cuda.synchronize()
        y = y.cpu().numpy()
        assert info["converged"]
        for r in (0, 3):
            yr, _ = P.sqrt_matvec(to_dev(z[r]), tol=1e-10, max_iter=100)
            torch.cuda.synchronize()
            assert _rel(yr.cpu().numpy(), y[r]) <= 1e-8
    finally:
        P.free()


def test_argument_errors():
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    pos, g = _cloud(50, 5.0, 1)
    P = R.Plan(to_dev(pos), 0.5, 1.0, 1e-6)
    try:
        z = to_dev(g.standard_normal((1, 50, 3)))
        L = R.lib()
        info = R.rpy_sqrt_info_t()
        for tol, it in ((0.0, 10), (1.0, 10), (1e-6, 0), (1e-6, 101)):
            assert L.rpy_sqrt_matvec(P.handle, 1, z.data_ptr(), z.data_ptr() + 8, tol, it, C.byref(info)) \
                == R.RPY_EINVAL
        assert L.rpy_sqrt_matvec(P.handle, 1, z.data_ptr(), z.data_ptr(), 1e-6, 10, C.byref(info)) == R.RPY_EINVAL
        assert b"alias" in L.rpy_last_error()
        torch.cuda.synchronize()
    finally:
        P.free()
