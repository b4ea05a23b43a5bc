"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

rpy_oracle.c is built a second time with -fsanitize=address,undefined (any
finding aborts) and every entry point runs in a child process that preloads
the ASan runtime: the direct sum, the dense matrix, the tree and its lists on
clustered beads with overlaps (W, X and O lists non-empty), the expansion
operators, both evaluation approaches of the FMM and the brute-force
four-Laplace sum.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import oracle as orc
import workloads as W
w = W.clustered(1500, 6, 10.0, 0.7, 0.3, 2, seed=5)
u = orc.rpy_direct(w.pos, w.forces, w.a, w.eta)
D = orc.rpy_dense(w.pos[:40], w.a, w.eta)
t = orc.Tree(w.pos, 20, 14, w.a)
assert all(len(t.lists[k][1]) > 0 for k in ("W", "X", "O")), {k: len(v[1]) for k, v in t.lists.items()}
for ev in (0, 1):
    f = orc.fmm(w.pos, w.forces, w.a, w.eta, 8, 20, 90, eval_mode=ev)
    assert orc.rel_l2(f, u) < 1e-2
g = orc.far_four_laplace(w.pos[:300], w.forces[0, :300], w.a, w.eta)
P = orc.legendre(6, 0.3)
Y = orc.ynm(6, 0.4, 1.1)
p = 7
src = np.random.default_rng(1).random((30, 3))
q = np.random.default_rng(2).standard_normal(30)
M = orc.p2m(p, src, q, np.full(3, 0.5))
L = orc.p2l(p, src, q, np.array([4.0, 0.5, 0.5]))
M2 = orc.translate(p, "m2m", M, np.full(3, 0.5), np.zeros(3))
L2 = orc.translate(p, "m2l", M, np.full(3, 0.5), np.array([4.0, 0.5, 0.5]))
L3 = orc.translate(p, "l2l", L2, np.array([4.0, 0.5, 0.5]), np.array([4.1, 0.4, 0.6]))
vm = orc.eval_expansion(p, "M", M, np.array([3.0, 0.2, 0.1]))
vl = orc.eval_expansion(p, "L", L, np.array([0.1, 0.2, 0.1]))
s = orc.solid_monomials(5, 3, 2)
print("sanitized oracle ok")
"""


def _runtime():
    try:
        path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_runs_clean_under_asan_and_ubsan(tmp_path):
    asan = _runtime()
    if asan is None:
        pytest.skip("no ASan runtime for gcc here")
    lib = tmp_path / "liborc_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-o", str(lib), os.path.join(ROOT, "oracle", "rpy_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0", RPY_ORACLE_LIB=str(lib),
               OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
