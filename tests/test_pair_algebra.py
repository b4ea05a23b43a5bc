"""Algebra behind the pair kernels' overlap correction (host-side, no GPU).

For a pair closer than 2a in leaves that are not adjacent, the far field has
applied the r >= 2a branch of the RPY block (Sec. 1), so the kernels add the
difference of the two branches.  With the prefactor 1/(8 pi eta) taken out
and rho = r/(2a) the differences are
    A = (4/(3a))(1 - 9r/(32a)) - 1/r - (2a^2/3)/r^3,
    B = (4/(3a))(3/(32a))/r - (1 - 2a^2/r^2)/r^3      (B multiplies d d^T),
and the kernels evaluate them in the factored form
    A = -(2a^2/3) (1 - rho)^2 (9 rho^2 + 2 rho + 1) / r^3,
    B = 2a^2 (1 - rho)^2 (1 + rho)^2 / r^5,
in which nothing cancels as r approaches 2a.  The identities are checked
exactly, in rational arithmetic.
"""
from fractions import Fraction as Fr

import pytest


def _direct(a, r):
    A = Fr(4, 3) / a * (1 - Fr(9, 32) * r / a) - 1 / r - (2 * a * a / 3) / r ** 3
    B = Fr(4, 3) / a * Fr(3, 32) / a / r - (1 - 2 * a * a / r ** 2) / r ** 3
    return A, B


def _factored(a, r):
    rho = r / (2 * a)
    A = -(2 * a * a / 3) * (1 - rho) ** 2 * (9 * rho ** 2 + 2 * rho + 1) / r ** 3
    B = 2 * a * a * (1 - rho) ** 2 * (1 + rho) ** 2 / r ** 5
    return A, B


@pytest.mark.parametrize("a", [Fr(1, 2), Fr(1), Fr(3, 7), Fr(1, 10 ** 10)], ids=str)
def test_factored_overlap_difference_is_exact(a):
    for k in range(1, 41):
        r = 2 * a * Fr(k, 40)
        assert _factored(a, r) == _direct(a, r)
    # both branches meet at contact, with a double zero of the difference
    assert _direct(a, 2 * a) == (0, 0)


def test_factored_form_has_no_cancellation_near_contact():
    # in floating point, at a representable r just below 2a, the direct
    # difference loses digits to cancellation; the factored form keeps its
    # relative accuracy (1 - rho is exact there)
    a = 0.5
    for eps in (1e-3, 1e-6):
        r = 2 * a * (1 - eps)
        exact_A, exact_B = (float(v) for v in _direct(Fr(a), Fr(r)))
        fa, fb = _factored(a, r)
        da, db = _direct_float(a, r)
        assert abs(fa - exact_A) <= 1e-14 * abs(exact_A)
        assert abs(fb - exact_B) <= 1e-14 * abs(exact_B)
        assert abs(da - exact_A) > 100 * abs(fa - exact_A)


def _direct_float(a, r):
    A = 4 / (3 * a) * (1 - 9 * r / (32 * a)) - 1 / r - (2 * a * a / 3) / r ** 3
    B = 4 / (3 * a) * 3 / (32 * a) / r - (1 - 2 * a * a / r ** 2) / r ** 3
    return A, B
