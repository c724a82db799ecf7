"""Pins of the oracle's quadrature rules against the closed-form simplex
moments  int_K lam^alpha = d! alpha! / (|alpha| + d)! |K|  (reference |K| = 1/d!)."""
import itertools
from math import factorial

import numpy as np
import pytest

from oracle import quadrature


def exact_moment(alpha):
    d = len(alpha) - 1
    num = 1
    for a in alpha:
        num *= factorial(a)
    return num / factorial(sum(alpha) + d)   # d! |K| = 1 on the reference simplex


def moments(dim, degree):
    for alpha in itertools.product(range(degree + 1), repeat=dim + 1):
        if sum(alpha) <= degree:
            yield alpha


@pytest.mark.parametrize("dim,rule,deg", [
    (2, quadrature.triangle_deg5, 5),
    (3, quadrature.tet_deg5, 5),
    (2, lambda: quadrature.triangle_collapsed(5), 9),
    (3, lambda: quadrature.tet_collapsed(5), 9),
    (2, lambda: quadrature.triangle_collapsed_gl(5), 8),
])
def test_rule_exact_on_all_monomials(dim, rule, deg):
    lam, w = rule()
    assert lam.shape[1] == dim + 1
    np.testing.assert_allclose(lam.sum(axis=1), 1.0, atol=1e-15)
    assert abs(w.sum() - 1.0 / factorial(dim)) < 1e-15
    for alpha in moments(dim, deg):
        q = np.sum(w * np.prod(lam ** np.array(alpha), axis=1))
        assert abs(q - exact_moment(alpha)) < 2e-16, alpha


def test_radon_rule_is_not_exact_at_degree_6():
    # guards against a rule that is accidentally of higher degree (a sign of
    # a different rule than the stated one)
    lam, w = quadrature.triangle_deg5()
    errs = [abs(np.sum(w * np.prod(lam ** np.array(a), axis=1)) - exact_moment(a))
            for a in itertools.product(range(7), repeat=3) if sum(a) == 6]
    assert max(errs) > 1e-6
    assert len(w) == 7 and np.all(w > 0)


def test_collapsed_gauss_legendre_rule_stops_at_degree_8():
    """The P3-P2 rule: the Jacobian factor 1 - u costs one degree against the
    Gauss-Jacobi version, so some degree-9 moment is missed."""
    lam, w = quadrature.triangle_collapsed_gl(5)
    errs = [abs(np.sum(w * np.prod(lam ** np.array(a), axis=1)) - exact_moment(a))
            for a in itertools.product(range(10), repeat=3) if sum(a) == 9]
    assert max(errs) > 1e-8
    assert len(w) == 25 and np.all(w > 0)
