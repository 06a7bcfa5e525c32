"""Pins of the oracle's simplex integrals and quadrature rules.

The monomial formula and each rule are checked against an independent collapsed-
coordinate Gauss-Legendre integration (tests/_util.duffy_rule), which knows nothing
about barycentric orbits or the Eisenberg-Malvern formula.
"""

import itertools
import math

import numpy as np
import pytest

import oracle
from tests._util import bary_of_ref, duffy_rule


def _monomials(d, deg):
    for alpha in itertools.product(range(deg + 1), repeat=d + 1):
        if sum(alpha) <= deg:
            yield alpha


@pytest.mark.parametrize("d", [2, 3])
def test_monomial_formula_matches_duffy(d):
    pts, w = duffy_rule(d, 10)
    lam = bary_of_ref(pts)
    vol = 1.0 / math.factorial(d)
    for alpha in _monomials(d, 6):
        ref = float(np.sum(w * np.prod(lam ** np.array(alpha), axis=1))) / vol
        assert oracle.simplex_monomial(d, alpha) == pytest.approx(ref, rel=1e-13, abs=1e-16)


@pytest.mark.parametrize("d,degree,npts", [(2, 2, 3), (3, 2, 4), (3, 5, 14)])
def test_rule_exactness(d, degree, npts):
    bary, w = oracle.quad_rule(d, degree)
    assert bary.shape == (npts, d + 1)
    assert np.all(w > 0) and np.all(bary > 0) and np.all(bary < 1)
    assert np.allclose(bary.sum(1), 1.0, atol=1e-15)
    pts, wd = duffy_rule(d, 10)
    lam = bary_of_ref(pts)
    vol = 1.0 / math.factorial(d)
    count = 0
    for alpha in _monomials(d, degree):
        ref = float(np.sum(wd * np.prod(lam ** np.array(alpha), axis=1))) / vol
        got = float(np.sum(w * np.prod(bary ** np.array(alpha), axis=1)))
        assert got == pytest.approx(ref, rel=2e-14, abs=1e-16), alpha
        count += 1
    # all monomials of degree <= p in d+1 variables
    assert count == math.comb(degree + d + 1, d + 1)


@pytest.mark.parametrize("d,degree", [(2, 2), (3, 2), (3, 5)])
def test_rule_degree_is_sharp(d, degree):
    """Some monomial of degree p+1 is not integrated exactly (a rule of higher degree
    with the same number of points would signal a different rule)."""
    bary, w = oracle.quad_rule(d, degree)
    pts, wd = duffy_rule(d, 10)
    lam = bary_of_ref(pts)
    vol = 1.0 / math.factorial(d)
    errs = []
    for alpha in _monomials(d, degree + 1):
        if sum(alpha) != degree + 1:
            continue
        ref = float(np.sum(wd * np.prod(lam ** np.array(alpha), axis=1))) / vol
        got = float(np.sum(w * np.prod(bary ** np.array(alpha), axis=1)))
        errs.append(abs(got - ref))
    assert max(errs) > 1e-6


def test_tet14_known_orbits():
    """The degree-5 positive 14-point rule is unique for its orbit structure; its orbit
    parameters agree with the 10-digit values quoted in the literature."""
    bary, w = oracle.quad_rule(3, 5)
    a = sorted({round(float(np.median(p)), 12) for p in bary[:8]})  # the value taken 3 times
    assert a == pytest.approx([0.0927352503, 0.3108859193], abs=1e-10)
    assert min(bary[8]) == pytest.approx(0.0455037041, abs=1e-10)
    assert sorted(set(np.round(w, 12))) == pytest.approx(
        [0.0425460208, 0.0734930431, 0.1126879257], abs=1e-10)
