"""Pins of the validation oracle (Section 5.1 p-value testing, Section 5.2
evaluation metrics), each against a closed form or a hand-worked example:

* the t statistic on hand values; the right p-value against the closed forms
  of the t distribution with 1 degree of freedom (Cauchy: 1/2 - atan(T)/pi)
  and 2 (1/2 - T / (2 sqrt(2 + T^2))), and the normal tail at large n;
* correlation: +-1 for affinely related rows, 0 for a constant row, the
  textbook definition on a small example;
* Benjamini-Hochberg adjustment on a hand-worked example with ties;
* recovery ratio and error on the matching pattern the paper draws (one true
  community matched three times, one matched once, one unmatched, one matched
  twice), computed by hand;
* bridgeness: 0 for a pure membership, 1 for a uniform one, and a hand value.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import validation as va


def test_t_statistic_hand_values():
    assert va.t_statistic(np.array(0.6), 27) == pytest.approx(0.6 * 5.0 / 0.8, rel=1e-15)
    assert va.t_statistic(np.array(0.0), 10) == 0.0
    assert va.t_statistic(np.array(-0.5), 6) == pytest.approx(-0.5 * 2.0 / math.sqrt(0.75), rel=1e-15)
    assert va.t_statistic(np.array(1.0), 10) == np.inf


@pytest.mark.parametrize("T", [-3.0, -0.4, 0.0, 0.7, 2.5, 40.0])
def test_right_pvalue_closed_forms(T):
    # 1 degree of freedom (n = 3): the Cauchy tail
    assert va.right_pvalue(np.array(T), 1.0) == pytest.approx(0.5 - math.atan(T) / math.pi, rel=1e-12, abs=1e-15)
    # 2 degrees of freedom (n = 4)
    assert va.right_pvalue(np.array(T), 2.0) == pytest.approx(0.5 - T / (2.0 * math.sqrt(2.0 + T * T)), rel=1e-12,
                                                              abs=1e-15)
    # many degrees of freedom: the normal tail
    assert va.right_pvalue(np.array(T), 1e7) == pytest.approx(0.5 * math.erfc(T / math.sqrt(2.0)), rel=1e-5,
                                                              abs=1e-15)


def test_pvalue_matrix_is_the_right_tail_of_the_statistic():
    """Positively correlated pairs get small p-values, anti-correlated large."""
    g = np.random.default_rng(0)
    Pi = g.random((3, 500))
    Pi_hat = np.stack([Pi[1] + 0.1 * g.random(500), 1.0 - Pi[0], g.random(500)])
    p = va.pvalue_matrix(Pi_hat, Pi)
    assert p[0, 1] < 1e-100 and p[1, 0] > 0.999
    rho = va.correlation(Pi_hat, Pi)
    with np.errstate(divide="ignore"):   # rho = -1 exactly for 1 - Pi[0]: T = -inf
        T = rho * np.sqrt(498.0) / np.sqrt(1.0 - rho ** 2)
    np.testing.assert_allclose(p, 0.5 * stats.beta.cdf(498.0 / (498.0 + T * T), 249.0, 0.5) * (T > 0)
                               + (1.0 - 0.5 * stats.beta.cdf(498.0 / (498.0 + T * T), 249.0, 0.5)) * (T <= 0),
                               rtol=1e-9, atol=1e-300)


def test_correlation_definition():
    a = np.array([[1.0, 2.0, 3.0, 5.0], [2.0, 2.0, 2.0, 2.0], [4.0, 1.0, 0.0, 3.0]])
    b = np.array([[3.0, 5.0, 7.0, 11.0], [-1.0, -2.0, -3.0, -5.0]])
    rho = va.correlation(a, b)
    np.testing.assert_allclose(rho[0], [1.0, -1.0], atol=1e-15)
    np.testing.assert_array_equal(rho[1], [0.0, 0.0])
    x, y = a[2], b[0]
    xm, ym = x - x.mean(), y - y.mean()
    assert rho[2, 0] == pytest.approx(np.sum(xm * ym) / math.sqrt(np.sum(xm ** 2) * np.sum(ym ** 2)), rel=1e-14)


def test_bh_adjust_hand_example():
    # m = 6 p-values (two tied), sorted: .001 .008 .02 .02 .04 .5
    p = np.array([[0.02, 0.5, 0.001], [0.04, 0.02, 0.008]])
    # m p / rank: .006 .024 .04 .03 .048 .5 -> running minimum from the top:
    #             .006 .024 .03 .03 .048 .5
    want = np.array([[0.03, 0.5, 0.006], [0.048, 0.03, 0.024]])
    np.testing.assert_allclose(va.bh_adjust(p), want, rtol=1e-14)
    assert va.bh_adjust(np.array([0.9, 0.95])).max() <= 1.0
    np.testing.assert_array_equal(va.bh_adjust(np.array([0.7])), [0.7])


def test_recovery_ratio_and_error_on_the_drawn_matching_pattern():
    """k = 4 true and k_hat = 6 estimated communities; edges: true 1 with
    estimated 2, 3, 6; true 2 with estimated 1; true 4 with estimated 4, 5;
    true 3 unmatched (zero-based below)."""
    E = np.zeros((6, 4), dtype=bool)
    for i, j in ((1, 0), (2, 0), (5, 0), (0, 1), (3, 3), (4, 3)):
        E[i, j] = True
    assert va.recovery_ratio(E) == 0.75
    n = 4
    Pi = np.array([[1, 0, 0, .5], [0, 1, 0, .5], [0, 0, 1, 0], [0, 0, 0, 0.]])
    Pi_hat = np.array([[0, 1, 0, 0], [1, 0, 0, 0], [.5, 0, 0, .5], [0, 0, 0, 0], [0, 0, 1, 0], [1, 0, 0, 1.]])
    # sum over the 4 nodes of |Pi_hat_i - Pi_j| for the six edges:
    # (1,0) .5, (2,0) .5, (5,0) .5, (0,1) .5, (3,3) 0, (4,3) 1  -> 3.0
    # E = (1/k) sum (1/n) (...) = 3.0 / 4 / 4
    assert va.error(Pi_hat, Pi, E) == pytest.approx(0.1875, rel=1e-15)
    assert va.l1_distances(Pi_hat, Pi)[4, 3] == 0.25


def test_bridgeness_extremes_and_hand_value():
    M = np.array([[1.0, 0.25, 0.5], [0.0, 0.25, 0.5], [0.0, 0.25, 0.0], [0.0, 0.25, 0.0]])   # k_hat = 4, 3 nodes
    b = va.bridgeness(M)
    assert b[0] == pytest.approx(0.0, abs=1e-15)
    assert b[1] == pytest.approx(1.0, abs=1e-15)
    # (1/2, 1/2, 0, 0): sum (m - 1/4)^2 = 4 / 16, times 4/3 -> 1/3
    assert b[2] == pytest.approx(1.0 - math.sqrt(1.0 / 3.0), rel=1e-15)
    b2, B = va.bridgeness(M, degree=np.array([3.0, 7.0, 2.0]))
    np.testing.assert_allclose(B, [0.0, 7.0, 2.0 * b[2]], atol=1e-15)


def test_validate_recovers_a_permuted_noisy_estimate():
    """An estimate that is the truth with rows permuted plus small noise: every
    true community is recovered (R = 1) through exactly its own row, and E is
    the mean l1 noise."""
    g = np.random.default_rng(3)
    k, n = 5, 2000
    Pi = g.dirichlet(np.full(k, 0.2), size=n).T
    perm = g.permutation(k)
    Pi_hat = Pi[perm] + 0.01 * g.random((k, n))
    out = va.validate(Pi_hat, Pi)
    assert out["recovery_ratio"] == 1.0
    E = out["edges"]
    assert E.sum() == k and all(E[i, perm[i]] for i in range(k))
    expect = np.mean([np.abs(Pi_hat[i] - Pi[perm[i]]).mean() for i in range(k)])
    assert out["error"] == pytest.approx(expect, rel=1e-12)
