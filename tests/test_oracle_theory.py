"""Pins for the oracle's threshold and recursion code (paper, Sections 2-4, Appendix B)."""
import math

import numpy as np

import pytest

from oracle import theory


def test_thresholds_match_printed_values(golden):
    # Section 2 after eq. (cstar); Appendix C text and Figure 1 caption.
    for k, r, printed, decimals in golden("thresholds.txt"):
        c, _ = theory.cstar(int(k), int(r))
        assert round(c, int(decimals)) == pytest.approx(printed, abs=1e-12), (k, r, c)


@pytest.mark.parametrize("k,r", [(2, 3), (2, 4), (3, 3), (2, 5), (3, 4)])
def test_xstar_satisfies_first_order_condition(k, r):
    # Appendix C, eq. (starderiv): e^{-x}(S(k-2,x) - S(k-3,x)) = (1 - e^{-x}S(k-2,x)) / (x (r-1)).
    c, x = theory.cstar(k, r)
    S = theory.poisson_tail_sum
    lhs = math.exp(-x) * (S(k - 2, x) - S(k - 3, x))
    rhs = (1 - math.exp(-x) * S(k - 2, x)) / (x * (r - 1))
    assert lhs == pytest.approx(rhs, rel=1e-6)
    # and x* is a minimum of the objective
    assert theory.threshold_objective(x * 0.99, k, r) > c
    assert theory.threshold_objective(x * 1.01, k, r) > c


def test_table2_prediction_columns_exact(golden):
    # Table 2: lambda_t * n for r=4, k=2, n=10^6; the printed integers are rounded.
    rows = golden("table2.txt")
    lo = theory.survival(0.70, 2, 4, 20)
    hi = theory.survival(0.85, 2, 4, 20)
    for t, p70, _, p85, _ in rows:
        t = int(t)
        if p70 >= 1:
            assert round(lo[t - 1] * 1e6) == p70, (t, lo[t - 1] * 1e6)
        else:
            assert lo[t - 1] * 1e6 == pytest.approx(p70, abs=5e-6), t
        assert round(hi[t - 1] * 1e6) == p85, (t, hi[t - 1] * 1e6)


def test_table4_subtable_prediction_exact(golden):
    # Table 4: lambda'_{i,j} * n, r=4, k=2, n=10^6, c=0.7 (eq. newlambdaij).
    pred = dict(theory.subtable_survival(0.70, 2, 4, 7))
    for i, j, p, _ in golden("table4.txt"):
        v = pred[(int(i), int(j))] * 1e6
        if p >= 1:
            assert round(v) == p, (i, j, v)
        else:
            assert v == pytest.approx(p, abs=5e-4), (i, j, v)


def test_above_threshold_fixed_point_matches_table2_limit():
    # Table 2, c = 0.85: the prediction converges to 775010 vertices (of 10^6).
    fp = theory.fixed_point(0.85, 2, 4)
    assert round(fp["lambda"] * 1e6) == 775010
    # eq. (a): 0 < f'(0) < 1 above the threshold
    assert 0.0 < fp["fprime0"] < 1.0


def test_below_threshold_fixed_point_is_zero():
    fp = theory.fixed_point(0.70, 2, 4)
    assert fp["beta"] < 1e-9 and fp["lambda"] < 1e-9


def test_recovered_fraction_r4_load083(golden):
    # Table 6: r=4 at load 0.83 recovers 24.6% of the items.  Items left in the
    # 2-core are the edges whose r vertices all survive: rho^r of them.
    rows = {(int(r), l): p for r, l, p in golden("iblt_tables56.txt")}
    fp = theory.fixed_point(0.83, 2, 4)
    assert 100 * (1 - fp["edge_fraction"]) == pytest.approx(rows[(4, 0.83)], abs=0.05)
    # below the threshold everything is recovered
    assert theory.fixed_point(0.75, 2, 3)["edge_fraction"] < 1e-9


def test_doubly_exponential_bound():
    # Section 3.1: beta_{I+1} <= beta_I^{(k-1)(r-1)} r c / ((k-1)!)^{r-1}.
    for k, r, c in [(2, 4, 0.7), (2, 3, 0.75), (3, 3, 1.4)]:
        lam = theory.survival(c, k, r, 40)
        beta = r * c
        for _ in range(40):
            nxt = theory.p_at_least(k - 1, beta) ** (r - 1) * r * c
            bound = beta ** ((k - 1) * (r - 1)) * r * c / math.factorial(k - 1) ** (r - 1)
            assert nxt <= bound * (1 + 1e-12) + 1e-300
            beta = nxt
        assert lam[-1] < 1e-12


def test_fibonacci_growth_rates():
    # Appendix B: phi_2 is the golden ratio (~1.61); phi_3 ~ 1.83; phi_4 ~ 1.92.
    assert theory.fibonacci_growth(2) == pytest.approx((1 + math.sqrt(5)) / 2, abs=1e-12)
    assert abs(theory.fibonacci_growth(3) - 1.83) < 0.01
    assert abs(theory.fibonacci_growth(4) - 1.92) < 0.01


def test_predicted_rounds_bracket_table1(golden):
    # Table 1, c=0.7: the measured mean is 12.5-13 rounds; the recursion predicts 13 at n=10^6.
    assert theory.predicted_rounds(0.70, 2, 4, 10 ** 6) == 13
    assert theory.predicted_rounds(0.70, 2, 4, 10 ** 4) in (12, 13)


def test_rounds_near_threshold_grow_like_inverse_sqrt_distance():
    # Theorem 5: below the threshold, Theta(sqrt(1/nu)) + O(log log n) rounds with
    # nu = c* - c.  In the recursion's prediction, a 4x smaller nu doubles the
    # rounds once the sqrt term dominates.
    cs = theory.cstar(2, 4)[0]
    rounds = [theory.predicted_rounds(cs - nu, 2, 4, 1 << 24) for nu in (4e-3, 1e-3, 2.5e-4, 6.25e-5)]
    for a, b in zip(rounds, rounds[1:]):
        assert 1.8 <= b / a <= 2.2, rounds


def test_measured_rounds_near_threshold_follow_the_recursion():
    # the round-synchronous simulator just below c*_{2,4}, n = 2^20, 4 seeds:
    # the mean round count lands on the recursion's first t with lambda_t n < 1/2
    from oracle import native
    from workloads import gen
    n = 1 << 20
    for c, tol in ((0.76, 1.5), (0.77, 0.15 * theory.predicted_rounds(0.77, 2, 4, n))):
        rs = [native.peel_rounds(n, gen.partitioned_edges(n, int(c * n), 4, 50 + s), 2).rounds
              for s in range(4)]
        assert abs(np.mean(rs) - theory.predicted_rounds(c, 2, 4, n)) <= tol, (c, rs)
