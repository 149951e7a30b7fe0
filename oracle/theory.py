"""Threshold and survival recursions of the paper, in float64 (test infrastructure only).

Used to size the synthetic workloads and to give the statistical checks their
expected values; none of it is on the peeling path, which is integer and exact.

* ``cstar(k, r)``: the k-core threshold edge density c*_{k,r}, eq. (cstar) of
  Section 2: the minimum over x > 0 of x / (r (1 - e^{-x} S_{k-2}(x))^{r-1}),
  with S_a(x) = sum_{j=0}^{a} x^j / j!.
* ``survival(c, k, r, t)``: the idealised branching recursion of Section 3.1:
  beta_1 = r c, rho_i = 1 - e^{-beta_i} S_{k-2}(beta_i),
  lambda_i = 1 - e^{-beta_i} S_{k-1}(beta_i) (eq. lambdairecursion),
  beta_{i+1} = rho_i^{r-1} r c (eq. betairecursion).  lambda_t n predicts the
  number of vertices left after t rounds (Table 2, "Prediction").
* ``fixed_point(c, k, r)``: the limit beta of eq. (fixedpoint) above the
  threshold, the core fraction lambda and the contraction factor f'(0) of
  eq. (a1) (Section 4).
* ``subtable_survival(c, k, r, rounds)``: the subtable recursion of Appendix B,
  eq. (newlambdaij) and the averaged lambda'_{i,j} printed in Table 4.
"""
from __future__ import annotations

import math


def poisson_tail_sum(a: int, x: float) -> float:
    """S_a(x) = sum_{j=0}^{a} x^j / j! (0 for a < 0)."""
    if a < 0:
        return 0.0
    term, acc = 1.0, 1.0
    for j in range(1, a + 1):
        term *= x / j
        acc += term
    return acc


def p_at_least(a: int, mean: float) -> float:
    """Pr(Poisson(mean) >= a) = 1 - e^{-mean} S_{a-1}(mean).

    When the tail is small (mean below a) it is summed term by term, which
    avoids the cancellation of 1 - (something close to 1).
    """
    if a <= 0:
        return 1.0
    if mean < a:
        term = math.exp(-mean)
        for j in range(1, a + 1):
            term *= mean / j
        acc, j = 0.0, a
        while term > 0.0 and term > acc * 1e-18:
            acc += term
            j += 1
            term *= mean / j
        return acc
    return 1.0 - math.exp(-mean) * poisson_tail_sum(a - 1, mean)


def threshold_objective(x: float, k: int, r: int) -> float:
    """x / (r (1 - e^{-x} S_{k-2}(x))^{r-1}), the function minimised in eq. (cstar)."""
    inner = 1.0 - math.exp(-x) * poisson_tail_sum(k - 2, x)
    return x / (r * inner ** (r - 1))


def cstar(k: int, r: int) -> tuple[float, float]:
    """(c*_{k,r}, x*) of eq. (cstar): a global grid on (0, 50], then golden-section refinement."""
    if k < 1 or r < 2 or (k == 2 and r == 2):
        raise ValueError("threshold defined for k, r >= 2 except k = r = 2")
    step = 1e-3
    best_x, best_f = step, threshold_objective(step, k, r)
    x = step
    while x <= 50.0:
        f = threshold_objective(x, k, r)
        if f < best_f:
            best_x, best_f = x, f
        x += step
    lo, hi = max(best_x - step, 1e-9), best_x + step
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = hi - g * (hi - lo), lo + g * (hi - lo)
    fa, fb = threshold_objective(a, k, r), threshold_objective(b, k, r)
    while hi - lo > 1e-12:
        if fa < fb:
            hi, b, fb = b, a, fa
            a = hi - g * (hi - lo)
            fa = threshold_objective(a, k, r)
        else:
            lo, a, fa = a, b, fb
            b = lo + g * (hi - lo)
            fb = threshold_objective(b, k, r)
    xs = 0.5 * (lo + hi)
    return threshold_objective(xs, k, r), xs


def survival(c: float, k: int, r: int, t: int) -> list[float]:
    """[lambda_1, ..., lambda_t]: predicted fraction of vertices left after each round."""
    out = []
    beta = r * c  # beta_1 = rho_0^{r-1} r c with rho_0 = 1
    for _ in range(t):
        out.append(p_at_least(k, beta))
        rho = p_at_least(k - 1, beta)
        beta = rho ** (r - 1) * r * c
    return out


def predicted_rounds(c: float, k: int, r: int, n: int, cap: int = 10000) -> int:
    """First t with lambda_t n < 1/2 (cap if it never happens)."""
    for t, lam in enumerate(survival(c, k, r, cap), start=1):
        if lam * n < 0.5:
            return t
    return cap


def fixed_point(c: float, k: int, r: int, iters: int = 100000) -> dict:
    """Limit of the beta recursion from beta_1 = r c, the core fraction and f'(0)."""
    beta = r * c
    for _ in range(iters):
        nb = p_at_least(k - 1, beta) ** (r - 1) * r * c
        if abs(nb - beta) < 1e-15:
            beta = nb
            break
        beta = nb
    lam = p_at_least(k, beta)
    rho = p_at_least(k - 1, beta)
    if beta > 1e-12:
        fprime = ((r - 1) * beta * math.exp(-beta) / rho) * beta ** (k - 2) / math.factorial(k - 2)
    else:
        fprime = 0.0
    # An edge survives when all r of its vertices keep >= k-1 other surviving edges.
    edge_frac = rho ** r
    return {"beta": beta, "lambda": lam, "fprime0": fprime, "edge_fraction": edge_frac}


def subtable_survival(c: float, k: int, r: int, rounds: int):
    """Table 4 predictions: [((i, j), lambda'_{i,j}), ...] for i = 1..rounds, j = 1..r."""
    rho_prev = [1.0] * r      # rho_{0,j}
    lam_prev = [1.0] * r      # lambda_{0,j}
    out = []
    for i in range(1, rounds + 1):
        rho_cur = [0.0] * r
        lam_cur = [0.0] * r
        for j in range(r):
            prod = 1.0
            for h in range(j):
                prod *= rho_cur[h]
            for h in range(j + 1, r):
                prod *= rho_prev[h]
            beta = r * c * prod
            rho_cur[j] = p_at_least(k - 1, beta)
            lam_cur[j] = p_at_least(k, beta)
            avg = (sum(lam_cur[: j + 1]) + sum(lam_prev[j + 1:])) / r
            out.append(((i, j + 1), avg))
        rho_prev, lam_prev = rho_cur, lam_cur
    return out


def fibonacci_growth(order: int) -> float:
    """Growth rate of the Fibonacci sequence of the given order (each term sums the previous `order`)."""
    # Largest real root of x^order = x^{order-1} + ... + 1, by bisection on (1, 2].
    lo, hi = 1.0, 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid ** order - sum(mid ** p for p in range(order)) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)
