"""Exact rational arithmetic for pinning the oracle -- TEST INFRASTRUCTURE ONLY.

Independent of oracle.c: Python ``fractions.Fraction`` values, no floating
point rounding anywhere.  Used on tiny inputs to check that
  * each directed-rounding primitive returns the correctly rounded bound
    (the largest double <= the exact lower bound, the smallest double >= the
    exact upper bound);
  * every enclosure contains the exact value of F at points of the box
    (the enclosure property {F(x) : x in B} subset []F(B), Sec. 3.2);
  * exact interval Horner (the same formulas, no rounding) is contained in the
    rounded one, i.e. rounding is outward at every step.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def F(x) -> Fraction:
    return Fraction(float(x))


def next_up(x: float) -> float:
    return math.nextafter(x, math.inf)


def next_down(x: float) -> float:
    return math.nextafter(x, -math.inf)


def is_round_down(lo: float, exact: Fraction) -> bool:
    """lo == RD(exact): lo <= exact < next double above lo."""
    return F(lo) <= exact and (math.isinf(next_up(lo)) or F(next_up(lo)) > exact)


def is_round_up(hi: float, exact: Fraction) -> bool:
    return F(hi) >= exact and (math.isinf(next_down(hi)) or F(next_down(hi)) < exact)


def exact_mul(x, y):
    ps = [F(a) * F(b) for a in x for b in y]
    return min(ps), max(ps)


def exact_add(x, y):
    return F(x[0]) + F(y[0]), F(x[1]) + F(y[1])


# ---- exact interval Horner with Fraction endpoints (same operation order) ----

def _qmul(x, y):
    ps = [x[0] * y[0], x[0] * y[1], x[1] * y[0], x[1] * y[1]]
    return min(ps), max(ps)


def _qadd(x, y):
    return x[0] + y[0], x[1] + y[1]


def exact_muladd(x, y, c):
    """Exact range of the set x*y + c: (min P + c_lo, max P + c_hi)."""
    lo, hi = exact_mul(x, y)
    return lo + F(c[0]), hi + F(c[1])


def round_down_q(q: Fraction) -> float:
    """The largest double <= q (zero as +0)."""
    if q == 0:
        return 0.0
    x = float(q)  # correctly rounded to nearest
    return next_down(x) if F(x) > q else x


def round_up_q(q: Fraction) -> float:
    """The smallest double >= q (zero as +0)."""
    if q == 0:
        return 0.0
    x = float(q)
    return next_up(x) if F(x) < q else x


def stepwise_rounded_horner(coefs, cell) -> tuple:
    """Univariate interval Horner (descending exponents) in which every step
    J*I + c_e is computed exactly from the previous rounded J and then rounded
    outward once per endpoint.  coefs[e] = (lo, hi) of c_e."""
    J = (F(coefs[-1][0]), F(coefs[-1][1]))
    J = (round_down_q(J[0]), round_up_q(J[1]))
    for e in range(len(coefs) - 2, -1, -1):
        lo, hi = exact_muladd(J, cell, coefs[e])
        J = (round_down_q(lo), round_up_q(hi))
    return J


def exact_interval_eval(cube: np.ndarray, d: int, box) -> tuple:
    """Interval Horner in exact rationals, nested in the canonical order
    (x1 innermost, descending exponents)."""
    k = cube.ndim
    B = [(F(box[j][0]), F(box[j][1])) for j in range(k)]
    e = [0] * k

    def value(s, rem):
        acc = None
        for es in range(rem, -1, -1):
            e[s - 1] = es
            if s == 1:
                c = F(cube[tuple(e)])
                coef = (c, c)
            else:
                coef = value(s - 1, rem - es)
            acc = coef if acc is None else _qadd(_qmul(acc, B[s - 1]), coef)
        return acc

    return value(k, d)


def exact_point_value(cube: np.ndarray, d: int, x) -> Fraction:
    """Exact F(x) for a rational point x (sum of monomials, no Horner)."""
    k = cube.ndim
    xs = [Fraction(v) if isinstance(v, Fraction) else F(v) for v in x]
    total = Fraction(0)
    for e in np.argwhere(cube != 0):
        if int(e.sum()) > d:
            continue
        term = F(cube[tuple(e)])
        for j in range(k):
            term *= xs[j] ** int(e[j])
        total += term
    return total


def exact_box_range(poly_terms: dict, box) -> tuple:
    """Exact min and max over a box of a separable quadratic sum_j a_j x_j^2 + sum_j b_j x_j + c
    (poly_terms: {'a': [...], 'b': [...], 'c': c}), used for the closed-form sets."""
    lo = F(poly_terms.get("c", 0.0)); hi = lo
    for j, (u, v) in enumerate(box):
        a = F(poly_terms["a"][j]) if "a" in poly_terms else Fraction(0)
        b = F(poly_terms["b"][j]) if "b" in poly_terms else Fraction(0)
        u = F(u); v = F(v)
        cands = [a * u * u + b * u, a * v * v + b * v]
        if a != 0:
            xs = -b / (2 * a)
            if u <= xs <= v:
                cands.append(a * xs * xs + b * xs)
        lo += min(cands); hi += max(cands)
    return lo, hi
