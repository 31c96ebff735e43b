"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic.  Polynomials are returned as dense coefficient cubes
``c[e1, ..., ek]`` (numpy float64, C order, side d+1) whose entries outside the
total-degree simplex e1+...+ek <= d are zero.  The random coefficients are
drawn once, in C order over the cube, skipping the entries outside the
simplex, from ``numpy.random.Generator(PCG64(SeedSequence(seed)))``.

The workloads stand in for the random dense systems of the paper's
experiments (Sec. 4.1, Table 1: random total-degree polynomials, one, k-1 or k
equations in k variables); the distributions, domain [-1, 1]^k and depths are
the ones fixed for this implementation:

* ``tiny``   : k=2, d=20, integer coefficients uniform in [-100, 100], depth 8.
* ``surface``: k=3, d=40, N(0,1) coefficients, depth 9.
* ``points`` : three polynomials, k=3, d=20, uniform in [-10, 10], depth 9.
* ``curve``  : two polynomials, k=3, d=100, N(0,1), depth 10 (the paper's
  headline problem: a curve cut out by two trivariate degree-100 equations,
  Sec. 1.2 and Table 1, 3D curves, d=100).
* ``batch``  : 64 single-polynomial trivariate problems, degrees uniform in
  {10..60}, N(0,1), depth 8.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def simplex_mask(k: int, d: int) -> np.ndarray:
    """Boolean cube (side d+1) marking exponent tuples with total degree <= d."""
    grids = np.indices((d + 1,) * k)
    return grids.sum(axis=0) <= d


def n_monomials(k: int, d: int) -> int:
    """Number of exponent tuples of total degree <= d in k variables."""
    return math.comb(d + k, k)


def _fill_simplex(k: int, d: int, values: np.ndarray) -> np.ndarray:
    cube = np.zeros((d + 1,) * k, dtype=np.float64)
    mask = simplex_mask(k, d)
    cube[mask] = values  # boolean indexing walks the cube in C order
    return cube


def random_poly(k: int, d: int, rng: np.random.Generator, dist: str = "normal") -> np.ndarray:
    """Dense coefficient cube of a random polynomial of total degree d."""
    m = n_monomials(k, d)
    if dist == "normal":
        vals = rng.standard_normal(m)
    elif dist == "int100":
        vals = rng.integers(-100, 100, size=m, endpoint=True).astype(np.float64)
    elif dist == "uniform10":
        vals = rng.uniform(-10.0, 10.0, size=m)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return _fill_simplex(k, d, vals)


def _gen(seed) -> np.random.Generator:
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    return np.random.Generator(np.random.PCG64(ss))


@dataclass
class Workload:
    """A subdivision problem: one system of polynomials on [dom]^k to a depth."""
    name: str
    k: int
    depth: int
    polys: list  # list of dense coefficient cubes (one system)
    dom: tuple = (-1.0, 1.0)
    systems: list = field(default_factory=list)  # batched form: list of lists of cubes

    @property
    def degree(self) -> int:
        return max(p.shape[0] - 1 for p in self.polys)

    def domain(self) -> np.ndarray:
        return np.array([self.dom[0], self.dom[1]] * self.k, dtype=np.float64)


def tiny(seed: int = 1) -> Workload:
    """One bivariate degree-20 polynomial, integer coefficients, depth 8."""
    return Workload("tiny_k2_d20", 2, 8, [random_poly(2, 20, _gen(seed), "int100")])


def surface(seed: int = 2) -> Workload:
    """One trivariate degree-40 polynomial, N(0,1) coefficients, depth 9."""
    return Workload("surface_k3_d40", 3, 9, [random_poly(3, 40, _gen(seed), "normal")])


def curve(seed: int = 3, degree: int = 100, depth: int = 10) -> Workload:
    """Two trivariate degree-100 polynomials (a space curve), depth 10."""
    kids = np.random.SeedSequence(seed).spawn(2)
    polys = [random_poly(3, degree, _gen(s), "normal") for s in kids]
    return Workload(f"curve_k3_d{degree}", 3, depth, polys)


def points(seed: int = 6, k: int = 3, degree: int = 20, depth: int = 9) -> Workload:
    """k polynomials in k variables (isolated points), coefficients uniform
    in [-10, 10] as in the random-polynomial experiments (Sec. 4.1), depth 9
    (boxes of width 2^-8 on [-1, 1])."""
    kids = np.random.SeedSequence(seed).spawn(k)
    polys = [random_poly(k, degree, _gen(s), "uniform10") for s in kids]
    return Workload(f"points_k{k}_d{degree}", k, depth, polys)


def batch(seed: int = 5, count: int = 64, dmin: int = 10, dmax: int = 60, depth: int = 8) -> Workload:
    """`count` independent trivariate problems with degrees uniform in [dmin, dmax]."""
    ss = np.random.SeedSequence(seed)
    degrees = _gen(ss).integers(dmin, dmax, size=count, endpoint=True)
    kids = ss.spawn(count)
    systems = [[random_poly(3, int(dg), _gen(s), "normal")] for dg, s in zip(degrees, kids)]
    w = Workload(f"batch{count}_k3_d{dmin}-{dmax}", 3, depth, systems[0], systems=systems)
    return w


def small_random(k: int, d: int, seed: int, dist: str = "normal", npolys: int = 1) -> list:
    """Small random systems for parity and property tests."""
    kids = np.random.SeedSequence(seed).spawn(npolys)
    return [random_poly(k, d, _gen(s), dist) for s in kids]


# ---------------------------------------------------------------------------
# Closed-form polynomials (coefficients exactly representable unless noted).
# ---------------------------------------------------------------------------

def monomial_poly(k: int, d: int, terms: dict) -> np.ndarray:
    """Dense cube from {exponent tuple: coefficient}."""
    cube = np.zeros((d + 1,) * k, dtype=np.float64)
    for e, c in terms.items():
        assert len(e) == k and sum(e) <= d
        cube[tuple(e)] = c
    return cube


def circle() -> np.ndarray:
    """x1^2 + x2^2 - 1/2."""
    return monomial_poly(2, 2, {(2, 0): 1.0, (0, 2): 1.0, (0, 0): -0.5})


def sphere() -> np.ndarray:
    """x1^2 + x2^2 + x3^2 - 1/2."""
    return monomial_poly(3, 2, {(2, 0, 0): 1.0, (0, 2, 0): 1.0, (0, 0, 2): 1.0, (0, 0, 0): -0.5})


def plane_x3(c: float = 1.0 / 3.0, d: int = 2) -> np.ndarray:
    """x3 - c (c rounded to the nearest double), padded to degree d."""
    return monomial_poly(3, d, {(0, 0, 1): 1.0, (0, 0, 0): -c})


def plane_x1(k: int, c: float, d: int = 1) -> np.ndarray:
    """x1 - c in k variables."""
    e1 = (1,) + (0,) * (k - 1)
    return monomial_poly(k, d, {e1: 1.0, (0,) * k: -c})
