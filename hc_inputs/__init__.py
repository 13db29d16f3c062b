"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws random numbers and lays out polynomial-system *structure*
(which monomial sits in which equation).  It holds none of the homotopy method's
arithmetic: no evaluation, no solving, no tracking.  Both the CPU oracle and the
HIP path take what it returns as plain arrays.

Workloads follow the batched dense-quadratic setting of the method (a target
system F solved from a total-degree start system, section 3, Eq. (1)):

* every equation carries all C(n+2, 2) monomials of degree <= 2, in the order
  1, x_1..x_n, then x_a*x_b for a <= b lexicographically;
* coefficients are i.i.d. standard complex Gaussian CN(0, 1): real and imaginary
  parts independently N(0, 1/2);
* one random unit-modulus gamma = exp(2*pi*i*theta), theta ~ U[0, 1), per instance.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, Tuple

import numpy as np

__all__ = [
    "PolySystem",
    "dense_quadratic_monomials",
    "dense_quadratic_system",
    "complex_gaussian",
    "dense_quadratic_instances",
    "unit_gammas",
    "monomials_upto",
    "support_system",
    "support_instances",
    "WORKLOADS",
    "workload",
]


@dataclasses.dataclass(frozen=True)
class PolySystem:
    """Structure of a square polynomial system F(x; c) = 0 with n equations in n unknowns.

    Term k belongs to equation ``term_eq[k]`` and is c_k * prod_j x_j ** term_exp[k, j];
    the coefficient vector c (length n_terms) is supplied per instance.
    """

    n: int
    term_eq: np.ndarray   # int32 [n_terms]
    term_exp: np.ndarray  # int32 [n_terms, n]

    @property
    def n_terms(self) -> int:
        return int(self.term_eq.shape[0])


def dense_quadratic_monomials(n: int) -> np.ndarray:
    """Exponent vectors of all monomials of degree <= 2 in n unknowns, [C(n+2,2), n] int32.

    Order: 1, x_1, ..., x_n, then x_a*x_b for a <= b in lexicographic order.
    """
    rows = [np.zeros(n, np.int32)]
    for j in range(n):
        e = np.zeros(n, np.int32)
        e[j] = 1
        rows.append(e)
    for a in range(n):
        for b in range(a, n):
            e = np.zeros(n, np.int32)
            e[a] += 1
            e[b] += 1
            rows.append(e)
    return np.stack(rows).astype(np.int32)


def dense_quadratic_system(n: int) -> PolySystem:
    """n dense quadratic equations: equation i holds every monomial of degree <= 2."""
    mons = dense_quadratic_monomials(n)
    T = mons.shape[0]
    term_eq = np.repeat(np.arange(n, dtype=np.int32), T)
    term_exp = np.tile(mons, (n, 1)).astype(np.int32)
    return PolySystem(n=n, term_eq=term_eq, term_exp=term_exp)


def monomials_upto(n: int, deg: int, vars_) -> np.ndarray:
    """Exponent vectors (length n) of every monomial of degree <= deg in the
    unknowns listed in vars_, [m, n] int32, in graded lexicographic order."""
    vars_ = list(vars_)
    rows = []

    def rec(i, left, e):
        if i == len(vars_):
            rows.append(e.copy())
            return
        for a in range(left + 1):
            e[vars_[i]] = a
            rec(i + 1, left - a, e)
        e[vars_[i]] = 0

    rec(0, deg, np.zeros(n, np.int32))
    rows.sort(key=lambda r: (int(r.sum()), tuple(-r)))
    return np.stack(rows).astype(np.int32)


def support_system(n: int, spec) -> PolySystem:
    """Equation i holds every monomial of degree <= d_i in the unknowns V_i, for
    spec = [(d_1, V_1), ..., (d_n, V_n)]: dense on its own support, of degree d_i."""
    eqs, exps = [], []
    for i, (d, vs) in enumerate(spec):
        m = monomials_upto(n, d, vs)
        eqs.append(np.full(len(m), i, np.int32))
        exps.append(m)
    return PolySystem(n=n, term_eq=np.concatenate(eqs), term_exp=np.concatenate(exps).astype(np.int32))


def support_instances(n: int, spec, n_inst: int, seed: int) -> Tuple[PolySystem, np.ndarray, np.ndarray]:
    """support_system with CN(0, 1) coefficients and unit gammas."""
    sys_ = support_system(n, spec)
    rng = np.random.default_rng(seed)
    coef = complex_gaussian(rng, (n_inst, sys_.n_terms))
    gam = unit_gammas(rng, n_inst)
    return sys_, np.ascontiguousarray(coef), np.ascontiguousarray(gam)


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """CN(0, 1) samples: (N(0,1) + i N(0,1)) / sqrt(2)."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def unit_gammas(rng: np.random.Generator, n_inst: int) -> np.ndarray:
    """n_inst random unit-modulus complex constants exp(2 pi i theta), theta ~ U[0,1)."""
    theta = rng.random(n_inst)
    return np.exp(2j * np.pi * theta)


def dense_quadratic_instances(n: int, n_inst: int, seed: int) -> Tuple[PolySystem, np.ndarray, np.ndarray]:
    """(structure, coefficients [n_inst, n*T] complex128, gammas [n_inst] complex128)."""
    sys_ = dense_quadratic_system(n)
    rng = np.random.default_rng(seed)
    coef = complex_gaussian(rng, (n_inst, sys_.n_terms))
    gam = unit_gammas(rng, n_inst)
    return sys_, np.ascontiguousarray(coef), np.ascontiguousarray(gam)


# Workloads of the batched total-degree setting.  "tracks" = start solutions per
# instance = Bezout number 2**n of a quadratic system.
WORKLOADS: Dict[str, dict] = {
    # one instance, n = 3, 8 tracks, complex FP64: the latency-bound small case
    "dense3_single": dict(n=3, n_inst=1, seed=1),
    # 512 instances, n = 8, 256 tracks each (131,072 tracks): the throughput case
    "dense8_batch512": dict(n=8, n_inst=512, seed=2),
}


def workload(name: str, n_inst: int | None = None):
    """Instances of a named workload; ``n_inst`` takes the first instances only."""
    spec = WORKLOADS[name]
    sys_, coef, gam = dense_quadratic_instances(spec["n"], spec["n_inst"], spec["seed"])
    if n_inst is not None:
        coef, gam = coef[:n_inst], gam[:n_inst]
    return sys_, coef, gam
