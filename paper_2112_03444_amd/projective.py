"""Projective (random-patch) tracking on top of the C ABI.

Paths whose roots lie at infinity diverge in affine coordinates and end only
when |x| passes the infinity bound (or the step size collapses).  Tracking in
projective space keeps them bounded: the system F(x) = 0 in n unknowns becomes
the homogeneous system F^(x, x_h) = 0 in n + 1 unknowns (every term of equation
i multiplied by x_h^(d_i - its degree)), closed by one random affine patch
equation a . (x, x_h) = 1.  Its total-degree homotopy has the same prod d_i
paths (the patch equation has degree 1); a root of F is (x, 1)/(a . (x, 1)) on
the patch, a root at infinity has x_h = 0.  The GPU tracks the (n + 1)-unknown
system through the same kernels; the endpoints are mapped back to x / x_h, and
those with |x_h| <= inf_tol |(x, x_h)|_inf are reported at infinity.

This is the random-patch half of end-game support; singular endpoints still end
with the tracker's own classification.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import hc as _hc


@dataclasses.dataclass(frozen=True)
class Homogenized:
    """The homogenized system with its patch equation: n = n_affine + 1
    unknowns (x_h last), the patch as the last equation (n_affine + 2 terms:
    x_0 .. x_h, constant)."""
    n: int
    term_eq: np.ndarray
    term_exp: np.ndarray
    n_affine: int

    @property
    def n_terms(self) -> int:
        return int(self.term_eq.shape[0])


def homogenize_system(system) -> Homogenized:
    """Structure of F^ plus the patch equation for a system with fields n,
    term_eq, term_exp."""
    n = int(system.n)
    eq = np.asarray(system.term_eq, np.int64)
    ex = np.asarray(system.term_exp, np.int64)
    deg = ex.sum(axis=1)
    d = np.zeros(n, np.int64)
    np.maximum.at(d, eq, deg)
    ex_h = np.concatenate([ex, (d[eq] - deg)[:, None]], axis=1)
    patch = np.concatenate([np.eye(n + 1, dtype=np.int64), np.zeros((1, n + 1), np.int64)])
    term_eq = np.concatenate([eq, np.full(n + 2, n)]).astype(np.int32)
    term_exp = np.concatenate([ex_h, patch]).astype(np.int32)
    return Homogenized(n + 1, term_eq, term_exp, n)


def random_patch(n_affine: int, rng: np.random.Generator) -> np.ndarray:
    """Patch coefficients a [n_affine + 1], i.i.d. CN(0, 1)."""
    return (rng.standard_normal(n_affine + 1) + 1j * rng.standard_normal(n_affine + 1)) / np.sqrt(2.0)


def coefficients(coef: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Coefficients of F^ plus the patch: the original term coefficients (the
    homogenizing powers change no coefficient), then a and -1."""
    c = np.atleast_2d(np.asarray(coef, np.complex128))
    tail = np.concatenate([np.asarray(a, np.complex128), [-1.0 + 0.0j]])
    return np.ascontiguousarray(np.concatenate([c, np.broadcast_to(tail, (c.shape[0], tail.size))], axis=1))


def dehomogenize(xh: np.ndarray, status: np.ndarray, inf_tol: float = 1e-8):
    """(affine endpoints x / x_h, status with the reached paths whose |x_h| is
    below inf_tol times the largest coordinate turned into AT_INFINITY).  At a
    root at infinity every term of an equation can vanish together, so its
    relative backward error is 0/0 and the refinement may have reported
    REFINE_FAILED: x_h decides for those too."""
    xh = np.asarray(xh)
    h = xh[..., -1]
    big = np.max(np.abs(xh), axis=-1)
    at_inf = np.abs(h) <= inf_tol * big
    with np.errstate(divide="ignore", invalid="ignore"):
        x = xh[..., :-1] / h[..., None]
    st = np.array(status, copy=True)
    reached = (st == _hc.HC_T_SUCCESS) | (st == _hc.HC_T_REFINE_FAILED)
    st[reached & at_inf] = _hc.HC_T_AT_INFINITY
    return x, st


def track_projective(ctx, system, coef, gamma, opts: Optional[_hc.Opts] = None, seed: int = 0,
                     inf_tol: float = 1e-8):
    """Total-degree tracking of `system` at the instances `coef` [n_inst,
    n_terms] in projective space on the GPU (ctx: a Context).  Returns the
    affine endpoints [n_inst, paths, n], status, info and the projective
    endpoints [n_inst, paths, n + 1]."""
    H = homogenize_system(system)
    a = random_patch(H.n_affine, np.random.default_rng(seed))
    handle = ctx.load_system(H)
    try:
        xh, st, info = ctx.track(handle, coefficients(coef, a), gamma, opts=opts)
    finally:
        ctx.free_system(handle)
    x, st2 = dehomogenize(xh, st, inf_tol)
    return x, st2, info, xh
