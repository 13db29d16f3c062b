"""Start solutions of a generic parameter instance by monodromy, with every path
tracked on the GPU (the paper computes its vision start sets offline by
monodromy; published method: Duff, Hill, Jensen, Lee, Leykin, Sommars, IMA J.
Numer. Anal. 2019).

1. A fabricated exact pair (p0, x0): x0 solves the instance p0.
2. Loops p0 -> pa -> pb -> p0 over random complex parameter points carry every
   known solution around; distinct new endpoints join the set (closed under
   the family's known symmetries).  The merge runs on the device
   (hc_distinct_device).
3. Stop after `stall` loops without growth, at `target` solutions, or after
   `max_loops`.

A family supplies: system() (a PolySystem), coef(p) (the coefficient vector of
parameters p), waypoints(p_from, p_to) (parameter points of a path on whose
legs the coefficients are affine in t, so each leg is one linear coefficient
homotopy), random(rng), fabricate(rng) -> (p0, x0), orbit(x) (images of
solutions [N, n] under known symmetries, [m, N, n]) or None.  LinearFamily is
the one whose parameters are the coefficients themselves.
"""
from __future__ import annotations

import time
from typing import Optional

import numpy as np

from . import hc as _hc


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


class LinearFamily:
    """Every coefficient is a parameter: p is the coefficient vector."""

    def __init__(self, system):
        self._system = system

    def system(self):
        return self._system

    @staticmethod
    def coef(p):
        return np.asarray(p, np.complex128)

    @staticmethod
    def waypoints(p_from, p_to):
        return [np.asarray(p_from, np.complex128), np.asarray(p_to, np.complex128)]

    def random(self, rng):
        return _cn(rng, self._system.n_terms)

    def fabricate(self, rng):
        """Random complex x0 and coefficients; per equation the coefficient of
        the term with the largest monomial value at x0 is solved for."""
        S = self._system
        x0 = _cn(rng, S.n)
        c0 = _cn(rng, S.n_terms)
        mono = np.prod(x0[None, :] ** np.asarray(S.term_exp), axis=1)
        for i in range(S.n):
            ks = np.flatnonzero(np.asarray(S.term_eq) == i)
            k = ks[np.argmax(np.abs(mono[ks]))]
            others = ks[ks != k]
            c0[k] = -np.sum(c0[others] * mono[others]) / mono[k]
        return c0, x0

    @staticmethod
    def orbit(x):
        return None


def distinct(sols: np.ndarray, tol: float = 1e-8) -> np.ndarray:
    """Rows of sols with near-duplicates (relative inf-norm distance <= tol,
    relative to the larger row) removed, the first of equal rows kept.  Rows
    are keyed by a fixed random real projection of the row scaled by
    s = max(1, |x|_inf); two rows within tol of each other differ by at most
    2 tol after scaling, so their keys by at most 4 |w|_1 tol, and each row is
    compared only with the earlier rows inside that window of the sorted keys."""
    sols = np.asarray(sols)
    n_rows = len(sols)
    if n_rows <= 1:
        return sols
    w = np.random.default_rng(12345).standard_normal(sols.shape[1])
    scale = np.maximum(1.0, np.max(np.abs(sols), axis=1))
    y = sols / scale[:, None]
    key = (y @ w).real + (y @ w[::-1]).imag
    reach = 4.0 * np.abs(w).sum() * tol * (1.0 + 1e-9)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    keep = np.zeros(n_rows, bool)
    for i in range(n_rows):
        lo = np.searchsorted(ks, key[i] - reach, side="left")
        hi = np.searchsorted(ks, key[i] + reach, side="right")
        dup = False
        for j in order[lo:hi]:
            if j < i and keep[j] and np.max(np.abs(sols[i] - sols[j])) <= tol * max(scale[i], scale[j]):
                dup = True
                break
        keep[i] = not dup
    return sols[keep]


def distinct_on_device(ctx, sols: np.ndarray, tol: float = 1e-8) -> np.ndarray:
    """`distinct` by the library's device kernel (hc_distinct_device): a row is
    dropped when any earlier row lies within tol (the host version compares with
    the kept rows only; the two differ only where near-duplicates chain)."""
    import torch
    sols = np.asarray(sols, np.complex128)
    if len(sols) <= 1:
        return sols
    keep = ctx.distinct_device(torch.from_numpy(np.ascontiguousarray(sols)).to("cuda"), tol)
    return sols[keep.cpu().numpy().astype(bool)]


def _close(sols, orbit, tol, dedup=distinct):
    if orbit is None or len(sols) == 0:
        return sols
    imgs = orbit(sols)
    if imgs is None:
        return sols
    return dedup(np.concatenate([sols, np.asarray(imgs).reshape(-1, sols.shape[1])]), tol)


def _path(ctx, handle, family, p_from, p_to, sols, opts):
    pts = family.waypoints(p_from, p_to)
    for a, b in zip(pts[:-1], pts[1:]):
        if len(sols) == 0:
            break
        ep, st, _ = ctx.track(handle, family.coef(b)[None, :], start=sols, p_start=family.coef(a), opts=opts)
        sols = ep[0][st[0] == _hc.HC_T_SUCCESS]
    return sols


def monodromy(ctx, family, seed: int = 0, stall: int = 10, max_loops: int = 500, target: Optional[int] = None,
              precision: str = "fp64", tol: float = 1e-6, log=None):
    """(p0, solutions [N, n]) of a generic member of `family` by monodromy loops
    on the GPU (`ctx`: a Context).  Endpoints closer than tol (relative) are one
    root: refinement of badly conditioned roots leaves copies ~1e-8 apart."""
    system = family.system()
    handle = ctx.load_system(system, kind=_hc.HC_PARAMETER)
    opts = _hc.default_opts(precision=precision)
    rng = np.random.default_rng(seed)
    p0, x0 = family.fabricate(rng)

    def dedup(x, tl):
        return distinct_on_device(ctx, x, tl)

    sols = _close(np.asarray(x0)[None, :], family.orbit, tol, dedup)
    quiet = 0
    t0 = time.time()
    try:
        for loop in range(max_loops):
            pa, pb = family.random(rng), family.random(rng)
            xa = _path(ctx, handle, family, p0, pa, sols, opts)
            xb = _path(ctx, handle, family, pa, pb, xa, opts)
            back = _path(ctx, handle, family, pb, p0, xb, opts)
            merged = _close(dedup(np.concatenate([sols, back]), tol), family.orbit, tol, dedup) if len(back) \
                else sols
            grew = len(merged) - len(sols)
            sols = merged
            quiet = 0 if grew > 0 else quiet + 1
            if log is not None:
                log(f"loop {loop}: {len(sols)} solutions (+{grew}), {time.time() - t0:.1f} s")
            if quiet >= stall or (target is not None and len(sols) >= target):
                break
    finally:
        ctx.free_system(handle)
    return p0, sols
