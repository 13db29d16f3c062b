"""Start solutions of a generic parameter instance by monodromy.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): it writes the start
instance and start solutions that the parameter-homotopy workloads track from.
Those are inputs, consumed alike by the oracle and by the HIP path.

The paper solves its vision problems from a random complex start instance whose
solutions were computed offline by monodromy (section 7).  This restates the
published method (Duff, Hill, Jensen, Lee, Leykin, Sommars, IMA J. Numer. Anal.
2019), with the oracle's FP64 tracker doing every path:

1. fabricate one exact pair: random complex x0 and coefficients c0, then one
   coefficient per equation is solved for so that F(x0; c0) = 0;
2. loop c0 -> ca -> cb -> c0 over fresh random complex instances ca, cb (linear
   coefficient segments: the paper's parameter homotopy), carrying every known
   solution around the loop; new distinct endpoints join the set;
3. stop once the set has not grown for `stall` consecutive loops.

Structured families (coefficients that are functions of fewer parameters,
such as products of image coordinates) loop in parameter space instead; each
segment follows the family's waypoints so that every leg is a linear
coefficient homotopy that stays inside the family (`monodromy_family`).

Usage (writes tests/golden/start_triang4.npz, start_triang3.npz,
start_trifocal.npz or start_fivept.npz and prints its sha256):

    python -m oracle.monodromy triang4
    python -m oracle.monodromy triang3
    python -m oracle.monodromy trifocal
    python -m oracle.monodromy fivept

The trifocal set can also be grown from a stored one (trifocal-resume
[--seed=S] [--checkpoint=PATH]); trifocal-check writes an independent run from
its own parameter point (tests/golden/trifocal_check.npz) and trifocal-compare
carries each run's set to the other's parameter point and records what either
misses.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

from . import LINEAR, SUCCESS, eval_system, residual, track

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _cn(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def monomials(system, x):
    """Value of every term's monomial at x."""
    return np.prod(np.asarray(x)[None, :] ** system.term_exp, axis=1)


def fabricate_pair(system, rng):
    """(c0, x0) with F(x0; c0) = 0 exactly up to rounding: per equation, the
    coefficient of its term with the largest monomial value is solved for."""
    x0 = _cn(rng, system.n)
    c0 = _cn(rng, system.n_terms)
    m = monomials(system, x0)
    for i in range(system.n):
        ks = np.flatnonzero(system.term_eq == i)
        k = ks[np.argmax(np.abs(m[ks]))]
        rest = np.sum(c0[ks] * m[ks]) - c0[k] * m[k]
        c0[k] = -rest / m[k]
    return c0, x0


def distinct_rows(sols, tol=1e-8):
    """Rows of `sols` with duplicates (relative inf-norm distance <= tol) removed;
    the first of equal rows is kept."""
    sols = np.asarray(sols)
    keep = []
    for k in range(len(sols)):
        if keep:
            y = sols[keep]
            d = np.max(np.abs(y - sols[k]), axis=1) / np.maximum(1.0, np.max(np.abs(y), axis=1))
            if np.min(d) <= tol:
                continue
        keep.append(k)
    return sols[keep]


def _segment(system, c_from, c_to, sols, n_threads):
    ep, st, _ = track(system, c_to[None, :], start=sols, coef0=c_from, kind=LINEAR, n_threads=n_threads)
    return ep[0][st[0] == SUCCESS]


def _close(sols, orbit):
    """sols together with their images under `orbit` (a map [N, n] -> [m, N, n]
    of known symmetries of the family), duplicates removed."""
    if orbit is None or len(sols) == 0:
        return sols
    return distinct_rows(np.concatenate([sols, orbit(sols).reshape(-1, sols.shape[1])]))


def _close_tol(sols, orbit, tol):
    """`_close` with a merge tolerance."""
    if orbit is None or len(sols) == 0:
        return sols
    return distinct_rows(np.concatenate([sols, orbit(sols).reshape(-1, sols.shape[1])]), tol)


def monodromy(system, seed=0, stall=10, max_loops=500, n_threads=None, log=print, orbit=None, target=None):
    """(c0, solutions [N, n]) of a generic instance of the linear-coefficient
    family with the support of `system`.  `orbit`, if given, maps solutions to
    the other members of their symmetry orbits (applied to every new solution);
    the loop also stops once `target` solutions are known."""
    rng = np.random.default_rng(seed)
    c0, x0 = fabricate_pair(system, rng)
    sols = _close(x0[None, :], orbit)
    quiet = 0
    t0 = time.time()
    for loop in range(max_loops):
        ca, cb = _cn(rng, system.n_terms), _cn(rng, system.n_terms)
        xa = _segment(system, c0, ca, sols, n_threads)
        xb = _segment(system, ca, cb, xa, n_threads)
        back = _segment(system, cb, c0, xb, n_threads)
        merged = _close(distinct_rows(np.concatenate([sols, back])), orbit) if len(back) else sols
        grew = len(merged) - len(sols)
        sols = merged
        quiet = 0 if grew > 0 else quiet + 1
        log(f"loop {loop}: {len(sols)} solutions (+{grew}), {time.time() - t0:.0f} s")
        if quiet >= stall or (target is not None and len(sols) >= target):
            break
    return c0, sols


def _path(family, system, p_from, p_to, sols, n_threads):
    """Endpoints of `sols` carried from parameters p_from to p_to: one linear
    coefficient homotopy per leg between the family's waypoints (on each leg
    the coefficients of the family are affine in t, so the path stays in the
    family)."""
    pts = family.waypoints(p_from, p_to)
    for a, b in zip(pts[:-1], pts[1:]):
        if len(sols) == 0:
            break
        sols = _segment(system, family.coef(a), family.coef(b), sols, n_threads)
    return sols


def monodromy_family(family, seed=0, stall=10, max_loops=500, n_threads=None, log=print, target=None,
                     on_loop=None, tol=1e-8, resume=None):
    """(p0, solutions [N, n]) of a generic member of a structured parameter
    family (one whose coefficients are not free: `family` supplies the system,
    c(p), the waypoints of a path between two parameter points, random
    parameter points, a fabricated start pair and the solution symmetries).
    Loops p0 -> pa -> pb -> p0 as in `monodromy`; on_loop(p0, sols), if given,
    sees the set after every loop.  Endpoints closer than `tol` (relative) are
    one solution.  resume = (p0, sols) continues the loops from a set found
    before (the seed then only draws the loop parameters)."""
    system = family.system()
    rng = np.random.default_rng(seed)
    if resume is None:
        p0, x0 = family.fabricate(rng)
        sols = _close(x0[None, :], family.orbit)
    else:
        p0, sols = resume
        sols = distinct_rows(np.asarray(sols), tol)
    quiet = 0
    t0 = time.time()
    for loop in range(max_loops):
        pa, pb = family.random(rng), family.random(rng)
        xa = _path(family, system, p0, pa, sols, n_threads)
        xb = _path(family, system, pa, pb, xa, n_threads)
        back = _path(family, system, pb, p0, xb, n_threads)
        merged = _close_tol(distinct_rows(np.concatenate([sols, back]), tol), family.orbit, tol) if len(back) \
            else sols
        grew = len(merged) - len(sols)
        sols = merged
        quiet = 0 if grew > 0 else quiet + 1
        log(f"loop {loop}: {len(sols)} solutions (+{grew}), {time.time() - t0:.0f} s")
        if on_loop is not None:
            on_loop(p0, sols)
        if quiet >= stall or (target is not None and len(sols) >= target):
            break
    return p0, sols


def check(system, c0, sols):
    """Every solution has a tiny residual and the set is pairwise distinct."""
    eta = max(residual(system, c0, x) for x in sols)
    d = len(distinct_rows(sols)) == len(sols)
    return eta, d


# A run ends after this many consecutive loops without a new solution.
TRIFOCAL_STALL = 10
# Roots of the trifocal family closer than this (relative) are one root: FP64
# refinement of its worst-conditioned roots (condition numbers up to 1e13)
# leaves copies ~1e-8 apart, while distinct roots are >= 1e-4 apart.
TRIFOCAL_MERGE_TOL = 1e-6
TRIFOCAL_CHECK_FILE = os.path.join(ROOT, "tests", "golden", "trifocal_check.npz")


def _save_trifocal(TF, S, p0, sols, out, **extra):
    eta, d = check(S, TF.coefficients(p0), sols)
    print(f"{len(sols)} solutions, max residual {eta:.2e}, distinct {d}", flush=True)
    np.savez(out, params0=p0, coef0=TF.coefficients(p0), solutions=sols, **extra)
    print(out, hashlib.sha256(open(out, "rb").read()).hexdigest(), flush=True)


def _trifocal_run(TF, seed, resume=None, checkpoint=None, n_threads=None):
    """Monodromy on the trifocal family to the stall rule; every loop's set is
    written to `checkpoint` (if given), so a stopped run can be resumed."""
    def on_loop(p0, sols):
        if checkpoint:
            np.savez(checkpoint, params0=p0, solutions=sols)
    log = lambda m: print(m, flush=True)  # noqa: E731
    return monodromy_family(TF.Family, seed=seed, stall=TRIFOCAL_STALL, max_loops=100000, log=log,
                            tol=TRIFOCAL_MERGE_TOL, resume=resume, on_loop=on_loop, n_threads=n_threads)


def _carry(TF, S, p_from, p_to, sols, n_threads=None):
    """Distinct finite endpoints of `sols` carried from p_from to p_to along the
    family's two legs."""
    out = _path(TF.Family, S, p_from, p_to, sols, n_threads)
    return distinct_rows(out, TRIFOCAL_MERGE_TOL) if len(out) else out


def _trifocal_main(cmd, opts):
    import hc_inputs.trifocal as TF
    S = TF.trifocal_system()
    ckpt = opts.get("checkpoint")
    nt = int(opts["threads"]) if "threads" in opts else None
    if cmd == "trifocal":
        # from one fabricated pair (seed 4) to the stall rule
        p0, sols = _trifocal_run(TF, 4, checkpoint=ckpt, n_threads=nt)
        _save_trifocal(TF, S, p0, sols, TF.START_FILE)
    elif cmd == "trifocal-resume":
        # more loops (drawn from --seed) on a set written before by this script:
        # the stored set, or the checkpoint of a stopped run
        src = ckpt if ckpt and os.path.exists(ckpt) else TF.START_FILE
        z = np.load(src)
        p0, sols = _trifocal_run(TF, int(opts.get("seed", 40)), resume=(z["params0"], z["solutions"]),
                                 checkpoint=ckpt, n_threads=nt)
        _save_trifocal(TF, S, p0, sols, TF.START_FILE)
    elif cmd == "trifocal-check":
        # an independent run: its own fabricated pair (seed 5), so its own
        # generic parameter point, to the stall rule
        if ckpt and os.path.exists(ckpt):
            z = np.load(ckpt)
            p0, sols = _trifocal_run(TF, int(opts.get("seed", 50)), resume=(z["params0"], z["solutions"]),
                                     checkpoint=ckpt, n_threads=nt)
        else:
            p0, sols = _trifocal_run(TF, 5, checkpoint=ckpt, n_threads=nt)
        _save_trifocal(TF, S, p0, sols, TRIFOCAL_CHECK_FILE)
    elif cmd == "trifocal-compare":
        # both sets carried to the other run's parameter point: a complete set
        # reaches every root of the other (what the homotopy loses on the way
        # is counted, not hidden)
        a, b = np.load(TF.START_FILE), np.load(TRIFOCAL_CHECK_FILE)
        ab = _carry(TF, S, b["params0"], a["params0"], b["solutions"], nt)
        ba = _carry(TF, S, a["params0"], b["params0"], a["solutions"], nt)

        def diff(x, ref):
            ref = np.asarray(ref)
            miss = 0
            for y in ref:
                d = np.max(np.abs(x - y), axis=1) / max(1.0, np.max(np.abs(y))) if len(x) else [np.inf]
                miss += np.min(d) > TRIFOCAL_MERGE_TOL
            return int(miss)
        rep = dict(n_start=len(a["solutions"]), n_check=len(b["solutions"]), check_carried=len(ab),
                   start_carried=len(ba), start_roots_not_reached=diff(ab, a["solutions"]),
                   check_roots_not_reached=diff(ba, b["solutions"]),
                   carried_not_in_start=diff(a["solutions"], ab), carried_not_in_check=diff(b["solutions"], ba))
        print(rep, flush=True)
        _save_trifocal(TF, S, b["params0"], b["solutions"], TRIFOCAL_CHECK_FILE,
                       compare=np.array([rep[k] for k in sorted(rep)]), compare_keys=np.array(sorted(rep)))
    else:
        raise SystemExit(f"unknown command {cmd}")


def main(argv):
    name = argv[1] if len(argv) > 1 else "triang4"
    opts = dict(a[2:].split("=", 1) for a in argv[2:] if a.startswith("--") and "=" in a)
    if name.startswith("trifocal"):
        _trifocal_main(name, opts)
        return
    if name == "fivept":
        import hc_inputs.fivept as FP
        S = FP.fivept_system()
        p0, sols = monodromy_family(FP.Family, seed=4, stall=10, max_loops=200)
        eta, d = check(S, FP.coefficients(p0), sols)
        print(f"{len(sols)} solutions, max residual {eta:.2e}, distinct {d}")
        np.savez(FP.START_FILE, params0=p0, coef0=FP.coefficients(p0), solutions=sols)
        print(FP.START_FILE, hashlib.sha256(open(FP.START_FILE, "rb").read()).hexdigest())
        return
    if name not in ("triang4", "triang3"):
        raise SystemExit(f"unknown family {name}")
    import hc_inputs.vision as V
    n_views = int(name[-1])
    S = V.triangulation_system(n_views)
    c0, sols = monodromy(S, seed=4)
    eta, d = check(S, c0, sols)
    print(f"{len(sols)} solutions, max residual {eta:.2e}, distinct {d}")
    out = os.path.join(ROOT, "tests", "golden", f"start_triang{n_views}.npz")
    np.savez(out, coef0=c0, solutions=sols)
    print(out, hashlib.sha256(open(out, "rb").read()).hexdigest())


if __name__ == "__main__":
    main(sys.argv)
