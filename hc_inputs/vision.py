"""Seeded synthetic instances of the N-view triangulation problem (section 4),
N = 4 (the build's main vision workload) and N = 3.

Like the rest of ``hc_inputs`` this module only lays out problem structure and
draws random scenes; it holds none of the homotopy method's arithmetic.

Formulation (section 4, N-view triangulation; the printed equations are garbled,
this is the reading the build uses).  A 3D point is seen in N views (N = 4 below) at
normalised image coordinates gamma_k = ((p_x - 320)/f, (p_y - 240)/f, 1).  The
optimal corrections (u_k, v_k) minimise sum_k u_k^2 + v_k^2 subject to the
epipolar constraints of every pair p = (i, j), i < j:

    c_p = g_j^T E_ij g_i = 0,      g_k = gamma_k - (u_k, v_k, 0)^T.

With one multiplier lambda_p per pair, the critical points of the Lagrangian
sum u^2 + v^2 + sum lambda_p c_p solve 14 equations in the 14 unknowns

    x = (u_1, v_1, ..., u_4, v_4, lambda_12, lambda_13, lambda_14, lambda_23, lambda_24, lambda_34):

    2 u_k + sum_{p containing k} lambda_p dc_p/du_k = 0      (8 gradient equations, 10 terms each)
    2 v_k + sum_{p containing k} lambda_p dc_p/dv_k = 0
    c_p = 0                                                  (6 constraints, 9 terms each)

134 terms, all of degree <= 2.  With N = 3: 9 unknowns (u_k, v_k, k < 3, and
lambda_12, lambda_13, lambda_23), 6 gradient equations of 7 terms and 3
constraints of 9 terms, 69 terms.

Calibration noise.  With essential matrices of one consistent set of camera
poses the six constraints are dependent wherever the corrected points are
consistent (those form a 3-dimensional set in the 8 correction coordinates, so
only 5 of the 6 constraint gradients are independent there): the multipliers
are then never unique and no critical point is isolated.  The paper's own
4-view experiment perturbs the poses; here each pair's relative pose is
perturbed independently (rotation by N(0, (0.5 deg)^2) per axis, translation by
N(0, (0.01 |t|)^2) per coordinate) before E_ij is formed, which makes the
critical points isolated.

Scene recipe: the point X ~ U[-1, 1]^3; camera k has its centre at 6 u_k (u_k
uniform on the unit sphere), looks at the origin (optical axis -u_k) with a
roll ~ U[0, 2 pi); f = 1000 px, 640 x 480 images, principal point (320, 240);
pixel noise N(0, sigma^2) per coordinate (sigma = 0.5 px); a scene whose point
falls outside an image is drawn again.  E_ij = [t]_x R with R = R_j R_i^T and
t = R_j (C_i - C_j) (so that x_j^T E_ij x_i = 0), scaled to unit Frobenius norm.

Parameter homotopy (section 6: the coefficients move linearly between a start
and a target instance): the start instance is one fixed generic member of the
same monomial-support family, coefficients i.i.d. CN(0, 1).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Tuple

import numpy as np

from . import PolySystem, complex_gaussian

N_VIEWS = 4                                   # the default: 4-view triangulation
FOCAL = 1000.0
WIDTH, HEIGHT = 640.0, 480.0
CX, CY = 320.0, 240.0


def pairs(n_views: int) -> List[Tuple[int, int]]:
    """The view pairs (i, j), i < j, in the order of their multipliers."""
    return list(itertools.combinations(range(n_views), 2))


def n_unknowns(n_views: int) -> int:
    return 2 * n_views + len(pairs(n_views))


PAIRS: List[Tuple[int, int]] = pairs(N_VIEWS)
N_UNK = n_unknowns(N_VIEWS)  # 14


def _u(k: int) -> int:
    return 2 * k


def _v(k: int) -> int:
    return 2 * k + 1


def _lam(p: int, n_views: int) -> int:
    return 2 * n_views + p


def _mono(n_unk: int, *idx: int) -> np.ndarray:
    e = np.zeros(n_unk, np.int32)
    for i in idx:
        e[i] += 1
    return e


def _structure(n_views: int):
    """(term_eq, term_exp, recipe): recipe[k] says how term k's coefficient is
    formed from (E, gamma) -- see ``_coefficients``."""
    prs, nu = pairs(n_views), n_unknowns(n_views)
    eq, ex, recipe = [], [], []
    # gradient equations: d/du_k and d/dv_k, k < n_views
    for k in range(n_views):
        for axis in (0, 1):               # 0: u_k, 1: v_k
            row = len(set(eq)) if eq else 0
            own = _u(k) if axis == 0 else _v(k)
            eq.append(row)
            ex.append(_mono(nu, own))
            recipe.append(("two",))
            for p, (i, j) in enumerate(prs):
                if k not in (i, j):
                    continue
                o = j if k == i else i   # the other view of the pair
                side = "i" if k == i else "j"
                lam = _lam(p, n_views)
                eq.append(row)
                ex.append(_mono(nu, lam))
                recipe.append(("gconst", p, side, axis))
                eq.append(row)
                ex.append(_mono(nu, lam, _u(o)))
                recipe.append(("glin", p, side, axis, 0))
                eq.append(row)
                ex.append(_mono(nu, lam, _v(o)))
                recipe.append(("glin", p, side, axis, 1))
    # epipolar constraints
    for p, (i, j) in enumerate(prs):
        row = 2 * n_views + p
        terms = [((), ("cconst", p)),
                 ((_u(i),), ("ci", p, 0)), ((_v(i),), ("ci", p, 1)),
                 ((_u(j),), ("cj", p, 0)), ((_v(j),), ("cj", p, 1)),
                 ((_u(i), _u(j)), ("cq", p, 0, 0)), ((_u(i), _v(j)), ("cq", p, 0, 1)),
                 ((_v(i), _u(j)), ("cq", p, 1, 0)), ((_v(i), _v(j)), ("cq", p, 1, 1))]
        for idx, rc in terms:
            eq.append(row)
            ex.append(_mono(nu, *idx))
            recipe.append(rc)
    return np.asarray(eq, np.int32), np.stack(ex).astype(np.int32), recipe


_STRUCT = {nv: _structure(nv) for nv in (3, 4)}


def triangulation_system(n_views: int = N_VIEWS) -> PolySystem:
    """Structure of the N-view triangulation system (4 views: 14 x 14, 134
    terms; 3 views: 9 x 9, 69 terms)."""
    eq, ex, _ = _STRUCT[n_views]
    return PolySystem(n=n_unknowns(n_views), term_eq=eq.copy(), term_exp=ex.copy())


def _coefficients(E: np.ndarray, gam: np.ndarray) -> np.ndarray:
    """Coefficients of the system's terms for essential matrices E [pairs, 3, 3]
    and normalised image points gam [N, 3] (N = 4: 134 terms; N = 3: 69).

    With g_i = gamma_i - u_i e_0 - v_i e_1 (e_a the unit vectors) the constraint
    of pair (i, j) expands to
        c = gamma_j^T E gamma_i - u_i (gamma_j^T E e_0) - v_i (gamma_j^T E e_1)
            - u_j (e_0^T E gamma_i) - v_j (e_1^T E gamma_i)
            + u_i u_j E_00 + u_i v_j E_10 + v_i u_j E_01 + v_i v_j E_11,
    and its derivatives are read off the same expansion."""
    n_views = gam.shape[0]
    prs = pairs(n_views)
    recipe = _STRUCT[n_views][2]
    out = np.empty(len(recipe), np.complex128)
    for k, rc in enumerate(recipe):
        kind = rc[0]
        if kind == "two":
            out[k] = 2.0
            continue
        p = rc[1]
        i, j = prs[p]
        e = E[p]
        gi, gj = gam[i], gam[j]
        if kind == "cconst":
            out[k] = gj @ e @ gi
        elif kind == "ci":          # coefficient of u_i (a=0) or v_i (a=1)
            out[k] = -(gj @ e[:, rc[2]])
        elif kind == "cj":          # coefficient of u_j or v_j
            out[k] = -(e[rc[2], :] @ gi)
        elif kind == "cq":          # u_i/v_i (a) times u_j/v_j (b): E[b][a]
            a, b = rc[2], rc[3]
            out[k] = e[b, a]
        elif kind == "gconst":      # dc/d(u or v of view `side`) at zero corrections
            side, axis = rc[2], rc[3]
            out[k] = -(gj @ e[:, axis]) if side == "i" else -(e[axis, :] @ gi)
        elif kind == "glin":        # ... times u_o (b=0) or v_o (b=1) of the other view
            side, axis, b = rc[2], rc[3], rc[4]
            out[k] = e[b, axis] if side == "i" else e[axis, b]
        else:
            raise AssertionError(kind)
    return out


def _look_at_rotation(centre: np.ndarray, roll: float) -> np.ndarray:
    """World-to-camera rotation of a camera at `centre` looking at the origin."""
    z = -centre / np.linalg.norm(centre)
    a = np.array([0.0, 0.0, 1.0]) if abs(z[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    x = np.cross(a, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    c, s = np.cos(roll), np.sin(roll)
    x, y = c * x + s * y, -s * x + c * y
    return np.stack([x, y, z])


def _skew(t: np.ndarray) -> np.ndarray:
    return np.array([[0.0, -t[2], t[1]], [t[2], 0.0, -t[0]], [-t[1], t[0], 0.0]])


def _rotation(w: np.ndarray) -> np.ndarray:
    """exp([w]_x) by Rodrigues' formula."""
    th = np.linalg.norm(w)
    if th == 0.0:
        return np.eye(3)
    K = _skew(w / th)
    return np.eye(3) + np.sin(th) * K + (1.0 - np.cos(th)) * (K @ K)


def random_scene(rng: np.random.Generator, sigma: float = 0.5, sigma_rot_deg: float = 0.5,
                 sigma_t_rel: float = 0.01, n_views: int = N_VIEWS):
    """One scene of N views: (E [pairs,3,3], gamma [N,3], X [3], pixels [N,2],
    R [N,3,3], C [N,3]);
    R_k is camera k's world-to-camera rotation and C_k its centre.  E_ij is built
    from the pair's relative pose perturbed by the calibration noise."""
    while True:
        X = rng.uniform(-1.0, 1.0, 3)
        Rs, Cs, px = [], [], []
        ok = True
        for _ in range(n_views):
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            C = 6.0 * u
            R = _look_at_rotation(C, rng.uniform(0.0, 2.0 * np.pi))
            xc = R @ (X - C)
            if xc[2] <= 0:
                ok = False
            pix = np.array([FOCAL * xc[0] / xc[2] + CX, FOCAL * xc[1] / xc[2] + CY])
            pix = pix + sigma * rng.standard_normal(2)
            if not (0.0 <= pix[0] < WIDTH and 0.0 <= pix[1] < HEIGHT):
                ok = False
            Rs.append(R)
            Cs.append(C)
            px.append(pix)
        if not ok:
            continue
        E = np.empty((len(pairs(n_views)), 3, 3))
        for p, (i, j) in enumerate(pairs(n_views)):
            Rr = Rs[j] @ Rs[i].T
            t = Rs[j] @ (Cs[i] - Cs[j])
            if sigma_rot_deg > 0.0:
                Rr = _rotation(rng.normal(0.0, np.deg2rad(sigma_rot_deg), 3)) @ Rr
            if sigma_t_rel > 0.0:
                t = t + rng.normal(0.0, sigma_t_rel * np.linalg.norm(t), 3)
            e = _skew(t) @ Rr
            E[p] = e / np.linalg.norm(e)
        px = np.asarray(px)
        gam = np.column_stack([(px[:, 0] - CX) / FOCAL, (px[:, 1] - CY) / FOCAL, np.ones(n_views)])
        return E, gam, X, px, np.asarray(Rs), np.asarray(Cs)


def triangulation_instances(n_inst: int, seed: int, sigma: float = 0.5, sigma_rot_deg: float = 0.5,
                            sigma_t_rel: float = 0.01, n_views: int = N_VIEWS):
    """(structure, target coefficients [n_inst, terms] complex128, scenes).

    scenes is a dict of arrays: E [n_inst, pairs, 3, 3], gamma [n_inst, N, 3],
    X [n_inst, 3], pixels [n_inst, N, 2], R [n_inst, N, 3, 3], C [n_inst, N, 3]."""
    rng = np.random.default_rng(seed)
    coefs, Es, gs, Xs, ps, Rs, Cs = [], [], [], [], [], [], []
    for _ in range(n_inst):
        E, gam, X, px, R, C = random_scene(rng, sigma, sigma_rot_deg, sigma_t_rel, n_views)
        coefs.append(_coefficients(E, gam))
        Es.append(E)
        gs.append(gam)
        Xs.append(X)
        ps.append(px)
        Rs.append(R)
        Cs.append(C)
    scenes = dict(E=np.asarray(Es), gamma=np.asarray(gs), X=np.asarray(Xs), pixels=np.asarray(ps),
                  R=np.asarray(Rs), C=np.asarray(Cs))
    return triangulation_system(n_views), np.ascontiguousarray(np.asarray(coefs)), scenes


def start_instance_coefficients(seed: int = 4, n_views: int = N_VIEWS) -> np.ndarray:
    """Generic complex member of the triangulation support family, CN(0, 1) per term."""
    return complex_gaussian(np.random.default_rng(seed), (len(_STRUCT[n_views][2]),))


VISION_WORKLOADS: Dict[str, dict] = {
    # 4096 noisy 4-view triangulation instances (0.5 px pixel noise, calibration
    # noise per pair), parameter homotopy from the fixed generic start instance
    "triang4_batch4096": dict(n_inst=4096, seed=3, sigma=0.5, sigma_rot_deg=0.5, sigma_t_rel=0.01),
    # the same recipe with 3 views
    "triang3_batch4096": dict(n_inst=4096, seed=6, sigma=0.5, sigma_rot_deg=0.5, sigma_t_rel=0.01, n_views=3),
}


def start_instance(n_views: int = N_VIEWS):
    """(start coefficients [terms], start solutions [count, unknowns]) of the
    N-view triangulation family: a generic complex instance solved offline by
    monodromy (written by ``python -m oracle.monodromy triang4`` or ``triang3``;
    4 views: 296 solutions, 3 views: 94, the paper's counts)."""
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                        f"start_triang{n_views}.npz")
    z = np.load(path, allow_pickle=False)
    return np.ascontiguousarray(z["coef0"]), np.ascontiguousarray(z["solutions"])


def vision_workload(name: str, n_inst: int | None = None):
    """(structure, target coefficients, scenes) of a named vision workload;
    ``n_inst`` takes the first instances only."""
    spec = dict(VISION_WORKLOADS[name])
    total = spec.pop("n_inst")
    S, coef, scenes = triangulation_instances(total if n_inst is None else min(n_inst, total), **spec)
    return S, coef, scenes
