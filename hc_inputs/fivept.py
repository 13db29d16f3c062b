"""Seeded synthetic instances of 5-point relative pose with depth
reconstruction (section 4: the rigid-motion equations of five correspondences,
solved for rotation, translation and all depths at once).

Like the rest of ``hc_inputs`` this module only lays out problem structure and
draws random scenes; it holds none of the homotopy method's arithmetic.

Formulation (this build's reading; the paper gives the equations and the size
16 x 16 but not its gauge).  Calibrated image points gamma_i, gbar_i =
((p_x - 320)/f, (p_y - 240)/f, 1) in views 1 and 2, i < 5:

    s_i gbar_i = rho_i R(q) gamma_i + T,      i = 0..4     (15 equations)
    q . q = 1                                               (1 equation)

with R(q) the rotation of the quaternion q = (a, b, c, d) written out as a
quadratic form (a rotation whenever q . q = 1), and the scale fixed by rho_0 = 1.
Unknowns x = (q (4), T (3), rho_1..rho_4, s_0..s_4): 16.  Each rigid-motion
equation has 10 terms (s_i; rho_i times the 8 quadratic monomials of q that
its row of R uses; T_k), the norm equation 5: 155 terms of degree <= 3.
q -> -q maps solutions to solutions.  The coefficients are affine in the 20
image coordinates, so a straight line between two parameter points is a linear
coefficient homotopy that stays in the family.

Scene recipe: f = 1000 px, 640 x 480, principal point (320, 240); camera 1 =
[I | 0], camera 2 = [R | T] with R = exp([w]_x), w ~ N(0, 0.2^2 I), T ~
U[-1, 1]^3; five points with pixel positions uniform in view 1 and depths ~
U[4, 8], each redrawn (up to 100 times, then the whole scene) until camera 2
sees it inside its image; pixel noise N(0, sigma^2) in both views.  The
noise-free scene's unknown vector (depths and T divided by the first depth) is
the planted ground truth.
"""
from __future__ import annotations

import os
from typing import Dict, List, Tuple

import numpy as np

from . import PolySystem, complex_gaussian

FOCAL = 1000.0
WIDTH, HEIGHT = 640.0, 480.0
CX, CY = 320.0, 240.0
N_PTS = 5
N_UNK = 16
N_PARAMS = 4 * N_PTS  # (x, y) of gamma_i and of gbar_i

# R(q) as quadratic forms in q = (a, b, c, d) = indices (0, 1, 2, 3):
# entry (k, j) -> {(u, v): coefficient of q_u q_v}
_R = {
    (0, 0): {(0, 0): 1, (1, 1): 1, (2, 2): -1, (3, 3): -1},
    (0, 1): {(1, 2): 2, (0, 3): -2},
    (0, 2): {(1, 3): 2, (0, 2): 2},
    (1, 0): {(1, 2): 2, (0, 3): 2},
    (1, 1): {(0, 0): 1, (1, 1): -1, (2, 2): 1, (3, 3): -1},
    (1, 2): {(2, 3): 2, (0, 1): -2},
    (2, 0): {(1, 3): 2, (0, 2): -2},
    (2, 1): {(2, 3): 2, (0, 1): 2},
    (2, 2): {(0, 0): 1, (1, 1): -1, (2, 2): -1, (3, 3): 1},
}


def rotation(q: np.ndarray) -> np.ndarray:
    """R(q) from the quadratic forms (a rotation when q . q = 1)."""
    R = np.zeros((3, 3), dtype=np.result_type(q, np.float64))
    for (k, j), form in _R.items():
        R[k, j] = sum(c * q[u] * q[v] for (u, v), c in form.items())
    return R


def _iq(k):
    return k            # q_k


def _iT(k):
    return 4 + k        # T_k


def _irho(i):
    return 7 + i - 1    # rho_i, i = 1..4


def _is(i):
    return 11 + i       # s_i, i = 0..4


def _row_monomials(k: int) -> List[Tuple[int, int]]:
    out = []
    for j in range(3):
        for uv in _R[(k, j)]:
            if uv not in out:
                out.append(uv)
    return sorted(out)


def _structure():
    """(term_eq, term_exp, recipe); recipe[t] says how term t's coefficient is
    formed from the parameters -- see ``coefficients``."""
    eq, ex, recipe = [], [], []

    def term(e, idx, rc):
        v = np.zeros(N_UNK, np.int32)
        for i in idx:
            v[i] += 1
        eq.append(e)
        ex.append(v)
        recipe.append(rc)

    for i in range(N_PTS):
        for k in range(3):
            e = 3 * i + k
            term(e, (_is(i),), ("gbar", i, k))
            for (u, v) in _row_monomials(k):
                idx = (_iq(u), _iq(v)) if i == 0 else (_irho(i), _iq(u), _iq(v))
                term(e, idx, ("rot", i, k, u, v))
            term(e, (_iT(k),), ("const", -1.0))
    for u in range(4):
        term(15, (_iq(u), _iq(u)), ("const", 1.0))
    term(15, (), ("const", -1.0))
    return np.asarray(eq, np.int32), np.stack(ex).astype(np.int32), recipe


_EQ, _EXP, _RECIPE = _structure()


def fivept_system() -> PolySystem:
    """Structure of the 5-point pose + depth system (16 x 16, 155 terms, degree 3)."""
    return PolySystem(n=N_UNK, term_eq=_EQ.copy(), term_exp=_EXP.copy())


def _points(p: np.ndarray):
    """gamma [5, 3], gbar [5, 3] of a parameter vector (x, y of gamma_i, then of gbar_i)."""
    p = np.asarray(p)
    g = np.concatenate([p[:2 * N_PTS].reshape(N_PTS, 2), np.ones((N_PTS, 1))], axis=1)
    gb = np.concatenate([p[2 * N_PTS:].reshape(N_PTS, 2), np.ones((N_PTS, 1))], axis=1)
    return g, gb


def coefficients(p: np.ndarray) -> np.ndarray:
    """Coefficients of the 155 terms at parameters p [20] (complex allowed)."""
    g, gb = _points(p)
    out = np.empty(len(_RECIPE), np.complex128)
    for t, rc in enumerate(_RECIPE):
        if rc[0] == "const":
            out[t] = rc[1]
        elif rc[0] == "gbar":
            out[t] = gb[rc[1], rc[2]]
        else:  # -(R(q) gamma_i)_k's coefficient of q_u q_v
            _, i, k, u, v = rc
            out[t] = -sum(_R[(k, j)].get((u, v), 0) * g[i, j] for j in range(3))
    return out


def _skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def _rodrigues(w):
    th = np.linalg.norm(w)
    if th == 0.0:
        return np.eye(3)
    K = _skew(w / th)
    return np.eye(3) + np.sin(th) * K + (1.0 - np.cos(th)) * (K @ K)


def rotation_to_quaternion(R: np.ndarray) -> np.ndarray:
    """A unit quaternion q with rotation(q) = R (one of +-q)."""
    a = np.sqrt(max(0.0, 1.0 + R[0, 0] + R[1, 1] + R[2, 2])) / 2.0
    if a > 1e-6:
        return np.array([a, (R[2, 1] - R[1, 2]) / (4 * a), (R[0, 2] - R[2, 0]) / (4 * a), (R[1, 0] - R[0, 1]) / (4 * a)])
    # rotation by ~pi: from the largest diagonal entry
    k = int(np.argmax(np.diag(R)))
    q = np.zeros(4)
    i, j, m = k, (k + 1) % 3, (k + 2) % 3
    q[1 + i] = np.sqrt(max(0.0, 1.0 + R[i, i] - R[j, j] - R[m, m])) / 2.0
    q[0] = (R[m, j] - R[j, m]) / (4 * q[1 + i])
    q[1 + j] = (R[j, i] + R[i, j]) / (4 * q[1 + i])
    q[1 + m] = (R[m, i] + R[i, m]) / (4 * q[1 + i])
    return q


def random_scene(rng: np.random.Generator, sigma: float = 0.5):
    """(params [20] observed, ground truth x [16] of the noise-free scene,
    R [3, 3], T [3], depths [5] in view 1)."""
    while True:
        R = _rodrigues(rng.normal(0.0, 0.2, 3))
        T = rng.uniform(-1.0, 1.0, 3)
        px1, px2, rho = [], [], []
        ok = True
        for _ in range(N_PTS):
            for _try in range(100):
                pix = np.array([rng.uniform(0.0, WIDTH), rng.uniform(0.0, HEIGHT)])
                d = rng.uniform(4.0, 8.0)
                X = d * np.array([(pix[0] - CX) / FOCAL, (pix[1] - CY) / FOCAL, 1.0])
                Y = R @ X + T
                if Y[2] <= 0:
                    continue
                pix2 = np.array([FOCAL * Y[0] / Y[2] + CX, FOCAL * Y[1] / Y[2] + CY])
                if 0.0 <= pix2[0] < WIDTH and 0.0 <= pix2[1] < HEIGHT:
                    break
            else:
                ok = False
                break
            px1.append(pix)
            px2.append(pix2)
            rho.append(d)
        if not ok:
            continue
        px1, px2, rho = np.asarray(px1), np.asarray(px2), np.asarray(rho)
        # ground truth with rho_0 = 1: depths, s and T scaled by 1 / rho_0
        X = rho[:, None] * np.column_stack([(px1[:, 0] - CX) / FOCAL, (px1[:, 1] - CY) / FOCAL, np.ones(N_PTS)])
        Y = X @ R.T + T
        sc = 1.0 / rho[0]
        gt = np.concatenate([rotation_to_quaternion(R), T * sc, rho[1:] * sc, Y[:, 2] * sc])
        o1 = px1 + sigma * rng.standard_normal(px1.shape)
        o2 = px2 + sigma * rng.standard_normal(px2.shape)
        params = np.concatenate([((o1 - [CX, CY]) / FOCAL).ravel(), ((o2 - [CX, CY]) / FOCAL).ravel()])
        return params, gt, R, T, rho


def fivept_instances(n_inst: int, seed: int, sigma: float = 0.5):
    """(structure, coefficients [n_inst, 155], scenes dict: params [n_inst, 20],
    gt [n_inst, 16])."""
    rng = np.random.default_rng(seed)
    ps, gts = [], []
    for _ in range(n_inst):
        p, gt, _, _, _ = random_scene(rng, sigma)
        ps.append(p)
        gts.append(gt)
    ps = np.asarray(ps)
    coef = np.stack([coefficients(p) for p in ps])
    return fivept_system(), np.ascontiguousarray(coef), dict(params=ps, gt=np.asarray(gts))


# ---------------------------------------------------------------- the family (monodromy)

def waypoints(p_from, p_to):
    """Coefficients are affine in the parameters: one straight leg."""
    return [np.asarray(p_from, np.complex128), np.asarray(p_to, np.complex128)]


def random_parameters(rng: np.random.Generator) -> np.ndarray:
    return complex_gaussian(rng, (N_PARAMS,))


def fabricate_pair(rng: np.random.Generator):
    """(p0, x0) with x0 an exact solution at the complex parameters p0: a random
    complex unit quaternion (q . q = 1), translation, depths and view-1 points;
    the view-2 points follow from the rigid motion."""
    q = complex_gaussian(rng, (4,))
    q = q / np.sqrt(q @ q)
    T = complex_gaussian(rng, (3,))
    rho = np.concatenate([[1.0], complex_gaussian(rng, (N_PTS - 1,))])
    g = np.concatenate([complex_gaussian(rng, (N_PTS, 2)), np.ones((N_PTS, 1))], axis=1)
    W = rho[:, None] * (g @ rotation(q).T) + T
    s = W[:, 2]
    gb = W / s[:, None]
    p0 = np.concatenate([g[:, :2].ravel(), gb[:, :2].ravel()])
    x0 = np.concatenate([q, T, rho[1:], s])
    return p0, x0


def symmetry_orbit(x: np.ndarray) -> np.ndarray:
    """Images [1, N, 16] of solutions under q -> -q."""
    y = np.array(x, copy=True)
    y[..., :4] = -y[..., :4]
    return y[None]


class Family:
    """The 5-point family as the monodromy driver needs it."""
    system = staticmethod(fivept_system)
    coef = staticmethod(coefficients)
    waypoints = staticmethod(waypoints)
    random = staticmethod(random_parameters)
    fabricate = staticmethod(fabricate_pair)
    orbit = staticmethod(symmetry_orbit)


START_FILE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden",
                          "start_fivept.npz")


def start_instance():
    """(params0 [20], solutions [N, 16]) of the family's generic complex start
    instance (written by ``python -m oracle.monodromy fivept``)."""
    z = np.load(START_FILE, allow_pickle=False)
    return np.ascontiguousarray(z["params0"]), np.ascontiguousarray(z["solutions"])


FIVEPT_WORKLOADS: Dict[str, dict] = {
    "fivept_batch1024": dict(n_inst=1024, seed=8, sigma=0.5),
}


def fivept_workload(name: str, n_inst: int | None = None):
    spec = dict(FIVEPT_WORKLOADS[name])
    total = spec.pop("n_inst")
    return fivept_instances(total if n_inst is None else min(n_inst, total), **spec)
