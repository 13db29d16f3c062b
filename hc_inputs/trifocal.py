"""Seeded synthetic instances of trifocal relative pose with a shared unknown
focal length (section 4).

Like the rest of ``hc_inputs`` this module only lays out problem structure and
draws random scenes; it holds none of the homotopy method's arithmetic.

Formulation (section 4, trifocal pose with unknown focal length; the printed
model has the depth and K^{-1} R in an order for which the true pose is no
solution, and its unknown count does not add up, so this is the reading the
build uses).  Three pinhole cameras share K = diag(f, f, 1); camera 1 is
[I | 0] and camera k in {2, 3} maps a point X of camera 1's frame to
R_k X + t_k.  A point seen at centred pixel coordinates (x_k, y_k) in view k
with depth rho_k satisfies

    rho_k K^{-1} (x_k, y_k, 1)^T = rho_1 R_k K^{-1} (x_1, y_1, 1)^T + t_k.

Scaled by f0 = 1000 (x~ = x / f0, f~ = f / f0, d_k = (x~_k, y~_k, f~)) this is
rho_k d_k = rho_1 R_k d_1 + f~ t_k.  The third row gives rho_k f~ = A_3 with
A = rho_1 R_k d_1 + f~ t_k, and the first two rows then give the two
equations

    x~_k A_3 - f~ A_1 = 0,      y~_k A_3 - f~ A_2 = 0

per point and view k in {2, 3}: 16 equations for 4 points.  Rotations are
quaternions q = (a, b, c, d) with the unnormalised rotation matrix
R(q) (a^2 + b^2 - c^2 - d^2 on the diagonal, ...) and one equation |q|^2 = 1
each.  The scale gauge fixes the first point's depth in view 1 to 1.  Unknowns
(18):

    x = (f~, q_12 (4), q_13 (4), t_12 (3), t_13 (3), rho^(2), rho^(3), rho^(4))

where rho^(p) is point p's depth in view 1.  Terms have degree up to 5
(f~^2 rho q q).  Every monomial is even in each quaternion, so q -> -q maps
solutions to solutions.  A negative focal length is a rotation of every image
by pi about its optical axis: with D = diag(-1, -1, 1), (f~, R_k, t_k, rho) ->
(-f~, D R_k D, D t_k, rho) negates the 16 projection equations and keeps the
norms, i.e. f~ -> -f~, q = (a, b, c, d) -> (a, -b, -c, d), t -> (-t_x, -t_y,
t_z).  Solutions come in orbits of eight.

Scene recipe: f ~ U[500, 1500] px, 640 x 480 images, principal point
(320, 240); cameras 2 and 3 have R = exp([w]_x) with w ~ N(0, 0.2^2 I) and
centres C ~ U[-1, 1]^3 (t = -R C); each of the 4 points has pixel position
uniform in view 1's image and depth ~ U[4, 8]; a point that is behind a camera
or projects outside an image is drawn again.  Pixel noise N(0, sigma^2) per
coordinate (sigma = 0.5 px) in all three views.
"""
from __future__ import annotations

import os
from typing import Dict

import numpy as np

from . import PolySystem

N_UNK = 18
N_PTS = 4
F0 = 1000.0
WIDTH, HEIGHT = 640.0, 480.0
CX, CY = 320.0, 240.0

# unknown indices
I_F = 0
I_Q = {2: 1, 3: 5}      # first index of q_12, q_13
I_T = {2: 9, 3: 12}     # first index of t_12, t_13
I_RHO = {1: 15, 2: 16, 3: 17}  # view-1 depth of points 2, 3, 4 (0-based point index 1..3)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
START_FILE = os.path.join(ROOT, "tests", "golden", "start_trifocal.npz")


# ---------------------------------------------------------------- polynomials as {exponent tuple: coefficient}

def _var(i: int) -> dict:
    e = [0] * N_UNK
    e[i] = 1
    return {tuple(e): 1.0}


def _const(c) -> dict:
    return {(0,) * N_UNK: c}


def _add(*ps) -> dict:
    out: dict = {}
    for p in ps:
        for e, c in p.items():
            out[e] = out.get(e, 0.0) + c
    return out


def _scale(p: dict, s) -> dict:
    return {e: s * c for e, c in p.items()}


def _mul(p: dict, q: dict) -> dict:
    out: dict = {}
    for e1, c1 in p.items():
        for e2, c2 in q.items():
            e = tuple(a + b for a, b in zip(e1, e2))
            out[e] = out.get(e, 0.0) + c1 * c2
    return out


def _rotation_entries(k: int):
    """R(q_1k) as a 3 x 3 array of quadratic polynomials in q_1k = (a, b, c, d)."""
    a, b, c, d = (_var(I_Q[k] + i) for i in range(4))
    sq = lambda u: _mul(u, u)  # noqa: E731
    two = lambda u, v: _scale(_mul(u, v), 2.0)  # noqa: E731
    neg = lambda u: _scale(u, -1.0)  # noqa: E731
    return [
        [_add(sq(a), sq(b), neg(sq(c)), neg(sq(d))), _add(two(b, c), neg(two(a, d))), _add(two(b, d), two(a, c))],
        [_add(two(b, c), two(a, d)), _add(sq(a), neg(sq(b)), sq(c), neg(sq(d))), _add(two(c, d), neg(two(a, b)))],
        [_add(two(b, d), neg(two(a, c))), _add(two(c, d), two(a, b)), _add(sq(a), neg(sq(b)), neg(sq(c)), sq(d))],
    ]


def _equations(pts: np.ndarray):
    """The 18 polynomials for scaled, centred image points pts [3 views, 4 points, 2]
    (x~, y~); numeric coefficients (any number type)."""
    f = _var(I_F)
    eqs = []
    for k in (2, 3):
        R = _rotation_entries(k)
        t = [_var(I_T[k] + i) for i in range(3)]
        for p in range(N_PTS):
            rho = _const(1.0) if p == 0 else _var(I_RHO[p])
            d1 = [_const(pts[0, p, 0]), _const(pts[0, p, 1]), f]
            A = [_add(_mul(rho, _add(*[_mul(R[i][j], d1[j]) for j in range(3)])), _mul(f, t[i])) for i in range(3)]
            xk, yk = pts[k - 1, p, 0], pts[k - 1, p, 1]
            eqs.append(_add(_scale(A[2], xk), _scale(_mul(f, A[0]), -1.0)))
            eqs.append(_add(_scale(A[2], yk), _scale(_mul(f, A[1]), -1.0)))
    for k in (2, 3):
        q = [_var(I_Q[k] + i) for i in range(4)]
        eqs.append(_add(*[_mul(u, u) for u in q], _const(-1.0)))
    return eqs


def _support():
    """Per equation, its monomials (exponent tuples) in a fixed order: degree
    descending, then lexicographic; taken from generic image points."""
    rng = np.random.default_rng(12345)
    eqs = _equations(rng.standard_normal((3, N_PTS, 2)))
    return [sorted((e for e, c in eq.items() if c != 0.0), key=lambda e: (-sum(e), tuple(-v for v in e)))
            for eq in eqs]


_SUPPORT = None


def trifocal_system() -> PolySystem:
    """Structure of the trifocal system (18 x 18, terms of degree <= 5)."""
    global _SUPPORT
    if _SUPPORT is None:
        _SUPPORT = _support()
    term_eq = np.concatenate([np.full(len(m), i, np.int32) for i, m in enumerate(_SUPPORT)])
    term_exp = np.array([e for m in _SUPPORT for e in m], np.int32)
    return PolySystem(n=N_UNK, term_eq=term_eq, term_exp=term_exp)


def coefficients(pts: np.ndarray) -> np.ndarray:
    """Coefficient vector (in trifocal_system's term order) for scaled, centred
    image points pts [3, 4, 2]."""
    S = trifocal_system()
    eqs = _equations(pts)
    out = np.zeros(S.n_terms, np.complex128)
    k = 0
    for i, mons in enumerate(_SUPPORT):
        extra = set(eqs[i]) - set(mons)
        assert all(eqs[i][e] == 0 for e in extra), "monomial outside the fixed support"
        for e in mons:
            out[k] = eqs[i].get(e, 0.0)
            k += 1
    return out


# ---------------------------------------------------------------- scenes

def _rotation(w: np.ndarray) -> np.ndarray:
    """exp([w]_x) by Rodrigues' formula."""
    th = np.linalg.norm(w)
    if th < 1e-15:
        return np.eye(3)
    k = w / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)


def rotation_to_quaternion(R: np.ndarray) -> np.ndarray:
    """Unit quaternion (a, b, c, d), a >= 0, of a rotation matrix (largest-pivot
    extraction)."""
    tr = np.trace(R)
    m = np.argmax([tr, R[0, 0], R[1, 1], R[2, 2]])
    if m == 0:
        a = 0.5 * np.sqrt(1 + tr)
        q = np.array([a, (R[2, 1] - R[1, 2]) / (4 * a), (R[0, 2] - R[2, 0]) / (4 * a), (R[1, 0] - R[0, 1]) / (4 * a)])
    elif m == 1:
        b = 0.5 * np.sqrt(1 + 2 * R[0, 0] - tr)
        q = np.array([(R[2, 1] - R[1, 2]) / (4 * b), b, (R[0, 1] + R[1, 0]) / (4 * b), (R[0, 2] + R[2, 0]) / (4 * b)])
    elif m == 2:
        c = 0.5 * np.sqrt(1 + 2 * R[1, 1] - tr)
        q = np.array([(R[0, 2] - R[2, 0]) / (4 * c), (R[0, 1] + R[1, 0]) / (4 * c), c, (R[1, 2] + R[2, 1]) / (4 * c)])
    else:
        d = 0.5 * np.sqrt(1 + 2 * R[2, 2] - tr)
        q = np.array([(R[1, 0] - R[0, 1]) / (4 * d), (R[0, 2] + R[2, 0]) / (4 * d), (R[1, 2] + R[2, 1]) / (4 * d), d])
    return q if q[0] >= 0 else -q


def _try_scene(rng: np.random.Generator):
    f = rng.uniform(500.0, 1500.0)
    R = {1: np.eye(3)}
    t = {1: np.zeros(3)}
    for k in (2, 3):
        R[k] = _rotation(rng.normal(0.0, 0.2, 3))
        C = rng.uniform(-1.0, 1.0, 3)
        t[k] = -R[k] @ C
    X = np.zeros((N_PTS, 3))
    pix = np.zeros((3, N_PTS, 2))
    for p in range(N_PTS):
        for _ in range(100):
            u = rng.uniform(0.0, WIDTH)
            v = rng.uniform(0.0, HEIGHT)
            z = rng.uniform(4.0, 8.0)
            Xp = z * np.array([(u - CX) / f, (v - CY) / f, 1.0])
            obs = []
            for k in (1, 2, 3):
                Xk = R[k] @ Xp + t[k]
                if Xk[2] <= 0.1:
                    break
                uk, vk = f * Xk[0] / Xk[2] + CX, f * Xk[1] / Xk[2] + CY
                if not (0.0 <= uk < WIDTH and 0.0 <= vk < HEIGHT):
                    break
                obs.append((uk, vk))
            if len(obs) == 3:
                X[p] = Xp
                pix[:, p, :] = obs
                break
        else:
            return None
    return f, R, t, X, pix


def random_scene(rng: np.random.Generator, sigma: float = 0.5) -> dict:
    """One scene: focal length, poses, points, pixel observations [3, 4, 2]
    (with noise), the scaled observations pts [3, 4, 2] and the ground-truth
    unknown vector gt [18] of the noise-free scene.  A point is drawn again
    (up to 100 times) until all three cameras see it; failing that, the whole
    scene is drawn again."""
    while True:
        scene = _try_scene(rng)
        if scene is not None:
            break
    f, R, t, X, pix = scene
    noisy = pix + rng.normal(0.0, sigma, pix.shape) if sigma > 0 else pix.copy()
    pts = np.stack([(noisy[..., 0] - CX) / F0, (noisy[..., 1] - CY) / F0], axis=-1)
    z1 = X[0, 2]
    gt = np.zeros(N_UNK)
    gt[I_F] = f / F0
    for k in (2, 3):
        gt[I_Q[k]:I_Q[k] + 4] = rotation_to_quaternion(R[k])
        gt[I_T[k]:I_T[k] + 3] = t[k] / z1
    for p in (1, 2, 3):
        gt[I_RHO[p]] = X[p, 2] / z1
    return dict(f=f, R=R, t=t, X=X, pix=pix, pts=pts, gt=gt)


def trifocal_instances(n_inst: int, seed: int, sigma: float = 0.5):
    """(structure, target coefficients [n_inst, n_terms] complex128, scenes:
    dict of arrays 'pts' [n_inst, 3, 4, 2], 'gt' [n_inst, 18], 'f' [n_inst])."""
    S = trifocal_system()
    rng = np.random.default_rng(seed)
    scenes = [random_scene(rng, sigma) for _ in range(n_inst)]
    coef = np.stack([coefficients(s["pts"]) for s in scenes])
    out = dict(pts=np.stack([s["pts"] for s in scenes]), gt=np.stack([s["gt"] for s in scenes]),
               f=np.array([s["f"] for s in scenes]))
    return S, np.ascontiguousarray(coef), out


def sign_orbit(x: np.ndarray) -> np.ndarray:
    """The four images of solution(s) x [..., 18] under q_12 -> -q_12 and
    q_13 -> -q_13, [4, ..., 18]."""
    out = []
    for s2 in (1.0, -1.0):
        for s3 in (1.0, -1.0):
            y = np.array(x, copy=True)
            y[..., I_Q[2]:I_Q[2] + 4] *= s2
            y[..., I_Q[3]:I_Q[3] + 4] *= s3
            out.append(y)
    return np.stack(out)


def focal_flip(x: np.ndarray) -> np.ndarray:
    """The image of solution(s) x [..., 18] under f~ -> -f~ (D = diag(-1, -1, 1)
    applied to the rotations by conjugation and to the translations)."""
    y = np.array(x, copy=True)
    y[..., I_F] *= -1
    for k in (2, 3):
        y[..., I_Q[k] + 1:I_Q[k] + 3] *= -1
        y[..., I_T[k]:I_T[k] + 2] *= -1
    return y


def symmetry_orbit(x: np.ndarray) -> np.ndarray:
    """The eight images of solution(s) x [..., 18] under the sign changes of
    the two quaternions and the focal flip, [8, ..., 18]."""
    s = sign_orbit(x)
    return np.concatenate([s, sign_orbit(focal_flip(x))])


TRIFOCAL_WORKLOADS: Dict[str, dict] = {
    # 1024 instances per launch, each tracked from the stored start instance
    "trifocal_batch1024": dict(n_inst=1024, seed=5, sigma=0.5),
}


def start_instance():
    """(start parameters [3, 4, 2] complex, start solutions [N, 18]) of the
    trifocal family, as written by `python -m oracle.monodromy trifocal`."""
    z = np.load(START_FILE)
    return z["params0"], z["solutions"]


def trifocal_workload(name: str, n_inst: int | None = None):
    w = dict(TRIFOCAL_WORKLOADS[name])
    if n_inst is not None:
        w["n_inst"] = n_inst
    return trifocal_instances(w["n_inst"], w["seed"], w["sigma"])


# ---------------------------------------------------------------- the structured parameter family
# Parameters p are the 24 scaled image coordinates pts [3, 4, 2]; the system's
# coefficients c(p) are products of them.  Along a segment where only view 1's
# coordinates move, or only views 2 and 3 move, every coefficient is an affine
# function of the moving coordinates, so on such a segment the linear
# coefficient homotopy between its end instances stays inside the family.

def waypoints(p_from: np.ndarray, p_to: np.ndarray):
    """Parameter points of the path p_from -> p_to: first view 1's coordinates
    move, then those of views 2 and 3."""
    mid = np.array(p_from, dtype=np.complex128, copy=True)
    mid[0] = p_to[0]
    return [np.asarray(p_from, np.complex128), mid, np.asarray(p_to, np.complex128)]


def random_parameters(rng: np.random.Generator) -> np.ndarray:
    """A generic complex parameter point: CN(0, 1) per coordinate, scaled like
    the real ones (|x~| ~ 0.3)."""
    return 0.3 * (rng.standard_normal((3, N_PTS, 2)) + 1j * rng.standard_normal((3, N_PTS, 2))) / np.sqrt(2.0)


def fabricate_pair(rng: np.random.Generator):
    """(p0, x0): random complex unknowns (quaternions scaled to q.q = 1) and
    view-1 coordinates; views 2 and 3 by projecting A = rho R d_1 + f~ t, so
    x0 solves the system of c(p0) exactly up to rounding."""
    cn = lambda *s: (rng.standard_normal(s) + 1j * rng.standard_normal(s)) / np.sqrt(2.0)  # noqa: E731
    x0 = cn(N_UNK)
    for k in (2, 3):
        q = x0[I_Q[k]:I_Q[k] + 4]
        x0[I_Q[k]:I_Q[k] + 4] = q / np.sqrt(q @ q)
    p0 = np.zeros((3, N_PTS, 2), np.complex128)
    p0[0] = 0.3 * cn(N_PTS, 2)
    f = x0[I_F]
    for k in (2, 3):
        a, b, c, d = x0[I_Q[k]:I_Q[k] + 4]
        R = np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                      [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                      [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])
        t = x0[I_T[k]:I_T[k] + 3]
        for p in range(N_PTS):
            rho = 1.0 if p == 0 else x0[I_RHO[p]]
            A = rho * (R @ np.array([p0[0, p, 0], p0[0, p, 1], f])) + f * t
            p0[k - 1, p] = [f * A[0] / A[2], f * A[1] / A[2]]
    return p0, x0


class Family:
    """The trifocal family as the monodromy driver needs it."""
    system = staticmethod(trifocal_system)
    coef = staticmethod(coefficients)
    waypoints = staticmethod(waypoints)
    random = staticmethod(random_parameters)
    fabricate = staticmethod(fabricate_pair)
    orbit = staticmethod(symmetry_orbit)
