"""Seeded synthetic instances of the P3P problem in the depth formulation of
section 4 (three quadratics in the depths rho_1, rho_2, rho_3).

Like the rest of ``hc_inputs`` this module only lays out problem structure and
draws random scenes; it holds none of the homotopy method's arithmetic.

Formulation.  Image points gamma_i = ((p_x - 320)/f, (p_y - 240)/f, 1) and the
3D points Gamma_i = rho_i gamma_i in the camera frame.  Rotation and
translation drop out of the pairwise distances and dot products:

    |rho_2 g_2 - rho_1 g_1|^2 = |G_2 - G_1|^2
    |rho_3 g_3 - rho_1 g_1|^2 = |G_3 - G_1|^2
    (rho_2 g_2 - rho_1 g_1) . (rho_3 g_3 - rho_1 g_1) = (G_2 - G_1) . (G_3 - G_1)

with G_i the world points (distances are the same in any frame).  Terms per
equation: rho_1^2, rho_1 rho_2, rho_2^2, 1 | rho_1^2, rho_1 rho_3, rho_3^2, 1 |
rho_1^2, rho_1 rho_2, rho_1 rho_3, rho_2 rho_3, 1; 13 terms, every monomial of
even degree, so rho -> -rho maps solutions to solutions.  Total degree 8, the
solution count of Table 2.

Scene recipe: f = 1000 px, 640 x 480 images, principal point (320, 240); three
points with pixel positions uniform in the image and depths ~ U[4, 8] (the
camera frame), the world points being the same points after a random rigid
motion (rotation by a uniform random quaternion, translation ~ U[-1, 1]^3);
pixel noise N(0, sigma^2) per coordinate on the observed image points.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import PolySystem, unit_gammas

FOCAL = 1000.0
WIDTH, HEIGHT = 640.0, 480.0
CX, CY = 320.0, 240.0

# (equation, exponents of rho_1, rho_2, rho_3) of the 13 terms
_TERMS = [(0, (2, 0, 0)), (0, (1, 1, 0)), (0, (0, 2, 0)), (0, (0, 0, 0)),
          (1, (2, 0, 0)), (1, (1, 0, 1)), (1, (0, 0, 2)), (1, (0, 0, 0)),
          (2, (2, 0, 0)), (2, (1, 1, 0)), (2, (1, 0, 1)), (2, (0, 1, 1)), (2, (0, 0, 0))]


def p3p_system() -> PolySystem:
    """Structure of the P3P depth system (3 x 3, 13 terms, degree 2)."""
    return PolySystem(n=3, term_eq=np.array([e for e, _ in _TERMS], np.int32),
                      term_exp=np.array([x for _, x in _TERMS], np.int32))


def coefficients(gam: np.ndarray, G: np.ndarray) -> np.ndarray:
    """Coefficients of the 13 terms for image points gam [3, 3] (rows gamma_i)
    and world points G [3, 3]."""
    g11, g22, g33 = gam[0] @ gam[0], gam[1] @ gam[1], gam[2] @ gam[2]
    g12, g13, g23 = gam[0] @ gam[1], gam[0] @ gam[2], gam[1] @ gam[2]
    d12, d13 = G[1] - G[0], G[2] - G[0]
    return np.array([g11, -2.0 * g12, g22, -(d12 @ d12),
                     g11, -2.0 * g13, g33, -(d13 @ d13),
                     g11, -g12, -g13, g23, -(d12 @ d13)], np.complex128)


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.standard_normal(4)
    a, b, c, d = q / np.linalg.norm(q)
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def random_scene(rng: np.random.Generator, sigma: float = 0.5):
    """(gamma [3, 3] observed, world points G [3, 3], true depths [3], pixels [3, 2])."""
    px = np.column_stack([rng.uniform(0.0, WIDTH, 3), rng.uniform(0.0, HEIGHT, 3)])
    rho = rng.uniform(4.0, 8.0, 3)
    ray = np.column_stack([(px[:, 0] - CX) / FOCAL, (px[:, 1] - CY) / FOCAL, np.ones(3)])
    P = rho[:, None] * ray                      # camera-frame points
    R, T = _random_rotation(rng), rng.uniform(-1.0, 1.0, 3)
    G = P @ R.T + T                             # world points
    obs = px + sigma * rng.standard_normal((3, 2))
    gam = np.column_stack([(obs[:, 0] - CX) / FOCAL, (obs[:, 1] - CY) / FOCAL, np.ones(3)])
    return gam, G, rho, obs


def p3p_instances(n_inst: int, seed: int, sigma: float = 0.5):
    """(structure, coefficients [n_inst, 13], gammas [n_inst] of the total-degree
    homotopy, scenes dict: gamma [n_inst, 3, 3], G [n_inst, 3, 3], rho [n_inst, 3])."""
    rng = np.random.default_rng(seed)
    coefs, gs, Gs, rhos = [], [], [], []
    for _ in range(n_inst):
        gam, G, rho, _ = random_scene(rng, sigma)
        coefs.append(coefficients(gam, G))
        gs.append(gam)
        Gs.append(G)
        rhos.append(rho)
    homotopy_gamma = unit_gammas(rng, n_inst)
    scenes = dict(gamma=np.asarray(gs), G=np.asarray(Gs), rho=np.asarray(rhos))
    return p3p_system(), np.ascontiguousarray(np.asarray(coefs)), homotopy_gamma, scenes


P3P_WORKLOADS: Dict[str, dict] = {
    # 65536 noisy P3P instances, 8 total-degree paths each
    "p3p_batch65536": dict(n_inst=65536, seed=7, sigma=0.5),
}


def p3p_workload(name: str, n_inst: int | None = None):
    spec = dict(P3P_WORKLOADS[name])
    total = spec.pop("n_inst")
    return p3p_instances(total if n_inst is None else min(n_inst, total), **spec)
