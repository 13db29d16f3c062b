"""Pins of the 5-point relative pose + depth workload (section 4: the rigid
motion of five correspondences, 16 x 16 with a unit quaternion) on the CPU:
the term table against the equations it stands for, the planted pose of
noise-free scenes, and the monodromy start set against the classical count of
the 5-point problem: 10 essential matrices (Demazure; Nister), each giving a
twisted pair of rotations and two quaternions per rotation under this build's
gauge rho_0 = 1 -- 40 solutions (Table 2 lists 160 for the paper's own,
unpublished, choice of unknowns)."""
import numpy as np
import pytest

import hc_inputs.fivept as F
import oracle
import oracle.monodromy as M


def geometric(x, p):
    """The 16 equations as written, at unknowns x and parameters p."""
    g, gb = F._points(p)
    q, T = x[:4], x[4:7]
    rho = np.concatenate([[1.0], x[7:11]])
    s = x[11:16]
    R = F.rotation(q)
    out = [s[i] * gb[i] - rho[i] * (R @ g[i]) - T for i in range(5)]
    return np.concatenate(out + [np.array([q @ q - 1.0])])


def test_structure():
    S = F.fivept_system()
    assert (S.n, S.n_terms) == (16, 155)
    assert np.bincount(S.term_eq).tolist() == [10] * 15 + [5]
    assert S.term_exp.sum(axis=1).max() == 3


def test_rotation_of_a_unit_quaternion():
    rng = np.random.default_rng(41)
    for _ in range(5):
        q = rng.standard_normal(4)
        q /= np.linalg.norm(q)
        R = F.rotation(q)
        assert np.max(np.abs(R @ R.T - np.eye(3))) < 1e-14 and abs(np.linalg.det(R) - 1.0) < 1e-14
        assert np.max(np.abs(F.rotation(F.rotation_to_quaternion(R)) - R)) < 1e-14


def test_terms_are_the_equations():
    S = F.fivept_system()
    rng = np.random.default_rng(42)
    for _ in range(3):
        p = F.random_parameters(rng)
        x = rng.standard_normal(16) + 1j * rng.standard_normal(16)
        Fv = oracle.eval_system(S, F.coefficients(p), x)
        Fv = Fv[0] if isinstance(Fv, tuple) else Fv
        g = geometric(x, p)
        assert np.max(np.abs(Fv - g)) <= 1e-12 * max(1.0, np.max(np.abs(g)))


def test_planted_pose_solves_noise_free_scenes():
    S, coef, sc = F.fivept_instances(4, seed=43, sigma=0.0)
    for i in range(4):
        gt = sc["gt"][i].astype(complex)
        assert oracle.residual(S, coef[i], gt) < 1e-14
        assert oracle.residual(S, coef[i], F.symmetry_orbit(gt)[0]) < 1e-14


def essential(x):
    """E = [T]_x R(q), scaled so that its largest entry is 1."""
    q, T = x[:4], x[4:7]
    Tx = np.array([[0, -T[2], T[1]], [T[2], 0, -T[0]], [-T[1], T[0], 0]])
    E = Tx @ F.rotation(q)
    return E / E.flat[np.argmax(np.abs(E))]


def test_start_set_is_ten_essential_matrices():
    S = F.fivept_system()
    p0, sols = F.start_instance()
    assert sols.shape == (40, 16)
    c0 = F.coefficients(p0)
    assert max(oracle.residual(S, c0, x) for x in sols) < 1e-12
    assert len(M.distinct_rows(sols)) == 40
    # closed under q -> -q
    for y in F.symmetry_orbit(sols)[0]:
        assert np.min(np.max(np.abs(sols - y), axis=1)) < 1e-8
    g, gb = F._points(p0)
    Es = np.array([essential(x) for x in sols])
    for E in Es:
        # the 5 epipolar constraints and Demazure's cubic constraint
        assert max(abs(gb[i] @ E @ g[i]) for i in range(5)) < 1e-10
        EEt = E @ E.T
        assert np.max(np.abs(2 * EEt @ E - np.trace(EEt) * E)) < 1e-9
    flat = Es.reshape(40, 9)
    classes = M.distinct_rows(flat, tol=1e-6)
    assert len(classes) == 10
    for C in classes:
        assert np.sum(np.max(np.abs(flat - C), axis=1) < 1e-6) == 4


def test_monodromy_reproduces_the_start_set():
    p0, sols = M.monodromy_family(F.Family, seed=4, stall=10, max_loops=200, log=lambda *_: None)
    p0s, sols_s = F.start_instance()
    assert np.array_equal(p0, p0s)
    assert len(sols) == len(sols_s)
    assert len(M.distinct_rows(np.concatenate([sols_s, sols]))) == len(sols_s)


def test_planted_pose_is_among_the_endpoints():
    """The oracle's parameter homotopy from the start instance to noise-free
    scenes ends on the planted pose."""
    S = F.fivept_system()
    p0, sols = F.start_instance()
    _, coef, sc = F.fivept_instances(3, seed=44, sigma=0.0)
    ep, st, _ = oracle.track(S, coef, start=sols, coef0=F.coefficients(p0), kind=oracle.LINEAR)
    for i in range(3):
        ok = ep[i][st[i] == oracle.SUCCESS]
        gt = sc["gt"][i]
        d = min(np.min(np.max(np.abs(ok - y), axis=1)) for y in (gt, F.symmetry_orbit(gt)[0]))
        assert d < 1e-8 * max(1.0, np.max(np.abs(gt)))
