"""Pins of the P3P workload (section 4, the depth form of three quadratics) on
the CPU: the term table against the geometric equations it stands for, the
planted depths of noise-free scenes, Table 2's solution count (8), the
rho -> -rho symmetry, and the oracle's solution sets against multi-start
Newton (brute force on this 3 x 3 system)."""
import numpy as np
import pytest

import hc_inputs.p3p as P
import oracle
import oracle.monodromy as M


def geometric(rho, gam, G):
    """The three equations as written: differences of scaled rays against
    world-point differences (plain transposes, so complex rho is allowed)."""
    a = rho[1] * gam[1] - rho[0] * gam[0]
    b = rho[2] * gam[2] - rho[0] * gam[0]
    d12, d13 = G[1] - G[0], G[2] - G[0]
    return np.array([a @ a - d12 @ d12, b @ b - d13 @ d13, a @ b - d12 @ d13])


def test_structure():
    S = P.p3p_system()
    assert (S.n, S.n_terms) == (3, 13)
    assert np.bincount(S.term_eq).tolist() == [4, 4, 5]
    assert set(S.term_exp.sum(axis=1).tolist()) == {0, 2}  # even monomials only
    assert oracle.degrees(S).tolist() == [2, 2, 2]


def test_terms_are_the_geometric_equations():
    S, coef, _, sc = P.p3p_instances(3, seed=31)
    rng = np.random.default_rng(3)
    for i in range(3):
        rho = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        F = oracle.eval_system(S, coef[i], rho)
        F = F[0] if isinstance(F, tuple) else F
        g = geometric(rho, sc["gamma"][i], sc["G"][i])
        assert np.max(np.abs(F - g)) <= 1e-12 * max(1.0, np.max(np.abs(g)))


def test_planted_depths_solve_noise_free_scenes():
    S, coef, _, sc = P.p3p_instances(4, seed=32, sigma=0.0)
    for i in range(4):
        assert oracle.residual(S, coef[i], sc["rho"][i].astype(complex)) < 1e-14


@pytest.fixture(scope="module")
def tracked():
    S, coef, gam, sc = P.p3p_instances(6, seed=33)
    ep, st, info = oracle.track(S, coef, gam)
    return S, coef, gam, sc, ep, st


def test_tables_count_and_symmetry(tracked):
    """Table 2: 8 solutions; each root's negation is a root."""
    S, coef, _, _, ep, st = tracked
    for i in range(len(coef)):
        ok = ep[i][st[i] == oracle.SUCCESS]
        assert len(ok) == 8
        assert len(M.distinct_rows(ok)) == 8
        assert max(oracle.residual(S, coef[i], x) for x in ok) < 1e-10
        for x in ok:
            d = np.max(np.abs(ok + x), axis=1) / max(1.0, np.max(np.abs(x)))
            assert d.min() < 1e-9


def newton_roots(S, c, rng, starts=3000):
    """Distinct roots reached by plain FP64 Newton (numpy solves, numerical
    Jacobian-free: the exact Jacobian of the 13-term table) from random complex
    starts."""
    exps = np.asarray(S.term_exp)
    eq = np.asarray(S.term_eq)

    def F_J(x):
        m = np.prod(x[None, :] ** exps, axis=1)
        F = np.zeros(3, complex)
        J = np.zeros((3, 3), complex)
        for k in range(len(c)):
            F[eq[k]] += c[k] * m[k]
            for j in range(3):
                if exps[k, j]:
                    e = exps[k].copy()
                    e[j] -= 1
                    J[eq[k], j] += c[k] * exps[k, j] * np.prod(x ** e)
        return F, J

    found = []
    for _ in range(starts):
        x = 8.0 * (rng.standard_normal(3) + 1j * rng.standard_normal(3))
        for _ in range(60):
            F, J = F_J(x)
            try:
                dx = np.linalg.solve(J, -F)
            except np.linalg.LinAlgError:
                break
            x = x + dx
            if np.max(np.abs(dx)) <= 1e-14 * max(1.0, np.max(np.abs(x))):
                break
        if np.all(np.isfinite(x)) and oracle.residual(S, c, x) < 1e-12:
            found.append(x)
    return M.distinct_rows(np.array(found), tol=1e-8) if found else np.zeros((0, 3))


def test_oracle_sets_equal_multistart_newton(tracked):
    """Brute force: Newton from 3000 random starts finds the same 8 roots."""
    S, coef, _, _, ep, st = tracked
    rng = np.random.default_rng(34)
    for i in range(2):
        ok = ep[i][st[i] == oracle.SUCCESS]
        roots = newton_roots(S, coef[i], rng)
        assert len(roots) == 8
        for x in ok:
            d = np.max(np.abs(roots - x), axis=1) / max(1.0, np.max(np.abs(x)))
            assert d.min() < 1e-9


def test_planted_depths_are_among_the_endpoints():
    S, coef, gam, sc = P.p3p_instances(4, seed=35, sigma=0.0)
    ep, st, _ = oracle.track(S, coef, gam)
    for i in range(4):
        ok = ep[i][st[i] == oracle.SUCCESS]
        d = np.max(np.abs(ok - sc["rho"][i]), axis=1) / np.max(sc["rho"][i])
        assert d.min() < 1e-9
