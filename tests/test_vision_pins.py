"""Pins of the 4-view triangulation workload (section 4) and of its start
instance, on the CPU: the system against the Lagrangian it comes from, the
degenerate consistent-pose case, the monodromy start set against the paper's
root count (Table 2), and the oracle's endpoints against an independent
constrained optimiser."""
import numpy as np
import pytest

import hc_inputs.vision as V
import oracle
import oracle.monodromy as M


def lagrangian(x, E, gam):
    u, v, lam = x[0:8:2], x[1:8:2], x[8:]
    s = np.sum(u * u + v * v)
    for p, (i, j) in enumerate(V.PAIRS):
        gi = gam[i] - np.array([u[i], v[i], 0.0])
        gj = gam[j] - np.array([u[j], v[j], 0.0])
        s = s + lam[p] * (gj @ E[p] @ gi)
    return s


def test_structure():
    S = V.triangulation_system()
    assert (S.n, S.n_terms) == (14, 134)
    assert np.bincount(S.term_eq).tolist() == [10] * 8 + [9] * 6
    assert S.term_exp.sum(axis=1).max() == 2


def test_equations_are_the_lagrangian_gradient():
    """F = grad L at a random complex point, by central differences (L is a
    polynomial, so the difference quotient is exact up to rounding)."""
    S, coef, sc = V.triangulation_instances(2, seed=11, sigma=0.5)
    rng = np.random.default_rng(1)
    for i in range(2):
        x = rng.standard_normal(14) + 1j * rng.standard_normal(14)
        F = oracle.eval_system(S, coef[i], x)
        F = F[0] if isinstance(F, tuple) else F
        h = 1e-6
        g = np.array([(lagrangian(x + h * e, sc["E"][i], sc["gamma"][i]) -
                       lagrangian(x - h * e, sc["E"][i], sc["gamma"][i])) / (2 * h) for e in np.eye(14)])
        assert np.max(np.abs(F - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_consistent_poses_make_the_multipliers_non_unique():
    """Reading behind the calibration noise: with the E_ij of one consistent set of
    poses and exact image points, x = 0 solves the system but the 8 x 6 matrix of
    constraint gradients has rank 5, so a whole line of multipliers goes with it;
    independently perturbed pairs restore rank 6."""
    S, coef, sc = V.triangulation_instances(3, seed=12, sigma=0.0, sigma_rot_deg=0.0, sigma_t_rel=0.0)
    for i in range(3):
        F = oracle.eval_system(S, coef[i], np.zeros(14, complex))
        F = F[0] if isinstance(F, tuple) else F
        assert np.max(np.abs(F)) < 1e-14
        for p, (a, b) in enumerate(V.PAIRS):
            assert abs(sc["gamma"][i][b] @ sc["E"][i][p] @ sc["gamma"][i][a]) < 1e-14
        # rows = dc_p/d(u_1, v_1, ..., u_4, v_4) at zero corrections: the
        # coefficients of the constraints' linear terms
        G = np.zeros((6, 8))
        for p, (a, b) in enumerate(V.PAIRS):
            e, ga, gb = sc["E"][i][p], sc["gamma"][i][a], sc["gamma"][i][b]
            G[p, 2 * a:2 * a + 2] = [-(gb @ e[:, 0]), -(gb @ e[:, 1])]
            G[p, 2 * b:2 * b + 2] = [-(e[0, :] @ ga), -(e[1, :] @ ga)]
        sv = np.linalg.svd(G, compute_uv=False)
        assert sv[4] > 1e-6 * sv[0] and sv[5] < 1e-12 * sv[0]
    _, coef, sc = V.triangulation_instances(3, seed=12, sigma=0.0)
    for i in range(3):
        G = np.zeros((6, 8))
        for p, (a, b) in enumerate(V.PAIRS):
            e, ga, gb = sc["E"][i][p], sc["gamma"][i][a], sc["gamma"][i][b]
            G[p, 2 * a:2 * a + 2] = [-(gb @ e[:, 0]), -(gb @ e[:, 1])]
            G[p, 2 * b:2 * b + 2] = [-(e[0, :] @ ga), -(e[1, :] @ ga)]
        sv = np.linalg.svd(G, compute_uv=False)
        assert sv[5] > 1e-6 * sv[0]


def test_start_set_has_the_papers_count():
    """Table 2 lists 296 solutions for 4-view triangulation; the stored monodromy
    set of the generic start instance has exactly that many, all regular roots
    (tiny backward error) and pairwise distinct."""
    S = V.triangulation_system()
    c0, sols = V.start_instance()
    assert sols.shape == (296, 14)
    assert max(oracle.residual(S, c0, x) for x in sols) < 1e-12
    assert len(M.distinct_rows(sols)) == 296


def test_monodromy_reproduces_the_start_set():
    """The stored set is what `python -m oracle.monodromy triang4` computes."""
    S = V.triangulation_system()
    c0, sols = M.monodromy(S, seed=4, log=lambda *_: None)
    c0s, sols_s = V.start_instance()
    assert np.array_equal(c0, c0s)
    assert len(sols) == len(sols_s)
    both = M.distinct_rows(np.concatenate([sols_s, sols]))
    assert len(both) == len(sols_s)


def test_fabricated_pair_is_exact():
    S = V.triangulation_system()
    c0, x0 = M.fabricate_pair(S, np.random.default_rng(7))
    assert oracle.residual(S, c0, x0) < 1e-14


@pytest.fixture(scope="module")
def tracked():
    """The oracle's parameter homotopy from the start instance to 3 scenes."""
    S = V.triangulation_system()
    c0, sols = V.start_instance()
    _, coef, sc = V.triangulation_instances(3, seed=14)
    ep, st, info = oracle.track(S, coef, start=sols, coef0=c0, kind=oracle.LINEAR)
    return S, coef, ep, st, sc


def real_finite(ep, st):
    ok = ep[st == oracle.SUCCESS]
    return ok[np.max(np.abs(ok.imag), axis=1) < 1e-8 * np.maximum(1.0, np.max(np.abs(ok), axis=1))].real


def test_endpoints_are_distinct_critical_points(tracked):
    S, coef, ep, st, _ = tracked
    for i in range(3):
        ok = ep[i][st[i] == oracle.SUCCESS]
        assert 250 <= len(ok) <= 296
        assert len(M.distinct_rows(ok)) == len(ok)
        assert max(oracle.residual(S, coef[i], x) for x in ok) < 1e-10


def constrained_local_optimum(E, gam):
    """A local minimiser of sum u_k^2 + v_k^2 subject to the six epipolar
    constraints, by SLSQP from zero corrections: an independent optimiser on the
    original problem.  Returns the corrections (u_1, v_1, ..., u_4, v_4)."""
    from scipy.optimize import minimize

    def cons(z):
        out = []
        for p, (a, b) in enumerate(V.PAIRS):
            ga = gam[a] - np.array([z[2 * a], z[2 * a + 1], 0.0])
            gb = gam[b] - np.array([z[2 * b], z[2 * b + 1], 0.0])
            out.append(gb @ E[p] @ ga)
        return np.array(out)

    r = minimize(lambda z: z @ z, np.zeros(8), jac=lambda z: 2 * z, method="SLSQP",
                 constraints=[{"type": "eq", "fun": cons}], options={"ftol": 1e-16, "maxiter": 1000})
    assert np.max(np.abs(cons(r.x))) < 1e-12
    return r.x


def test_local_optimum_is_among_the_real_critical_points(tracked):
    """Homotopy continuation finds every critical point, so the local minimum an
    optimiser reaches is one of the real finite endpoints, and the least cost
    among them is no larger (the near-dependent constraints give this problem
    several real local minima)."""
    S, coef, ep, st, sc = tracked
    for i in range(3):
        real = real_finite(ep[i], st[i])
        assert len(real) > 0
        z = constrained_local_optimum(sc["E"][i], sc["gamma"][i])
        d = np.min(np.max(np.abs(real[:, :8] - z), axis=1))
        assert d <= 1e-6 * max(1.0, np.max(np.abs(z))), d
        assert np.min(np.sum(real[:, :8] ** 2, axis=1)) <= z @ z * (1 + 1e-9)
