"""Pins of the 3-view triangulation workload (section 4, N = 3: 9 unknowns) and
of its start instance, on the CPU: the system against the Lagrangian it comes
from, the noise-free scene's exact solution, the monodromy start set against
the paper's root count (Table 2 lists 94 solutions for 3 views), and the
oracle's endpoints against an independent constrained optimiser."""
import numpy as np
import pytest

import hc_inputs.vision as V
import oracle
import oracle.monodromy as M

NV = 3
PAIRS = V.pairs(NV)


def lagrangian(x, E, gam):
    u, v, lam = x[0:2 * NV:2], x[1:2 * NV:2], x[2 * NV:]
    s = np.sum(u * u + v * v)
    for p, (i, j) in enumerate(PAIRS):
        gi = gam[i] - np.array([u[i], v[i], 0.0])
        gj = gam[j] - np.array([u[j], v[j], 0.0])
        s = s + lam[p] * (gj @ E[p] @ gi)
    return s


def test_structure():
    S = V.triangulation_system(NV)
    assert (S.n, S.n_terms) == (9, 69)
    assert np.bincount(S.term_eq).tolist() == [7] * 6 + [9] * 3
    assert S.term_exp.sum(axis=1).max() == 2


def test_equations_are_the_lagrangian_gradient():
    """F = grad L at random complex points, by central differences."""
    S, coef, sc = V.triangulation_instances(2, seed=21, n_views=NV)
    rng = np.random.default_rng(2)
    for i in range(2):
        x = rng.standard_normal(9) + 1j * rng.standard_normal(9)
        F = oracle.eval_system(S, coef[i], x)
        F = F[0] if isinstance(F, tuple) else F
        h = 1e-6
        g = np.array([(lagrangian(x + h * e, sc["E"][i], sc["gamma"][i]) -
                       lagrangian(x - h * e, sc["E"][i], sc["gamma"][i])) / (2 * h) for e in np.eye(9)])
        assert np.max(np.abs(F - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def test_noise_free_scene_is_solved_by_zero_corrections():
    """Exact image points and the E_ij of one consistent set of poses: zero
    corrections with zero multipliers solve the system exactly."""
    S, coef, sc = V.triangulation_instances(3, seed=22, sigma=0.0, sigma_rot_deg=0.0, sigma_t_rel=0.0,
                                            n_views=NV)
    for i in range(3):
        F = oracle.eval_system(S, coef[i], np.zeros(9, complex))
        F = F[0] if isinstance(F, tuple) else F
        assert np.max(np.abs(F)) < 1e-14


def test_start_set_has_the_papers_count():
    """Table 2 lists 94 solutions for 3-view triangulation; the stored monodromy
    set of the generic start instance has exactly that many, all regular roots
    (tiny backward error) and pairwise distinct."""
    S = V.triangulation_system(NV)
    c0, sols = V.start_instance(NV)
    assert sols.shape == (94, 9)
    assert max(oracle.residual(S, c0, x) for x in sols) < 1e-12
    assert len(M.distinct_rows(sols)) == 94


def test_monodromy_reproduces_the_start_set():
    """The stored set is what `python -m oracle.monodromy triang3` computes."""
    S = V.triangulation_system(NV)
    c0, sols = M.monodromy(S, seed=4, log=lambda *_: None)
    c0s, sols_s = V.start_instance(NV)
    assert np.array_equal(c0, c0s)
    assert len(sols) == len(sols_s)
    assert len(M.distinct_rows(np.concatenate([sols_s, sols]))) == len(sols_s)


@pytest.fixture(scope="module")
def tracked():
    """The oracle's parameter homotopy from the start instance to 3 scenes."""
    S = V.triangulation_system(NV)
    c0, sols = V.start_instance(NV)
    _, coef, sc = V.triangulation_instances(3, seed=24, n_views=NV)
    ep, st, info = oracle.track(S, coef, start=sols, coef0=c0, kind=oracle.LINEAR)
    return S, coef, ep, st, sc


def test_endpoints_are_distinct_critical_points(tracked):
    S, coef, ep, st, _ = tracked
    for i in range(3):
        ok = ep[i][st[i] == oracle.SUCCESS]
        assert 60 <= len(ok) <= 94
        assert len(M.distinct_rows(ok)) == len(ok)
        assert max(oracle.residual(S, coef[i], x) for x in ok) < 1e-10


def constrained_local_optimum(E, gam):
    """A local minimiser of sum u_k^2 + v_k^2 subject to the three epipolar
    constraints, by SLSQP from zero corrections."""
    from scipy.optimize import minimize

    def cons(z):
        out = []
        for p, (a, b) in enumerate(PAIRS):
            ga = gam[a] - np.array([z[2 * a], z[2 * a + 1], 0.0])
            gb = gam[b] - np.array([z[2 * b], z[2 * b + 1], 0.0])
            out.append(gb @ E[p] @ ga)
        return np.array(out)

    r = minimize(lambda z: z @ z, np.zeros(2 * NV), jac=lambda z: 2 * z, method="SLSQP",
                 constraints=[{"type": "eq", "fun": cons}], options={"ftol": 1e-16, "maxiter": 1000})
    assert np.max(np.abs(cons(r.x))) < 1e-12
    return r.x


def test_local_optimum_is_among_the_real_critical_points(tracked):
    """Homotopy continuation finds every critical point, so the local minimum an
    optimiser reaches is one of the real finite endpoints, and the least cost
    among them is no larger."""
    S, coef, ep, st, sc = tracked
    for i in range(3):
        ok = ep[i][st[i] == oracle.SUCCESS]
        real = ok[np.max(np.abs(ok.imag), axis=1) < 1e-8 * np.maximum(1.0, np.max(np.abs(ok), axis=1))].real
        assert len(real) > 0
        z = constrained_local_optimum(sc["E"][i], sc["gamma"][i])
        d = np.min(np.max(np.abs(real[:, :2 * NV] - z), axis=1))
        assert d <= 1e-6 * max(1.0, np.max(np.abs(z))), d
        assert np.min(np.sum(real[:, :2 * NV] ** 2, axis=1)) <= z @ z * (1 + 1e-9)
