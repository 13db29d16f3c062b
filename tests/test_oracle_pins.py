"""Pins for the CPU oracle: each test checks it against something other than itself.

Kinds of pin used (no test re-types the oracle's own formula):
  * finite differences (the Jacobian and dH/dt are derivatives of what is evaluated);
  * hand-known values (x = 0 gives the constant terms, x = 1 gives coefficient sums);
  * a library routine (numpy.linalg.solve = LAPACK zgesv, numpy.roots = companion matrix);
  * a closed-form path for n = 1 (quadratic formula) and the order of RK4;
  * the Sylvester resultant for n = 2 (Cox, Little, O'Shea, ch. 3);
  * Bezout's theorem: 2**n distinct verified roots of a generic quadratic system are all of them;
  * mpmath 50-digit Newton polish; a planted root; gamma-invariance of the solution set.
"""
import numpy as np
import pytest

import hc_inputs
import oracle


def np_eval(system, coef, x):
    """Independent numpy evaluation of F (vectorised over terms) used only to verify roots."""
    mons = np.prod(np.power(x[None, :], system.term_exp), axis=1)
    F = np.zeros(system.n, np.complex128)
    np.add.at(F, system.term_eq, coef * mons)
    return F


def match_sets(a, b, tol):
    """Greedy one-to-one nearest matching of the rows of a and b; returns the max rel. error."""
    a = list(a)
    b = list(b)
    assert len(a) == len(b)
    worst = 0.0
    for p in a:
        d = [np.max(np.abs(p - q)) / max(1.0, np.max(np.abs(q))) for q in b]
        j = int(np.argmin(d))
        worst = max(worst, d[j])
        b.pop(j)
    assert worst <= tol, worst
    return worst


# ---------------------------------------------------------------- evaluation

def test_eval_special_points():
    S, c, _ = hc_inputs.dense_quadratic_instances(4, 1, seed=11)
    c = c[0]
    T = 15  # C(6,2)
    F0, J0 = oracle.eval_system(S, c, np.zeros(4))
    # at x = 0 only the constant term survives, and dF_i/dx_j is the x_j coefficient
    np.testing.assert_array_equal(F0, c.reshape(4, T)[:, 0])
    np.testing.assert_array_equal(J0, c.reshape(4, T)[:, 1:5])
    # at x = 1 every monomial is 1
    F1, _ = oracle.eval_system(S, c, np.ones(4))
    np.testing.assert_allclose(F1, c.reshape(4, T).sum(axis=1), rtol=1e-14)
    # x = 2 e_1: monomials 1, x1, x1^2 give 1, 2, 4
    F2, _ = oracle.eval_system(S, c, np.array([2, 0, 0, 0]))
    cc = c.reshape(4, T)
    np.testing.assert_allclose(F2, cc[:, 0] + 2 * cc[:, 1] + 4 * cc[:, 5], rtol=1e-14)


def test_jacobian_matches_finite_differences():
    rng = np.random.default_rng(5)
    for n in (2, 3, 5):
        S, c, _ = hc_inputs.dense_quadratic_instances(n, 1, seed=20 + n)
        x = hc_inputs.complex_gaussian(rng, n)
        _, J = oracle.eval_system(S, c[0], x)
        h = 1e-6
        for j in range(n):
            e = np.zeros(n)
            e[j] = h
            Fp, _ = oracle.eval_system(S, c[0], x + e)
            Fm, _ = oracle.eval_system(S, c[0], x - e)
            # holomorphic: the same derivative along the imaginary direction
            Fpi, _ = oracle.eval_system(S, c[0], x + 1j * e)
            Fmi, _ = oracle.eval_system(S, c[0], x - 1j * e)
            fd = (Fp - Fm) / (2 * h)
            fdi = (Fpi - Fmi) / (2j * h)
            scale = np.max(np.abs(J)) + 1.0
            assert np.max(np.abs(J[:, j] - fd)) <= 1e-8 * scale
            assert np.max(np.abs(J[:, j] - fdi)) <= 1e-8 * scale


def test_cubic_system_derivatives():
    # a sparse system with a cubic term, to exercise exponents > 2
    S = hc_inputs.PolySystem(
        n=2,
        term_eq=np.array([0, 0, 0, 1, 1], np.int32),
        term_exp=np.array([[2, 1], [0, 1], [0, 0], [1, 0], [0, 3]], np.int32))
    c = np.array([1.5 - 0.5j, 2j, -1, 0.25, 3 + 1j])
    x = np.array([0.7 - 0.2j, -1.1 + 0.4j])
    F, J = oracle.eval_system(S, c, x)
    # hand-expanded: F0 = c0 x1^2 x2 + c1 x2 + c2, F1 = c3 x1 + c4 x2^3
    x1, x2 = x
    assert abs(F[0] - (c[0] * x1 * x1 * x2 + c[1] * x2 + c[2])) < 1e-14
    assert abs(F[1] - (c[3] * x1 + c[4] * x2 ** 3)) < 1e-14
    assert abs(J[0, 0] - 2 * c[0] * x1 * x2) < 1e-14
    assert abs(J[0, 1] - (c[0] * x1 * x1 + c[1])) < 1e-14
    assert abs(J[1, 1] - 3 * c[4] * x2 * x2) < 1e-13
    np.testing.assert_array_equal(oracle.degrees(S), [3, 3])


@pytest.mark.parametrize("kind", [oracle.TOTAL_DEGREE, oracle.LINEAR])
def test_homotopy_time_derivative_and_endpoints(kind):
    n = 3
    S, c, g = hc_inputs.dense_quadratic_instances(n, 2, seed=31)
    rng = np.random.default_rng(3)
    x = hc_inputs.complex_gaussian(rng, n)
    kw = dict(coef1=c[1], gamma=g[0], kind=kind, coef0=c[0] if kind == oracle.LINEAR else None)
    t, d = 0.37, 1e-6
    _, Hx, Ht = oracle.homotopy_eval(S, x, t, **kw)
    Hp, _, _ = oracle.homotopy_eval(S, x, t + d, **kw)
    Hm, _, _ = oracle.homotopy_eval(S, x, t - d, **kw)
    np.testing.assert_allclose(Ht, (Hp - Hm) / (2 * d), rtol=0, atol=1e-8 * (1 + np.abs(Ht).max()))
    # H(., 1) is the target system
    H1, Hx1, _ = oracle.homotopy_eval(S, x, 1.0, **kw)
    F1, J1 = oracle.eval_system(S, c[1], x)
    np.testing.assert_allclose(H1, F1, rtol=1e-14)
    np.testing.assert_allclose(Hx1, J1, rtol=1e-14)
    H0, Hx0, _ = oracle.homotopy_eval(S, x, 0.0, **kw)
    if kind == oracle.LINEAR:
        F0, J0 = oracle.eval_system(S, c[0], x)
        np.testing.assert_allclose(H0, F0, rtol=1e-14)
    else:
        # H(., 0) = gamma (x_i^2 - 1): zero at every total-degree start point
        for b in range(2 ** n):
            xs = oracle.total_degree_start(S, b)
            H0s, _, _ = oracle.homotopy_eval(S, xs, 0.0, **kw)
            assert np.max(np.abs(H0s)) == 0.0
        np.testing.assert_allclose(H0, g[0] * (x * x - 1), rtol=1e-14)


def test_total_degree_start_points():
    # degrees (2, 3, 1): 6 start points, each with x_i^d_i = 1, all distinct
    S = hc_inputs.PolySystem(
        n=3, term_eq=np.array([0, 1, 2], np.int32),
        term_exp=np.array([[2, 0, 0], [1, 1, 1], [0, 0, 1]], np.int32))
    d = oracle.degrees(S)
    np.testing.assert_array_equal(d, [2, 3, 1])
    pts = np.array([oracle.total_degree_start(S, b) for b in range(6)])
    np.testing.assert_allclose(pts ** d[None, :], np.ones((6, 3)), atol=1e-15)
    assert len({tuple(np.round(p, 12)) for p in pts}) == 6
    # bit/digit convention: x_1 is the least significant digit
    np.testing.assert_array_equal(pts[1], [-1, 1, 1])


# ---------------------------------------------------------------- linear solve

def test_lu_solve_matches_lapack():
    rng = np.random.default_rng(7)
    for n in (1, 2, 3, 8, 14, 18, 32):
        A = hc_inputs.complex_gaussian(rng, (n, n))
        b = hc_inputs.complex_gaussian(rng, n)
        x = oracle.lu_solve(A, b)
        ref = np.linalg.solve(A, b)
        assert np.max(np.abs(x - ref)) <= 1e-10 * np.max(np.abs(ref)) * np.linalg.cond(A)
        # normwise backward error (Higham, ch. 9) within a small multiple of n u
        r = np.linalg.norm(A @ x - b, np.inf)
        eta = r / (np.linalg.norm(A, np.inf) * np.linalg.norm(x, np.inf) + np.linalg.norm(b, np.inf))
        assert eta <= 4 * n * 2.0 ** -53


def test_lu_needs_pivoting_and_graded():
    # zero leading entry: only a row interchange makes elimination possible
    A = np.array([[0, 1, 2], [3, 0, 1], [1, 1, 0]], np.complex128)
    b = np.array([1, 2, 3], np.complex128)
    np.testing.assert_allclose(oracle.lu_solve(A, b), np.linalg.solve(A, b), rtol=1e-14)
    # a tiny pivot that must be skipped: without pivoting the answer is garbage
    A = np.array([[1e-20, 1], [1, 1]], np.complex128)
    b = np.array([1, 2], np.complex128)
    np.testing.assert_allclose(oracle.lu_solve(A, b), [1, 1], rtol=1e-14)
    # strongly graded rows
    rng = np.random.default_rng(8)
    A = hc_inputs.complex_gaussian(rng, (6, 6)) * (10.0 ** np.arange(6))[:, None]
    b = hc_inputs.complex_gaussian(rng, 6)
    x = oracle.lu_solve(A, b)
    r = np.linalg.norm(A @ x - b, np.inf)
    assert r <= 1e-12 * (np.linalg.norm(A, np.inf) * np.linalg.norm(x, np.inf))
    # exactly singular: a zero pivot is reported
    A = np.array([[1, 2], [2, 4]], np.complex128)
    assert oracle.lu_solve(A, np.array([1, 1], np.complex128)) is None


def test_lu_small_integer_exact():
    # integer data whose solution is exactly representable
    A = np.array([[2, 1, 1], [4, -6, 0], [-2, 7, 2]], np.complex128)
    x_true = np.array([1, 1, 2], np.complex128)
    np.testing.assert_allclose(oracle.lu_solve(A, A @ x_true), x_true, rtol=1e-15)


# ---------------------------------------------------------------- n = 1: closed forms

def _n1(seed):
    S, c, g = hc_inputs.dense_quadratic_instances(1, 1, seed=seed)
    return S, c[0], g[0]


def _closed_form_path(c, gam, x0, t_end=1.0, n_grid=20000):
    """Follow the root of (1-t) gam (x^2 - 1) + t (c2 x^2 + c1 x + c0) by the quadratic formula."""
    c0, c1, c2 = c
    x = x0
    for t in np.linspace(0.0, t_end, n_grid + 1)[1:]:
        A = (1 - t) * gam + t * c2
        B = t * c1
        C = -(1 - t) * gam + t * c0
        s = np.sqrt(B * B - 4 * A * C + 0j)
        r = np.array([(-B + s) / (2 * A), (-B - s) / (2 * A)])
        x = r[np.argmin(np.abs(r - x))]
    return x


def test_rk4_order_on_closed_form_path():
    S, c, g = _n1(41)
    x_exact = _closed_form_path(c, g, 1.0 + 0j)
    errs = []
    for N in (32, 64, 128):
        x = oracle.rk4_fixed(S, np.array([1.0 + 0j]), N, coef1=c, gamma=g)
        errs.append(abs(x[0] - x_exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    # fourth order: halving h divides the error by about 2^4
    assert 13 < r1 < 19 and 13 < r2 < 19, (errs, r1, r2)


def test_tracker_n1_matches_companion_roots():
    for seed in (41, 42, 43):
        S, c, g = _n1(seed)
        ep, st, info = oracle.track(S, c[None, :], g)
        assert list(st[0]) == [oracle.SUCCESS] * 2
        ref = np.roots([c[2], c[1], c[0]])
        match_sets(ep[0, :, 0:1], ref[:, None], 1e-12)
        # each endpoint is also the end of the closed-form path from its own start point
        for b in range(2):
            x0 = oracle.total_degree_start(S, b)[0]
            assert abs(ep[0, b, 0] - _closed_form_path(c, g, x0)) < 1e-6


# ---------------------------------------------------------------- Newton

def test_newton_converges_quadratically():
    S, c, g = hc_inputs.dense_quadratic_instances(3, 1, seed=51)
    ep, st, _ = oracle.track(S, c, g)
    assert (st == oracle.SUCCESS).all()
    root = ep[0, 0]
    x0 = root + 1e-3 * np.array([1, -1j, 0.5 + 0.5j])
    norms, x = oracle.newton_trace(S, x0, 1.0, 4, coef1=c[0], gamma=g[0])
    assert norms[1] <= 100 * norms[0] ** 2
    assert norms[2] <= 100 * norms[1] ** 2 + 1e-15
    assert np.max(np.abs(x - root)) <= 1e-13 * max(1, np.max(np.abs(root)))


# ---------------------------------------------------------------- n = 2: resultant

def _resultant_roots_n2(c):
    """Common roots of two dense quadratics via the Sylvester resultant in x2.

    Monomials [1, x1, x2, x1^2, x1 x2, x2^2].  Each f = A2 x2^2 + A1(x1) x2 + A0(x1);
    Res = (A2 B0 - A0 B2)^2 - (A2 B1 - A1 B2)(A1 B0 - A0 B1), a quartic in x1.
    """
    P = np.polynomial.polynomial
    f, g = c.reshape(2, 6)

    def parts(q):
        return (np.array([q[5]]), np.array([q[2], q[4]]), np.array([q[0], q[1], q[3]]))

    A2, A1, A0 = parts(f)
    B2, B1, B0 = parts(g)
    t1 = P.polysub(P.polymul(A2, B0), P.polymul(A0, B2))
    t2 = P.polysub(P.polymul(A2, B1), P.polymul(A1, B2))
    t3 = P.polysub(P.polymul(A1, B0), P.polymul(A0, B1))
    res = P.polysub(P.polymul(t1, t1), P.polymul(t2, t3))
    # the same determinant numerically at a test point (guards the closed form)
    z = 0.3 - 0.7j
    M = np.array([[P.polyval(z, A2)[()], P.polyval(z, A1), P.polyval(z, A0), 0],
                  [0, P.polyval(z, A2)[()], P.polyval(z, A1), P.polyval(z, A0)],
                  [P.polyval(z, B2)[()], P.polyval(z, B1), P.polyval(z, B0), 0],
                  [0, P.polyval(z, B2)[()], P.polyval(z, B1), P.polyval(z, B0)]], np.complex128)
    assert abs(np.linalg.det(M) - P.polyval(z, res)) < 1e-10 * (1 + abs(P.polyval(z, res)))
    roots = []
    for x1 in np.roots(res[::-1]):
        a2, a1, a0 = (P.polyval(x1, A2), P.polyval(x1, A1), P.polyval(x1, A0))
        b2, b1, b0 = (P.polyval(x1, B2), P.polyval(x1, B1), P.polyval(x1, B0))
        # b2 f - a2 g is linear in x2
        x2 = -(b2 * a0 - a2 * b0) / (b2 * a1 - a2 * b1)
        roots.append(np.array([x1, x2]).ravel())
    return np.array(roots)


def _polish(S, c, x, iters=6):
    """Newton polish with an independent numpy Jacobian by complex-step-free differences."""
    x = np.array(x, np.complex128)
    for _ in range(iters):
        F = np_eval(S, c, x)
        n = len(x)
        J = np.zeros((n, n), np.complex128)
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1e-7
            J[:, j] = (np_eval(S, c, x + e) - np_eval(S, c, x - e)) / 2e-7
        x = x - np.linalg.solve(J, F)
    return x


def test_tracker_n2_matches_resultant():
    for seed in (61, 62, 63):
        S, c, g = hc_inputs.dense_quadratic_instances(2, 1, seed=seed)
        ep, st, _ = oracle.track(S, c, g)
        assert (st == oracle.SUCCESS).all()
        ref = np.array([_polish(S, c[0], r) for r in _resultant_roots_n2(c[0])])
        match_sets(ep[0], ref, 1e-9)


# ---------------------------------------------------------------- n >= 3: Bezout, mpmath, planted

@pytest.mark.parametrize("n,seed", [(3, 1), (3, 71), (4, 72), (5, 73), (6, 74)])
def test_bezout_count_distinct_verified(n, seed):
    S, c, g = hc_inputs.dense_quadratic_instances(n, 1, seed=seed)
    ep, st, info = oracle.track(S, c, g)
    assert (st == oracle.SUCCESS).all()
    assert ep.shape[1] == 2 ** n
    for x in ep[0]:
        F = np_eval(S, c[0], x)
        den = np.zeros(n)
        np.add.at(den, S.term_eq, np.abs(c[0]) * np.abs(np.prod(np.power(x[None, :], S.term_exp), 1)))
        assert np.max(np.abs(F) / den) <= 1e-13
    d = np.abs(ep[0][:, None, :] - ep[0][None, :, :]).max(-1) + np.eye(2 ** n) * 1e9
    assert d.min() > 1e-6
    assert np.all(info["residual"] <= 1e-13)


def test_quintic_n1_matches_companion_roots():
    """Degree 5 in one unknown (start system x^5 - 1, five roots of unity): the
    endpoints are numpy.roots' companion-matrix eigenvalues."""
    S = hc_inputs.support_system(1, [(5, [0])])
    rng = np.random.default_rng(44)
    c = hc_inputs.complex_gaussian(rng, (1, S.n_terms))
    g = hc_inputs.unit_gammas(rng, 1)
    ep, st, _ = oracle.track(S, c, g)
    assert ep.shape[1] == 5 and (st == oracle.SUCCESS).all()
    coeffs = np.zeros(6, complex)  # highest power first
    for k in range(S.n_terms):
        coeffs[5 - S.term_exp[k, 0]] += c[0, k]
    match_sets(ep[0], np.roots(coeffs)[:, None], 1e-10)


@pytest.mark.parametrize("spec,seed", [([(3, [0, 1]), (2, [0, 1])], 45),
                                       ([(4, [0, 1, 2]), (3, [0, 1, 2]), (2, [0, 1, 2])], 46),
                                       ([(5, [0, 1]), (1, [0, 1, 2]), (2, [1, 2])], 47)])
def test_bezout_count_mixed_degrees(spec, seed):
    """Equations dense on their supports with degrees d_i: prod d_i distinct,
    verified finite roots (Bezout; generic coefficients)."""
    n = len(spec)
    S = hc_inputs.support_system(n, spec)
    rng = np.random.default_rng(seed)
    c = hc_inputs.complex_gaussian(rng, (1, S.n_terms))
    g = hc_inputs.unit_gammas(rng, 1)
    ep, st, info = oracle.track(S, c, g)
    bez = int(np.prod([d for d, _ in spec]))
    assert ep.shape[1] == bez and (st == oracle.SUCCESS).all()
    for x in ep[0]:
        F = np_eval(S, c[0], x)
        den = np.zeros(n)
        np.add.at(den, S.term_eq, np.abs(c[0]) * np.abs(np.prod(np.power(x[None, :], S.term_exp), 1)))
        assert np.max(np.abs(F) / den) <= 1e-12
    d = np.abs(ep[0][:, None, :] - ep[0][None, :, :]).max(-1) + np.eye(bez) * 1e9
    assert d.min() > 1e-6


def test_config1_roots_polish_in_50_digits():
    mpmath = pytest.importorskip("mpmath")
    S, c, g = hc_inputs.workload("dense3_single")
    ep, st, _ = oracle.track(S, c, g)
    assert (st == oracle.SUCCESS).all()
    mpmath.mp.dps = 50
    cc = [mpmath.mpc(complex(v)) for v in c[0]]

    def F(*xs):
        out = [mpmath.mpc(0)] * 3
        for k in range(S.n_terms):
            m = cc[k]
            for j in range(3):
                m *= xs[j] ** int(S.term_exp[k, j])
            out[S.term_eq[k]] += m
        return out

    for x in ep[0]:
        r = mpmath.findroot(F, [mpmath.mpc(complex(v)) for v in x])
        r = np.array([complex(r[j]) for j in range(3)])
        assert np.max(np.abs(r - x)) <= 1e-13 * max(1, np.max(np.abs(r)))


def test_gamma_invariance():
    S, c, g = hc_inputs.dense_quadratic_instances(4, 1, seed=81)
    ep1, st1, _ = oracle.track(S, c, g)
    ep2, st2, _ = oracle.track(S, c, np.exp(1j * 2.1))
    assert (st1 == 0).all() and (st2 == 0).all()
    match_sets(ep1[0], ep2[0], 1e-10)


def test_planted_root_is_found():
    n = 4
    S, c, g = hc_inputs.dense_quadratic_instances(n, 1, seed=91)
    rng = np.random.default_rng(92)
    xstar = hc_inputs.complex_gaussian(rng, n)
    c = c[0].copy()
    T = c.size // n
    # move each equation's constant term so that F(x*) = 0
    mons = np.prod(np.power(xstar[None, :], S.term_exp), axis=1)
    for i in range(n):
        sl = slice(i * T, (i + 1) * T)
        c[i * T] = -np.sum(c[sl][1:] * mons[sl][1:])
    ep, st, _ = oracle.track(S, c[None, :], g)
    assert (st == 0).all()
    d = np.abs(ep[0] - xstar[None, :]).max(-1)
    assert d.min() <= 1e-10


def test_linear_parameter_homotopy_reaches_target_roots():
    n = 3
    S, c, g = hc_inputs.dense_quadratic_instances(n, 2, seed=101)
    ep0, st0, _ = oracle.track(S, c[0:1], g[0:1])
    ep1, st1, _ = oracle.track(S, c[1:2], g[1:2])
    assert (st0 == 0).all() and (st1 == 0).all()
    epL, stL, _ = oracle.track(S, c[1:2], start=ep0[0], coef0=c[0], kind=oracle.LINEAR)
    assert (stL == 0).all()
    match_sets(epL[0], ep1[0], 1e-9)


# ---------------------------------------------------------------- failure statuses

def test_path_to_infinity():
    # F = (x1 x2 - 1, x1 - 2): degrees (2, 1), Bezout 2, one finite root (2, 1/2)
    S = hc_inputs.PolySystem(
        n=2, term_eq=np.array([0, 0, 1, 1], np.int32),
        term_exp=np.array([[1, 1], [0, 0], [1, 0], [0, 0]], np.int32))
    c = np.array([1, -1, 1, -2], np.complex128)
    ep, st, _ = oracle.track(S, c[None, :], np.exp(0.7j))
    assert sorted(st[0].tolist()) == [oracle.SUCCESS, oracle.AT_INFINITY]
    ok = ep[0][st[0] == oracle.SUCCESS][0]
    np.testing.assert_allclose(ok, [2, 0.5], rtol=1e-12)


def test_double_root_is_not_success():
    # F = (x1^2, x2 - 1): both paths end at the double root (0, 1)
    S = hc_inputs.PolySystem(
        n=2, term_eq=np.array([0, 1, 1], np.int32),
        term_exp=np.array([[2, 0], [0, 1], [0, 0]], np.int32))
    c = np.array([1, 1, -1], np.complex128)
    ep, st, _ = oracle.track(S, c[None, :], np.exp(0.3j))
    assert not (st == oracle.SUCCESS).any()


def test_forced_failures():
    S, c, g = hc_inputs.dense_quadratic_instances(3, 1, seed=1)
    bad = c.copy()
    bad[0, 4] = np.nan
    _, st, _ = oracle.track(S, bad, g)
    assert (st == oracle.NONFINITE).all()
    _, st, _ = oracle.track(S, c, g, opts=oracle.default_opts(max_steps=1))
    assert (st == oracle.MAX_STEPS).all()
    _, st, info = oracle.track(S, c, g, opts=oracle.default_opts(max_newton=0, h_min=0.04))
    assert (st == oracle.MIN_STEP).all() and (info["rejects"] == 1).all()


def test_residual_hand_value():
    # F = x - 2 (terms x and 1, coefficients 1 and -2) at x = 3:
    # |F| = 1 and sum |c| |m| = 3 + 2, so the relative backward error is 1/5
    S = hc_inputs.PolySystem(n=1, term_eq=np.array([0, 0], np.int32),
                             term_exp=np.array([[1], [0]], np.int32))
    assert abs(oracle.residual(S, np.array([1, -2], np.complex128), np.array([3.0])) - 0.2) < 1e-15
    # at the root it is exactly zero; a zero denominator with F = 0 counts as zero
    assert oracle.residual(S, np.array([1, -2], np.complex128), np.array([2.0])) == 0.0
    assert oracle.residual(S, np.array([0, 0], np.complex128), np.array([2.0])) == 0.0
