"""Projective (random-patch) tracking, on the CPU: the package's homogenized
system against an independent construction written here, the
dehomogenization identity F^(x, 1) = F(x) and homogeneity of F^, and the
oracle tracking the homogenized system: a root at infinity ends with x_h -> 0
(bounded in projective space) while the finite roots equal the affine ones."""
import numpy as np

import hc_inputs
import oracle
import paper_2112_03444_amd.projective as PJ


def homogenize_here(S, coef, a):
    """Independent construction: for every equation, each term times x_h to
    the equation degree minus its own; then the patch a . (x, x_h) - 1."""
    n = S.n
    rows_eq, rows_ex, c = [], [], []
    for i in range(n):
        ks = [k for k in range(S.n_terms) if S.term_eq[k] == i]
        d = max(int(np.sum(S.term_exp[k])) for k in ks)
        for k in ks:
            rows_eq.append(i)
            rows_ex.append(list(S.term_exp[k]) + [d - int(np.sum(S.term_exp[k]))])
            c.append(coef[k])
    for j in range(n + 1):
        e = [0] * (n + 1)
        e[j] = 1
        rows_eq.append(n)
        rows_ex.append(e)
        c.append(a[j])
    rows_eq.append(n)
    rows_ex.append([0] * (n + 1))
    c.append(-1.0)
    return hc_inputs.PolySystem(n=n + 1, term_eq=np.array(rows_eq, np.int32),
                                term_exp=np.array(rows_ex, np.int32)), np.array(c, np.complex128)


def at_infinity_example():
    # F = (x1 x2 - 1, x1 - 2): Bezout 2, one finite root (2, 1/2), one at infinity
    S = hc_inputs.PolySystem(n=2, term_eq=np.array([0, 0, 1, 1], np.int32),
                             term_exp=np.array([[1, 1], [0, 0], [1, 0], [0, 0]], np.int32))
    return S, np.array([[1, -1, 1, -2]], np.complex128)


def evaluate(S, c, x):
    F = oracle.eval_system(S, c, x)
    return F[0] if isinstance(F, tuple) else F


def test_package_homogenization_equals_independent_one():
    rng = np.random.default_rng(51)
    for S, coef in (at_infinity_example(), hc_inputs.dense_quadratic_instances(3, 1, seed=52)[:2]):
        a = PJ.random_patch(S.n, rng)
        H = PJ.homogenize_system(S)
        ch = PJ.coefficients(coef, a)[0]
        S2, c2 = homogenize_here(S, coef[0], a)
        for _ in range(3):
            x = rng.standard_normal(S.n + 1) + 1j * rng.standard_normal(S.n + 1)
            np.testing.assert_allclose(evaluate(H, ch, x), evaluate(S2, c2, x), rtol=1e-13, atol=1e-13)


def test_dehomogenization_and_homogeneity():
    rng = np.random.default_rng(53)
    S, coef, _ = hc_inputs.dense_quadratic_instances(3, 1, seed=54)
    a = PJ.random_patch(3, rng)
    H = PJ.homogenize_system(S)
    ch = PJ.coefficients(coef, a)[0]
    x = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    F = evaluate(S, coef[0], x)
    Fh = evaluate(H, ch, np.concatenate([x, [1.0]]))
    np.testing.assert_allclose(Fh[:3], F, rtol=1e-13, atol=1e-13)
    xh = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    lam = 0.7 - 1.3j
    np.testing.assert_allclose(evaluate(H, ch, lam * xh)[:3], lam ** 2 * evaluate(H, ch, xh)[:3], rtol=1e-12)


def test_oracle_projective_tracking():
    """The root at infinity is reached with x_h -> 0 (both paths converge; the
    relative backward error is 0/0 at that root, where every term of the first
    equation vanishes); the finite one is (2, 1/2)."""
    S, coef = at_infinity_example()
    a = PJ.random_patch(2, np.random.default_rng(55))
    S2, c2 = homogenize_here(S, coef[0], a)
    g = np.array([np.exp(0.7j)])
    ep, st, info = oracle.track(S2, c2[None, :], g)
    h = ep[0][:, 2]
    inf = np.abs(h) <= 1e-8 * np.max(np.abs(ep[0]), axis=1)
    assert inf.sum() == 1
    assert st[0][~inf][0] == oracle.SUCCESS
    assert st[0][inf][0] in (oracle.SUCCESS, oracle.REFINE_FAILED)
    assert np.max(np.abs(evaluate(S2, c2, ep[0][inf][0]))) < 1e-14
    fin = ep[0][~inf][0]
    np.testing.assert_allclose(fin[:2] / fin[2], [2.0, 0.5], rtol=1e-12)


def test_finite_roots_equal_affine_tracking():
    S, coef, gam = hc_inputs.dense_quadratic_instances(3, 2, seed=56)
    a = PJ.random_patch(3, np.random.default_rng(57))
    ep, st, _ = oracle.track(S, coef, gam)
    for i in range(2):
        S2, c2 = homogenize_here(S, coef[i], a)
        eh, sh, _ = oracle.track(S2, c2[None, :], gam[i:i + 1])
        assert (sh[0] == oracle.SUCCESS).all()
        x = eh[0][:, :3] / eh[0][:, 3:]
        fin = ep[i][st[i] == oracle.SUCCESS]
        assert len(fin) == 8
        for y in fin:
            d = np.max(np.abs(x - y), axis=1) / max(1.0, np.max(np.abs(y)))
            assert d.min() < 1e-9
