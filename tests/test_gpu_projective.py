"""Projective (random-patch) tracking on the GPU (paper_2112_03444_amd.projective:
the homogenized system plus a patch equation tracked by the same kernels
through the C ABI), against the oracle on an independently homogenized
system: the root at infinity is classified at infinity with a bounded
projective endpoint, and the finite roots equal the affine ones."""
import numpy as np
import pytest

import hc_inputs
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hc():
    import paper_2112_03444_amd as hc
    return hc


@pytest.fixture(scope="module")
def ctx(hc):
    c = hc.Context(0)
    yield c
    c.close()


def homogenize_here(S, coef, a):
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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_root_at_infinity(hc, ctx, precision):
    import paper_2112_03444_amd.projective as PJ
    S = hc_inputs.PolySystem(n=2, term_eq=np.array([0, 0, 1, 1], np.int32),
                             term_exp=np.array([[1, 1], [0, 0], [1, 0], [0, 0]], np.int32))
    coef = np.array([[1, -1, 1, -2]], np.complex128)
    g = np.array([np.exp(0.7j)])
    x, st, info, xh = PJ.track_projective(ctx, S, coef, g, opts=hc.default_opts(precision=precision), seed=3)
    assert sorted(st[0].tolist()) == [hc.HC_T_SUCCESS, hc.HC_T_AT_INFINITY]
    np.testing.assert_allclose(x[0][st[0] == hc.HC_T_SUCCESS][0], [2.0, 0.5], rtol=1e-12)
    assert np.all(np.isfinite(xh)) and np.max(np.abs(xh)) < 1e3  # bounded in projective space
    # the oracle on the same homogenized system and patch reaches the same points
    a = PJ.random_patch(2, np.random.default_rng(3))
    S2, c2 = homogenize_here(S, coef[0], a)
    oep, ost, _ = oracle.track(S2, c2[None, :], g)
    for p in xh[0]:
        d = np.max(np.abs(oep[0] - p), axis=1) / max(1.0, np.max(np.abs(p)))
        assert d.min() < 1e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [3, 5])
def test_finite_roots_equal_affine(hc, ctx, n, precision):
    import paper_2112_03444_amd.projective as PJ
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 3, seed=7400 + n)
    x, st, info, _ = PJ.track_projective(ctx, S, coef, gam, opts=hc.default_opts(precision=precision), seed=4)
    oep, ost, _ = oracle.track(S, coef, gam)
    for i in range(3):
        fin = x[i][st[i] == hc.HC_T_SUCCESS]
        ofin = oep[i][ost[i] == oracle.SUCCESS]
        assert len(fin) == len(ofin) == 2 ** n
        for y in ofin:
            d = np.max(np.abs(fin - y), axis=1) / max(1.0, np.max(np.abs(y)))
            assert d.min() < 1e-9
