"""FP64 endpoint refinement and classification on the GPU, both table layouts,
through the C ABI.

The reported residual must be the relative backward error of the returned
endpoint, eta = max_i |F_i(x)| / sum_k |c_ik| |m_k(x)| (recomputed here from
that definition with numpy, not from either implementation), and the
refinement controls (max_refine, eta_max) must act as documented: no Newton
iterations when max_refine = 0, and a residual above eta_max turns a reached
path into REFINE_FAILED without changing its endpoint.
"""
import numpy as np
import pytest

import hc_inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def hc():
    import paper_2112_03444_amd as hc
    return hc


@pytest.fixture(scope="module")
def ctx(hc):
    c = hc.Context(0)
    yield c
    c.close()


def backward_error(S, c, x):
    """eta(x) for the system S with term coefficients c [n_terms]."""
    exps = np.asarray(S.term_exp)
    m = np.prod(x[None, :] ** exps, axis=1)
    eq = np.asarray(S.term_eq)
    terms = c * m
    num = np.abs(np.bincount(eq, weights=terms.real, minlength=S.n)
                 + 1j * np.bincount(eq, weights=terms.imag, minlength=S.n))
    den = np.bincount(eq, weights=np.abs(c) * np.abs(m), minlength=S.n)
    return float(np.max(num / den))


LAYOUTS = [(2, "dense"), (5, "dense"), (8, "dense"), (8, "terms"), (10, "auto")]


@pytest.mark.parametrize("n,layout", LAYOUTS)
def test_residual_is_backward_error_of_endpoint(hc, ctx, n, layout):
    """Unrefined endpoints (max_refine = 0, every finite residual accepted):
    the reported residual is eta of the returned point, up to the rounding of
    the sums (n_terms units in the last place of the denominator)."""
    lay = {"dense": hc.HC_LAYOUT_DENSE, "terms": hc.HC_LAYOUT_TERMS, "auto": hc.HC_LAYOUT_AUTO}[layout]
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 2, seed=7100 + n)
    sysh = ctx.load_system(S, layout=lay)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(max_refine=0, eta_max=1.0))
    ok = st == hc.HC_T_SUCCESS
    assert ok.mean() > 0.9, np.bincount(st.ravel(), minlength=7)
    assert (info["refine_its"][ok] == 0).all()
    slack = 4 * S.n_terms * U
    for i, j in zip(*np.nonzero(ok)):
        ref = backward_error(S, coef[i], ep[i, j])
        got = info["residual"][i, j]
        assert abs(got - ref) <= 1e-6 * ref + slack, (i, j, got, ref)


@pytest.mark.parametrize("n,layout", LAYOUTS)
def test_refinement_controls(hc, ctx, n, layout):
    """Default refinement: 1..max_refine iterations and eta <= 1e-10 on every
    SUCCESS path; eta_max below any attainable residual: the same endpoints and
    residuals, every such path REFINE_FAILED instead."""
    lay = {"dense": hc.HC_LAYOUT_DENSE, "terms": hc.HC_LAYOUT_TERMS, "auto": hc.HC_LAYOUT_AUTO}[layout]
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 2, seed=7200 + n)
    sysh = ctx.load_system(S, layout=lay)
    ep0, st0, info0 = ctx.track(sysh, coef, gam)
    ok = st0 == hc.HC_T_SUCCESS
    assert ok.mean() > 0.9, np.bincount(st0.ravel(), minlength=7)
    its = info0["refine_its"][ok]
    assert ((its >= 1) & (its <= 10)).all()
    assert (info0["residual"][ok] <= 1e-10).all()
    ep1, st1, info1 = ctx.track(sysh, coef, gam, opts=hc.default_opts(eta_max=1e-300))
    assert (st1[ok] == hc.HC_T_REFINE_FAILED).all()
    np.testing.assert_array_equal(st1[~ok], st0[~ok])
    np.testing.assert_array_equal(ep1, ep0)
    np.testing.assert_array_equal(info1["residual"][ok], info0["residual"][ok])
