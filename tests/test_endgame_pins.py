"""Pins of the oracle's power-series end-game (Morgan, Sommese and Wampler, Numer.
Math. 63, 1992), which the paper does not have (section 2 only warns that the
number of solutions HC reports needs checking): paths are sampled at geometric
distances s = 1 - t from the end, the cycle number c is estimated from how fast
successive samples approach each other, and the endpoint is extrapolated in
sigma = s^(1/c) in projective coordinates on a fixed patch.

Pinned against closed forms and facts of the systems themselves:
- the estimator on fractional power series whose limit and cycle number are
  known exactly;
- a double and a triple root of known position and multiplicity (every path's
  cycle number is the multiplicity of a generically perturbed isolated root of
  F = (x1^m, x2 - 1));
- a system with no finite root, whose paths can only go to infinity;
- regular paths, which the end-game must leave where the plain tracker puts them
  (cycle number 1, the same root)."""
import numpy as np
import pytest

import hc_inputs
import hc_inputs.vision as V
import oracle


def poly2(eq, exps):
    return hc_inputs.PolySystem(n=2, term_eq=np.array(eq, np.int32), term_exp=np.array(exps, np.int32))


@pytest.mark.parametrize("c", [1, 2, 3, 4])
def test_estimator_exact_on_quadratics_in_sigma(c):
    """y(s) = a + b sigma + d sigma^2 with sigma = s^(1/c): the cycle number is c
    and the quadratic extrapolation in sigma returns a to rounding."""
    rng = np.random.default_rng(c)
    a, b, d = (rng.standard_normal((3, 5)) + 1j * rng.standard_normal((3, 5)))
    d *= 0.1
    beta, s = 0.25, 1e-3
    ys = [a + b * (s * beta ** k) ** (1 / c) + d * (s * beta ** k) ** (2 / c) for k in range(3)]
    cyc, E = oracle.eg_extrapolate(*ys, beta)
    assert cyc == c
    np.testing.assert_allclose(E, a, rtol=0, atol=1e-12)


def test_estimator_error_order_and_no_decay():
    """A cubic term in sigma is what the estimate misses: the error shrinks like
    sigma^3 (by beta^(3/c) per sample); growing samples give no estimate."""
    a, b, e = 1.0 + 2.0j, 0.7 - 0.2j, 0.3 + 0.1j
    beta, c = 0.25, 2
    errs = []
    for k0 in range(6):
        ss = [1e-2 * beta ** (k0 + k) for k in range(3)]
        ys = [np.array([a + b * s ** (1 / c) + e * s ** (3 / c)]) for s in ss]
        cyc, E = oracle.eg_extrapolate(*ys, beta)
        assert cyc == c
        errs.append(abs(E[0] - a))
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    np.testing.assert_allclose(ratios, beta ** (3 / c), rtol=1e-3)
    grow = [np.array([1.0 / s]) for s in (1e-2, 2.5e-3, 6.25e-4)]
    assert oracle.eg_extrapolate(*grow, 0.25) is None


@pytest.mark.parametrize("m", [2, 3])
def test_multiple_root_of_known_multiplicity(m):
    """F = (x1^m, x2 - 1): the only root (0, 1) has multiplicity m; without the
    end-game no path succeeds, with it all m paths end there with cycle number m
    and status SINGULAR_END."""
    S = poly2([0, 1, 1], [[m, 0], [0, 1], [0, 0]])
    c = np.array([1, 1, -1], np.complex128)
    _, st0, _ = oracle.track(S, c[None, :], np.exp(0.3j))
    assert not (st0 == oracle.SUCCESS).any()
    ep, st, info, cyc = oracle.track(S, c[None, :], np.exp(0.3j), endgame=True)
    assert (st == oracle.SINGULAR_END).all()
    assert (cyc == m).all()
    assert np.max(np.abs(ep[0] - np.array([0.0, 1.0]))) <= 1e-8
    assert (info["refine_its"] == 0).all()


def test_no_finite_root_goes_to_infinity():
    """F = (x1 x2 - 1, x1 x2 - 2) has no finite root (x1 x2 cannot be 1 and 2), so
    every one of its 4 total-degree paths diverges; the plain tracker stops them
    at the minimum step, the end-game classifies them at infinity."""
    S = poly2([0, 0, 1, 1], [[1, 1], [0, 0], [1, 1], [0, 0]])
    c = np.array([1, -1, 1, -2], np.complex128)
    _, st0, _ = oracle.track(S, c[None, :], np.exp(0.3j))
    assert (st0 != oracle.SUCCESS).all()
    ep, st, info, cyc = oracle.track(S, c[None, :], np.exp(0.3j), endgame=True)
    assert (st == oracle.AT_INFINITY).all()
    assert (cyc >= 1).all()
    assert np.isnan(info["residual"]).all()


@pytest.mark.parametrize("n", [2, 3, 4])
def test_end_game_leaves_regular_paths_alone(n):
    """With every path sent through the end-game, regular paths report cycle
    number 1 and the plain tracker's root (after the same FP64 refinement)."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(n, 2, seed=40 + n)
    ep0, st0, _ = oracle.track(S, coef, gam)
    ep, st, info, cyc = oracle.track(S, coef, gam, endgame=oracle.default_eg_opts(every=1))
    ok = st0 == oracle.SUCCESS
    assert ok.all() and (st == oracle.SUCCESS).all()
    assert (cyc == 1).all()
    err = np.max(np.abs(ep - ep0), axis=-1) / np.maximum(1.0, np.max(np.abs(ep0), axis=-1))
    assert err.max() <= 1e-12


def test_end_game_only_touches_failed_paths():
    """By default only failed paths take the end-game: every SUCCESS of the plain
    tracker keeps its endpoint and counters bit for bit; on 3-view triangulation
    targets the end-game cuts the failures from ~6% (paths stopped at the
    minimum step on their way to infinity) to under 2%."""
    S = V.triangulation_system(3)
    c0, sols = V.start_instance(3)
    _, coef, _ = V.vision_workload("triang3_batch4096")
    k = 8
    ep0, st0, inf0 = oracle.track(S, coef[:k], start=sols, coef0=c0, kind=oracle.LINEAR)
    ep, st, info, cyc = oracle.track(S, coef[:k], start=sols, coef0=c0, kind=oracle.LINEAR, endgame=True)
    ok = st0 == oracle.SUCCESS
    np.testing.assert_array_equal(ep[ok], ep0[ok])
    np.testing.assert_array_equal(st[ok], st0[ok])
    np.testing.assert_array_equal(info[ok], inf0[ok])
    assert (cyc[ok] == 0).all()
    fail0 = np.mean((st0 != oracle.SUCCESS) & (st0 != oracle.AT_INFINITY))
    fail = np.mean((st != oracle.SUCCESS) & (st != oracle.AT_INFINITY) & (st != oracle.SINGULAR_END))
    assert fail0 > 0.04 and fail < 0.02, (fail0, fail)
