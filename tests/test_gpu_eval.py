"""Batched FP32 evaluation of dense quadratic systems and their Jacobians
(hc_eval_dense_device), both engines -- one Jacobian row per lane on the vector
ALUs and the matrix-core contraction -- against the FP64 oracle's evaluation.

Bar: every entry of F and J within 8 (n + 2) u sum |c| |m(x)| of the oracle's
value at the same (FP32-rounded) point, u = 2^-24, the sum taken over the
entry's terms (coefficient times monomial, or its derivative) in absolute value
-- the textbook bound of a sum of that many rounded products, widened for the
complex arithmetic and the rounding of the coefficients to FP32.  The sum is
the oracle's own evaluation of the system with |c| at |x|.
"""
import numpy as np
import pytest

import hc_inputs
import oracle

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def hc():
    import paper_2112_03444_amd as hc
    return hc


@pytest.fixture(scope="module")
def ctx(hc):
    c = hc.Context(0)
    yield c
    c.close()


def points(rng, n_inst, n_pts, n):
    x = rng.standard_normal((n_inst, n_pts, n, 2)).astype(np.float32)
    return (x[..., 0] + 1j * x[..., 1]).astype(np.complex64)


def run(hc, ctx, S, coef, x, engine, repeat=1):
    import torch
    sysh = ctx.load_system(S, layout=hc.HC_LAYOUT_DENSE)
    p = torch.from_numpy(coef).cuda()
    xd = torch.from_numpy(x).cuda()
    F, J = ctx.eval_dense_device(sysh, p, xd, engine=engine, repeat=repeat)
    torch.cuda.synchronize()
    return F.cpu().numpy(), J.cpu().numpy()


def check(S, coef, x, F, J, idx):
    """idx: (instance, point) pairs to compare."""
    n = S.n
    worst = 0.0
    for i, p in idx:
        xo = x[i, p].astype(np.complex128)
        Fo, Jo = oracle.eval_system(S, coef[i], xo)
        Fa, Ja = oracle.eval_system(S, np.abs(coef[i]), np.abs(xo))
        bound = 8 * (n + 2) * U32
        eF = np.abs(F[i, p] - Fo) / np.maximum(Fa, 1e-30)
        eJ = np.abs(J[i, p] - Jo) / np.maximum(Ja, 1e-30)
        e = max(eF.max(), eJ.max()) / bound
        assert e <= 1.0, (i, p, eF.max(), eJ.max(), bound)
        worst = max(worst, e)
    return worst


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 8])
def test_each_n_against_oracle(hc, ctx, n, engine):
    """3 instances x 100 points: several tiles of 16 (matrix cores) and groups of
    32 points (rows), with a ragged tail in both."""
    S, coef, _ = hc_inputs.dense_quadratic_instances(n, 3, seed=4100 + n)
    x = points(np.random.default_rng(n), 3, 100, n)
    F, J = run(hc, ctx, S, coef, x, engine)
    check(S, coef, x, F, J, [(i, p) for i in range(3) for p in range(100)])


@pytest.mark.parametrize("engine", [0, 1])
def test_repeat_gives_one_evaluation(hc, ctx, engine):
    S, coef, _ = hc_inputs.dense_quadratic_instances(8, 2, seed=4200)
    x = points(np.random.default_rng(7), 2, 70, 8)
    F1, J1 = run(hc, ctx, S, coef, x, engine, repeat=1)
    F3, J3 = run(hc, ctx, S, coef, x, engine, repeat=3)
    assert np.array_equal(F1, F3) and np.array_equal(J1, J3)


def test_engines_agree_on_the_dense_batch(hc, ctx):
    """The dense n = 8 batch of 512 instances at 256 points each (the tracking
    batch's shape): both engines within the bar of the oracle on 600 sampled
    points, and within twice the bar of each other everywhere."""
    S, coef, _ = hc_inputs.workload("dense8_batch512")
    x = points(np.random.default_rng(11), 512, 256, 8)
    F0, J0 = run(hc, ctx, S, coef, x, 0)
    F1, J1 = run(hc, ctx, S, coef, x, 1)
    rng = np.random.default_rng(3)
    idx = list(zip(rng.integers(0, 512, 300), rng.integers(0, 256, 300)))
    idx += [(511, 255), (0, 0), (255, 128)]
    check(S, coef, x, F0, J0, idx)
    check(S, coef, x, F1, J1, idx)
    scale = np.maximum(np.abs(J0), 1.0)
    assert np.max(np.abs(J0 - J1) / scale) <= 1e-4
    assert np.max(np.abs(F0 - F1) / np.maximum(np.abs(F0), 1.0)) <= 1e-4


def test_empty_and_errors(hc, ctx):
    import torch
    S, coef, _ = hc_inputs.dense_quadratic_instances(3, 2, seed=4300)
    sysh = ctx.load_system(S, layout=hc.HC_LAYOUT_DENSE)
    p = torch.from_numpy(coef).cuda()
    x0 = torch.zeros((2, 0, 3), dtype=torch.complex64, device="cuda")
    F, J = ctx.eval_dense_device(sysh, p, x0, engine=1)
    assert F.shape == (2, 0, 3) and J.shape == (2, 0, 3, 3)
    x = torch.zeros((2, 5, 3), dtype=torch.complex64, device="cuda")
    with pytest.raises(hc.HcError):
        ctx.eval_dense_device(sysh, p, x, engine=2)
    with pytest.raises(hc.HcError):
        ctx.eval_dense_device(sysh, p, x, repeat=0)
    tl = ctx.load_system(S, layout=hc.HC_LAYOUT_TERMS)
    with pytest.raises(hc.HcError):
        ctx.eval_dense_device(tl, p, x)
