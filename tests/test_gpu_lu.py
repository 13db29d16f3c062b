"""The standalone batched complex solver (section 6, "Linear System Solver":
LU with partial pivoting of the augmented matrix [A | b] in one fused kernel,
back substitution with the cached U) on the GPU, through the C ABI, against the
oracle's LU solve (itself pinned to LAPACK zgesv).

Bars, per system: the normwise backward error ||A x - b|| / (||A||_F ||x|| +
||b||) (Higham, Accuracy and Stability, ch. 9) at most 8 n u, u the unit
roundoff of the precision; and the forward difference to the oracle's x at most
8 n kappa(A) u relative (the first-order bound of two backward-stable solves).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

U = {True: 2.0 ** -24, False: 2.0 ** -53}


@pytest.fixture(scope="module")
def hc():
    import paper_2112_03444_amd as hc
    return hc


@pytest.fixture(scope="module")
def ctx(hc):
    c = hc.Context(0)
    yield c
    c.close()


def cn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)


def solve_gpu(ctx, A, b, fp32):
    import torch
    dt = torch.complex64 if fp32 else torch.complex128
    dev = torch.device("cuda:0")
    At = torch.from_numpy(A).to(dev, dt).contiguous()
    bt = torch.from_numpy(b).to(dev, dt).contiguous()
    xt = torch.empty_like(bt)
    info = torch.full((A.shape[0],), -1, dtype=torch.int32, device=dev)
    ctx.solve_batched_device(At, bt, xt, info)
    torch.cuda.synchronize()
    # the data the GPU solved (rounded to its precision), in FP64
    return xt.cpu().numpy().astype(np.complex128), info.cpu().numpy(), \
        At.cpu().numpy().astype(np.complex128), bt.cpu().numpy().astype(np.complex128)


def check(A, b, x, fp32, sample=None, kappa_max=None):
    n = A.shape[1]
    u = U[fp32]
    r = np.einsum("kij,kj->ki", A, x) - b
    # Frobenius norm of A (>= the 2-norm: a slightly weaker bound, cheap for 2^20 systems)
    bwd = np.linalg.norm(r, axis=1) / (np.linalg.norm(A.reshape(len(A), -1), axis=1) * np.linalg.norm(x, axis=1)
                                       + np.linalg.norm(b, axis=1))
    assert np.all(bwd <= 8 * n * u), bwd.max()
    idx = range(len(A)) if sample is None else sample
    for k in idx:
        xo = oracle.lu_solve(A[k], b[k])
        assert xo is not None
        kappa = np.linalg.cond(A[k])
        rel = np.max(np.abs(x[k] - xo)) / max(np.max(np.abs(xo)), 1e-300)
        assert rel <= 8 * n * kappa * u, (k, rel, kappa)


@pytest.mark.parametrize("fp32", [True, False])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 13, 16, 17, 20, 31, 32])
def test_random_systems_against_oracle(hc, ctx, n, fp32):
    rng = np.random.default_rng(9000 + n)
    batch = 203  # ragged against every group count per block
    A = cn(rng, batch, n, n)
    b = cn(rng, batch, n)
    x, info, Ag, bg = solve_gpu(ctx, A, b, fp32)
    assert np.all(info == 0)
    check(Ag, bg, x, fp32, sample=range(0, batch, 7))


@pytest.mark.parametrize("fp32", [True, False])
def test_pivoting_is_needed(hc, ctx, fp32):
    """Zero diagonals and a graded first column: without row exchanges the
    elimination would divide by zero or lose all accuracy."""
    rng = np.random.default_rng(9100)
    n, batch = 12, 64
    A = cn(rng, batch, n, n)
    A[:, np.arange(n), np.arange(n)] = 0.0
    A[: batch // 2, :, 0] *= 10.0 ** np.arange(n)[None, :] / 1e6
    b = cn(rng, batch, n)
    x, info, Ag, bg = solve_gpu(ctx, A, b, fp32)
    assert np.all(info == 0)
    check(Ag, bg, x, fp32, sample=range(batch))


@pytest.mark.parametrize("fp32", [True, False])
def test_singular_systems_are_flagged(hc, ctx, fp32):
    rng = np.random.default_rng(9200)
    n, batch = 6, 10
    A = cn(rng, batch, n, n)
    A[3, :, 2] = 0.0            # a zero column
    A[7, 4, :] = 0.0            # a zero row
    b = cn(rng, batch, n)
    x, info, Ag, bg = solve_gpu(ctx, A, b, fp32)
    assert info.tolist() == [0, 0, 0, 1, 0, 0, 0, 1, 0, 0]
    ok = info == 0
    check(Ag[ok], bg[ok], x[ok], fp32)


def test_identity_and_exact_integer_solution(hc, ctx):
    """A = I gives x = b bit for bit; an integer upper-triangular system with
    unit diagonal is solved exactly in FP64."""
    import torch
    n, batch = 9, 5
    A = np.broadcast_to(np.eye(n, dtype=np.complex128), (batch, n, n)).copy()
    b = np.arange(batch * n, dtype=np.float64).reshape(batch, n) + 1j
    x, info, _, _ = solve_gpu(ctx, A, b, False)
    assert np.array_equal(x, b) and np.all(info == 0)
    T = np.triu(np.ones((n, n))) + 0j
    xs = np.arange(1, n + 1) + 0j
    x, info, _, _ = solve_gpu(ctx, T[None], (T @ xs)[None], False)
    assert np.array_equal(x[0], xs)


def test_empty_batch_and_argument_errors(hc, ctx):
    import torch
    dev = torch.device("cuda:0")
    A = torch.zeros((0, 4, 4), dtype=torch.complex64, device=dev)
    b = torch.zeros((0, 4), dtype=torch.complex64, device=dev)
    ctx.solve_batched_device(A, b, torch.empty_like(b))  # no-op
    for n in (33,):
        A = torch.zeros((2, n, n), dtype=torch.complex64, device=dev)
        b = torch.zeros((2, n), dtype=torch.complex64, device=dev)
        with pytest.raises(hc.HcError):
            ctx.solve_batched_device(A, b, torch.empty_like(b))
    with pytest.raises(ValueError):
        ctx.solve_batched_device(torch.zeros((2, 4, 4), dtype=torch.complex64, device=dev),
                                 torch.zeros((2, 4), dtype=torch.complex128, device=dev),
                                 torch.zeros((2, 4), dtype=torch.complex64, device=dev))


def test_large_batch_sampled(hc, ctx):
    """2^20 systems of n = 8 in FP32 (one launch of 16384 blocks): backward
    error of every system, sampled systems against the oracle."""
    rng = np.random.default_rng(9300)
    n, batch = 8, 1 << 20
    A = cn(rng, batch, n, n).astype(np.complex64)
    b = cn(rng, batch, n).astype(np.complex64)
    x, info, Ag, bg = solve_gpu(ctx, A, b, True)
    assert np.all(info == 0)
    check(Ag, bg, x, True, sample=[0, 1, 12345, batch // 2, batch - 1])
