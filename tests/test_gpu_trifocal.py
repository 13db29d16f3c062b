"""Per-instance start systems and the trifocal-pose workload (section 4: three
views, shared unknown focal length, 18 x 18, terms of degree <= 5) on the GPU,
through the C ABI, against the CPU oracle.

The trifocal coefficients are products of the 24 image coordinates, so each
solve follows a two-leg path in parameter space: view 1's coordinates move
first, then those of views 2 and 3; on each leg every coefficient is affine in
t, so the linear coefficient homotopy of that leg stays inside the family.
Both sides follow the same legs.  Bar: equal finite-solution counts and a
one-to-one match within 1e-9 relative error, residual <= 1e-10 after the FP64
refinement.  Noisy scenes have some badly conditioned roots; where the first-
order forward-error bound of an FP64 root exceeds 1e-9 / 100 that root's bar
is 100 times its bound instead (check_parity_conditioned).
"""
import sys
import time

import numpy as np
import pytest

import hc_inputs
import hc_inputs.trifocal as TF
import oracle

pytestmark = pytest.mark.gpu

REL = 1e-9


@pytest.fixture(scope="module")
def hc():
    import paper_2112_03444_amd as hc
    return hc


@pytest.fixture(scope="module")
def ctx(hc):
    c = hc.Context(0)
    yield c
    c.close()


def rel_match(a, b):
    if len(a) != len(b):
        return np.inf
    b = list(b)
    worst = 0.0
    for p in a:
        d = [np.max(np.abs(p - q)) / max(1.0, np.max(np.abs(q))) for q in b]
        j = int(np.argmin(d))
        worst = max(worst, d[j])
        b.pop(j)
    return worst


def check_parity(ep_g, st_g, ep_o, st_o, hc, rel=REL):
    fg = ep_g[st_g == hc.HC_T_SUCCESS]
    fo = ep_o[st_o == oracle.SUCCESS]
    assert len(fg) == len(fo), (np.bincount(st_g, minlength=7), np.bincount(st_o, minlength=7))
    w = rel_match(fg, fo)
    assert w <= rel, w


U = 2.0 ** -53


def forward_error_bound(S, c1, c0, x):
    """First-order bound on the error of an FP64 root x of F(.; c1), relative to
    max(1, |x|_inf): ||J^-1||_2 u ||(sum_k |c_ik| |m_k(x)|)_i||_2 / max(1, |x|_inf)
    -- the rounding of F at x (within u times that sum per equation, up to the
    small constant of the evaluation) moved through the inverse Jacobian."""
    _, J, _ = oracle.homotopy_eval(S, x, 1.0, c1, coef0=c0, kind=oracle.LINEAR)
    inv = 1.0 / np.linalg.svd(J, compute_uv=False)[-1]
    m = np.prod(np.power(x[None, :], S.term_exp), axis=1)
    den = np.zeros(S.n)
    np.add.at(den, S.term_eq, np.abs(c1) * np.abs(m))
    return inv * U * np.linalg.norm(den) / max(1.0, np.max(np.abs(x)))


def check_parity_conditioned(ep_g, st_g, ep_o, st_o, S, c1, c0, hc, rel=REL, slack=100.0):
    """check_parity with each oracle root's own tolerance max(rel, slack x its
    forward-error bound): equal finite counts, and the nearest GPU root of every
    oracle root (a k-d tree in the real and imaginary parts, max-norm) is a
    one-to-one pairing within that tolerance.  For well-conditioned roots the
    bound is far below rel and the bar is rel; badly conditioned ones
    (near-degenerate scenes) cannot agree to rel between two correct FP64
    refinements."""
    from scipy.spatial import cKDTree
    fg = ep_g[st_g == hc.HC_T_SUCCESS]
    fo = ep_o[st_o == oracle.SUCCESS]
    assert len(fg) == len(fo), (np.bincount(st_g, minlength=7), np.bincount(st_o, minlength=7))
    if len(fo) == 0:
        return 0
    emb = lambda z: np.concatenate([z.real, z.imag], axis=1)  # noqa: E731
    _, j = cKDTree(emb(fg)).query(emb(fo), k=1, p=np.inf)
    assert len(np.unique(j)) == len(j), "nearest-root pairing is not one-to-one"
    d = np.max(np.abs(fg[j] - fo), axis=1) / np.maximum(1.0, np.max(np.abs(fo), axis=1))
    n_wide = 0
    for k in np.flatnonzero(d > rel):
        tol = slack * forward_error_bound(S, c1, c0, fo[k])
        n_wide += 1
        assert d[k] <= tol, (k, d[k], tol)
    return n_wide


def test_per_instance_start_equals_separate_calls(hc, ctx):
    """One call with a start system per instance returns, instance by instance,
    what a call on that instance with its own start system returns."""
    S, coef, gam = hc_inputs.dense_quadratic_instances(4, 6, seed=7000)
    td = ctx.load_system(S)
    ep0, st0, _ = ctx.track(td, coef[:3], gam[:3])  # three start instances with their roots
    ps = ctx.load_system(S, kind=hc.HC_PARAMETER)
    for precision in ("fp64", "mixed"):
        o = hc.default_opts(precision=precision)
        ep, st, info = ctx.track(ps, coef[3:], start=ep0, p_start=coef[:3], opts=o)
        for i in range(3):
            e1, s1, i1 = ctx.track(ps, coef[3 + i:4 + i], start=ep0[i], p_start=coef[i], opts=o)
            np.testing.assert_array_equal(ep[i], e1[0])
            np.testing.assert_array_equal(st[i], s1[0])
            np.testing.assert_array_equal(info[i], i1[0])


def test_per_instance_start_rejected_in_batch(hc, ctx):
    import torch
    S, coef, gam = hc_inputs.dense_quadratic_instances(3, 1, seed=7001)
    sysh = ctx.load_system(S)
    dev = torch.device("cuda:0")
    job = dict(sys=sysh, p_target=torch.from_numpy(coef).to(dev), gamma=torch.from_numpy(gam).to(dev),
               endpoints=torch.zeros((1, 8, 3), dtype=torch.complex128, device=dev),
               status=torch.zeros((1, 8), dtype=torch.int32, device=dev))
    o = hc.default_opts()
    o.per_instance_start = 1
    with pytest.raises(hc.HcError):
        ctx.track_batch_device([job], opts=o)


@pytest.fixture(scope="module")
def trifocal(hc, ctx):
    S = TF.trifocal_system()
    p0, sols = TF.start_instance()
    ps = ctx.load_system(S, kind=hc.HC_PARAMETER)
    return S, p0, sols, ps


def two_leg_coefficients(p0, pts):
    """Waypoint coefficients of the two-leg path from p0 to each target."""
    mids, ends = [], []
    for p1 in pts:
        w = TF.waypoints(p0, p1)
        mids.append(TF.coefficients(w[1]))
        ends.append(TF.coefficients(w[2]))
    return TF.coefficients(p0), np.stack(mids), np.stack(ends)


def progress(msg):
    """Progress of the long oracle runs, past pytest's capture."""
    print(msg, file=sys.__stderr__, flush=True)


def oracle_two_leg(S, c0, mids, ends, sols):
    """The oracle along the same legs: leg 1 for every instance from the shared
    start set, leg 2 per instance from its leg-1 roots."""
    t0 = time.time()
    progress(f"oracle: leg 1, {len(mids)} x {len(sols)} paths")
    e1, s1, _ = oracle.track(S, mids, start=sols, coef0=c0, kind=oracle.LINEAR)
    out_e, out_s = [], []
    for i in range(len(ends)):
        ok = e1[i][s1[i] == oracle.SUCCESS]
        progress(f"oracle: leg 2 of instance {i}, {len(ok)} paths ({time.time() - t0:.0f} s)")
        e2, s2, _ = oracle.track(S, ends[i:i + 1], start=ok, coef0=mids[i], kind=oracle.LINEAR)
        out_e.append(e2[0])
        out_s.append(s2[0])
    progress(f"oracle: done ({time.time() - t0:.0f} s)")
    return out_e, out_s


def test_trifocal_noise_free_ground_truth_on_gpu(hc, ctx, trifocal):
    """The planted pose of noise-free scenes, with its eight symmetry images, is
    among the GPU's endpoints."""
    S, p0, sols, ps = trifocal
    _, _, sc = TF.trifocal_instances(3, seed=7200, sigma=0.0)
    c0, mids, ends = two_leg_coefficients(p0, sc["pts"])
    ep, st, _ = ctx.track_piecewise(ps, [c0, mids, ends], sols, opts=hc.default_opts(precision="mixed"))
    for i in range(3):
        ok = ep[i][st[i] == hc.HC_T_SUCCESS]
        for x in TF.symmetry_orbit(sc["gt"][i]):
            assert np.max(np.abs(ok - x), axis=1).min() < 1e-8


SAMPLE = [0]  # the batch's most badly conditioned instance of those checked (a minute of oracle time)


@pytest.fixture(scope="module")
def batch(trifocal):
    """The trifocal_batch1024 workload's waypoint coefficients and the oracle's
    two-leg endpoints of the sampled instances (computed once)."""
    S, p0, sols, ps = trifocal
    _, _, sc = TF.trifocal_workload("trifocal_batch1024")
    c0, mids, ends = two_leg_coefficients(p0, sc["pts"])
    oe, os_ = oracle_two_leg(S, c0, mids[SAMPLE], ends[SAMPLE], sols)
    return c0, mids, ends, oe, os_


def test_trifocal_full_batch_sampled(hc, ctx, trifocal, batch):
    """The 1024-instance batch in FP64 on device buffers, as the benchmark runs
    it: every finite endpoint's residual, and the sampled instances against the
    oracle (mixed mode is checked on the sampled instances through the
    host-buffer entry point)."""
    import torch
    S, p0, sols, ps = trifocal
    c0, mids, ends, oe, os_ = batch
    dev = torch.device("cuda:0")
    n_inst, N = len(ends), len(sols)
    wp = [torch.from_numpy(c0).to(dev), torch.from_numpy(mids).to(dev), torch.from_numpy(ends).to(dev)]
    ep = torch.empty((n_inst, N, 18), dtype=torch.complex128, device=dev)
    st = torch.empty((n_inst, N), dtype=torch.int32, device=dev)
    inf = torch.empty((n_inst, N, 32), dtype=torch.uint8, device=dev)
    ctx.track_piecewise_device(ps, wp, torch.from_numpy(sols).to(dev), ep, st, inf,
                               opts=hc.default_opts(precision="fp64"))
    torch.cuda.synchronize()
    ep, st = ep.cpu().numpy(), st.cpu().numpy()
    info = inf.cpu().numpy().view(hc.INFO_DTYPE)[..., 0]
    ok = st == hc.HC_T_SUCCESS
    assert np.all(info["residual"][ok] <= 1e-10)
    assert ok.sum(axis=1).min() >= 0.5 * N
    for k, i in enumerate(SAMPLE):
        check_parity_conditioned(ep[i], st[i], oe[k], os_[k], S, ends[i], mids[i], hc)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_trifocal_sampled_instances_host_buffers(hc, ctx, trifocal, batch, precision):
    """The sampled instances alone through the host-buffer entry point, in both
    precisions, against the same oracle endpoints."""
    S, p0, sols, ps = trifocal
    c0, mids, ends, oe, os_ = batch
    ep, st, info = ctx.track_piecewise(ps, [c0, mids[SAMPLE], ends[SAMPLE]], sols,
                                       opts=hc.default_opts(precision=precision))
    for k, i in enumerate(SAMPLE):
        check_parity_conditioned(ep[k], st[k], oe[k], os_[k], S, ends[i], mids[i], hc)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)
