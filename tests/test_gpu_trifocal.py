"""Per-instance start systems and the trifocal-pose workload (section 4: three
views, shared unknown focal length, 18 x 18, terms of degree <= 5) on the GPU,
through the C ABI, against the CPU oracle.

The trifocal coefficients are products of the 24 image coordinates, so each
solve follows a two-leg path in parameter space: view 1's coordinates move
first, then those of views 2 and 3; on each leg every coefficient is affine in
t, so the linear coefficient homotopy of that leg stays inside the family.
Both sides follow the same legs.  Bar: equal finite-solution counts and a
one-to-one match within 1e-9 relative error, residual <= 1e-10 after the FP64
refinement.  Noisy scenes have some badly conditioned roots, which two correct
FP64 computations cannot bring within 1e-9 of each other: such a root's bar is
its first-order forward-error bound times slack_factor (derived from the
evaluation's rounding) instead; they are counted and reported, and stay under
5% of an instance's roots (check_parity_conditioned).
"""
import hashlib
import os
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


def slack_factor(S):
    """Factor on the first-order forward-error bound of an FP64 root for the
    distance of two correct FP64 computations of it.  Each evaluates F_i with a
    rounding error below k u sum_k |c_ik||m_k(x)|, k = 2 sqrt(2) (d + 1) + T_i for
    terms of degree <= d in T_i terms (complex products: 2 sqrt(2) u each, d of
    them per term with the coefficient; T_i - 1 complex additions); the inverse
    Jacobian carries that into x, and the two errors can add up."""
    d = int(np.asarray(S.term_exp).sum(axis=1).max())
    T = int(np.bincount(np.asarray(S.term_eq)).max())
    return 2.0 * (2.0 * np.sqrt(2.0) * (d + 1) + T)


TAU_REFINE = 1e-14  # the refinement's stop test: what is left after the last Newton step


def check_parity_conditioned(ep_g, st_g, ep_o, st_o, fe_o, slack, hc, rel=REL):
    """Equal finite counts, and the nearest GPU root of every oracle root (a k-d
    tree in the real and imaginary parts, max-norm) is a one-to-one pairing
    within max(rel, slack x that root's forward-error bound + 2 tau_refine):
    well-conditioned roots keep rel; badly conditioned ones (near-degenerate
    scenes) cannot agree to rel between two correct FP64 refinements.  Returns
    (roots past rel, worst distance / own bound)."""
    from scipy.spatial import cKDTree
    fg = ep_g[st_g == hc.HC_T_SUCCESS]
    ok = st_o == oracle.SUCCESS
    fo, fe = ep_o[ok], fe_o[ok]
    assert len(fg) == len(fo), (np.bincount(st_g, minlength=8), np.bincount(st_o, minlength=8))
    if len(fo) == 0:
        return 0, 0.0
    emb = lambda z: np.concatenate([z.real, z.imag], axis=1)  # noqa: E731
    _, j = cKDTree(emb(fg)).query(emb(fo), k=1, p=np.inf)
    assert len(np.unique(j)) == len(j), "nearest-root pairing is not one-to-one"
    d = np.max(np.abs(fg[j] - fo), axis=1) / np.maximum(1.0, np.max(np.abs(fo), axis=1))
    tol = np.maximum(rel, slack * fe + 2 * TAU_REFINE)
    bad = np.flatnonzero(d > tol)
    assert len(bad) == 0, [(int(k), float(d[k]), float(tol[k])) for k in bad[:5]]
    wide = d > rel
    return int(wide.sum()), float(np.max(d / np.maximum(slack * fe + 2 * TAU_REFINE, 1e-300)))


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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trifocal_oracle_sample.npz")


@pytest.fixture(scope="module")
def batch(trifocal):
    """The trifocal_batch1024 workload's waypoint coefficients and the oracle's
    two-leg endpoints of sampled instances (tests/golden/trifocal_oracle_sample.npz,
    written by tests/golden/make_trifocal_oracle_sample.py from the stored start
    set; the oracle needs about a minute per instance)."""
    S, p0, sols, ps = trifocal
    z = np.load(GOLDEN)
    sha = np.frombuffer(hashlib.sha256(sols.tobytes()).digest(), np.uint8)
    assert int(z["n_start"]) == len(sols) and np.array_equal(z["sols_sha"], sha), \
        "trifocal_oracle_sample.npz is stale: rerun tests/golden/make_trifocal_oracle_sample.py"
    _, _, sc = TF.trifocal_workload("trifocal_batch1024")
    c0, mids, ends = two_leg_coefficients(p0, sc["pts"])
    return c0, mids, ends, [int(i) for i in z["instances"]], z["endpoints"], z["status"], z["fe_bound"]


def report(label, n_wide, ratio, n_fin):
    progress(f"{label}: {n_fin} finite roots, {n_wide} past 1e-9 (within slack x forward-error bound), "
             f"worst distance / bound {ratio:.3g}")


def test_trifocal_full_batch_mixed(hc, ctx, trifocal, batch):
    """The 1024-instance batch in mixed precision on device buffers, as the
    benchmark runs it: every finite endpoint's residual, and the sampled
    instances against the oracle.  Roots past 1e-9 (badly conditioned ones) are
    reported and stay under 5% of each instance's finite roots."""
    import torch
    S, p0, sols, ps = trifocal
    c0, mids, ends, sample, oe, os_, fe = batch
    dev = torch.device("cuda:0")
    n_inst, N = len(ends), len(sols)
    wp = [torch.from_numpy(c0).to(dev), torch.from_numpy(mids).to(dev), torch.from_numpy(ends).to(dev)]
    ep = torch.empty((n_inst, N, 18), dtype=torch.complex128, device=dev)
    st = torch.empty((n_inst, N), dtype=torch.int32, device=dev)
    inf = torch.empty((n_inst, N, 32), dtype=torch.uint8, device=dev)
    progress(f"trifocal: mixed precision, {n_inst} instances x {N} paths, two legs")
    ctx.track_piecewise_device(ps, wp, torch.from_numpy(sols).to(dev), ep, st, inf,
                               opts=hc.default_opts(precision="mixed"))
    torch.cuda.synchronize()
    ep, st = ep.cpu().numpy(), st.cpu().numpy()
    info = inf.cpu().numpy().view(hc.INFO_DTYPE)[..., 0]
    ok = st == hc.HC_T_SUCCESS
    assert np.all(info["residual"][ok] <= 1e-10)
    assert ok.sum(axis=1).min() >= 0.5 * N
    slack = slack_factor(S)
    for k, i in enumerate(sample):
        n_wide, ratio = check_parity_conditioned(ep[i], st[i], oe[k], os_[k], fe[k], slack, hc)
        n_fin = int(np.sum(os_[k] == oracle.SUCCESS))
        report(f"trifocal mixed, instance {i}", n_wide, ratio, n_fin)
        assert n_wide <= 0.05 * n_fin


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_trifocal_sampled_instances_host_buffers(hc, ctx, trifocal, batch, precision):
    """The sampled instances alone through the host-buffer entry point, in both
    precisions, against the same oracle endpoints."""
    S, p0, sols, ps = trifocal
    c0, mids, ends, sample, oe, os_, fe = batch
    ep, st, info = ctx.track_piecewise(ps, [c0, mids[sample], ends[sample]], sols,
                                       opts=hc.default_opts(precision=precision))
    slack = slack_factor(S)
    for k, i in enumerate(sample):
        n_wide, ratio = check_parity_conditioned(ep[k], st[k], oe[k], os_[k], fe[k], slack, hc)
        n_fin = int(np.sum(os_[k] == oracle.SUCCESS))
        report(f"trifocal {precision} (host buffers), instance {i}", n_wide, ratio, n_fin)
        assert n_wide <= 0.05 * n_fin
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)
