"""Parity of the general-degree term-list kernels (terms of degree up to 8,
n <= 16 with 16 lanes per path, n <= 20 and n <= 32 with 32) with the CPU
oracle, on the GPU, through the C ABI.

Systems are dense on chosen supports (equation i: every monomial of degree
<= d_i in the unknowns V_i, CN(0, 1) coefficients), so the total-degree
homotopy (start system x_i^d_i - 1, section 3) has prod d_i paths, all ending
at finite roots.  Bar as in test_gpu_parity: the same number of finite
solutions as the oracle and a one-to-one match within 1e-9 relative error; in
mixed mode every finite endpoint also has residual <= 1e-10 after the FP64
refinement.
"""
import numpy as np
import pytest

import hc_inputs
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
    """Greedy one-to-one nearest matching; worst relative distance (inf if the
    sizes differ)."""
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


def linear_rows(n, count):
    return [(1, list(range(n)))] * count


# (n, spec): kinds 1 (any degree, n <= 16), 4 (n 17..18), 2 (n 19..20) and 6
# (n 21..32: the paper's largest Jacobian is 32 x 32, section 1), and the
# quadratic kind 0 (n 15..16)
SPECS = {
    "cubic3": (3, [(3, [0, 1, 2])] * 3),
    "deg54": (2, [(5, [0, 1]), (4, [0, 1])]),
    "deg8": (2, [(8, [0]), (1, [0, 1])]),
    "mixed5": (5, [(3, [0, 1, 2, 3, 4]), (2, [0, 1, 2, 3, 4]), (2, [1, 2, 3]), (1, [0, 1, 2, 3, 4]),
                   (1, [0, 2, 4])]),
    "deg5_n18": (18, [(5, [0, 1]), (3, [0, 1, 2])] + linear_rows(18, 16)),
    "cubic_n20": (20, [(3, [0, 1, 2]), (2, [0, 1, 2, 3])] + linear_rows(20, 18)),
    "quad_n17": (17, [(2, [0, 1, 2]), (2, [0, 1, 2])] + linear_rows(17, 15)),
    "quad_n15": (15, [(2, [0, 1, 2, 3]), (2, [0, 1, 2])] + linear_rows(15, 13)),
    "cubic_n24": (24, [(3, [0, 1, 2]), (2, [0, 1, 2, 3])] + linear_rows(24, 22)),
    "deg4_n32": (32, [(4, [0, 1]), (2, [0, 1, 2])] + linear_rows(32, 30)),
    "quad_n32": (32, [(2, [0, 1, 2, 3])] * 4 + linear_rows(32, 28)),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(SPECS))
def test_total_degree_general(hc, ctx, name, precision):
    n, spec = SPECS[name]
    S, coef, gam = hc_inputs.support_instances(n, spec, 2, seed=6000 + len(name) * 7 + n)
    sysh = ctx.load_system(S)
    assert sysh.bezout == int(np.prod([d for d, _ in spec]))
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision=precision))
    oep, ost, _ = oracle.track(S, coef, gam)
    for i in range(2):
        check_parity(ep[i], st[i], oep[i], ost[i], hc)
    ok = st == hc.HC_T_SUCCESS
    assert ok.mean() >= 0.9
    assert np.all(info["residual"][ok] <= 1e-10)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["mixed5", "deg5_n18", "deg4_n32"])
def test_parameter_homotopy_general(hc, ctx, name, precision):
    """Linear coefficient homotopy between two instances of one support: start
    points are the oracle's roots of instance 0 (section 3, parameter
    homotopy)."""
    n, spec = SPECS[name]
    S, coef, gam = hc_inputs.support_instances(n, spec, 4, seed=6100 + n)
    e0, s0, _ = oracle.track(S, coef[:1], gam[:1])
    start = np.ascontiguousarray(e0[0][s0[0] == oracle.SUCCESS])
    ps = ctx.load_system(S, kind=hc.HC_PARAMETER)
    ep, st, info = ctx.track(ps, coef[1:], start=start, p_start=coef[0], opts=hc.default_opts(precision=precision))
    oep, ost, _ = oracle.track(S, coef[1:], start=start, coef0=coef[0], kind=oracle.LINEAR)
    for i in range(3):
        check_parity(ep[i], st[i], oep[i], ost[i], hc)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


@pytest.mark.parametrize("name", ["cubic3", "mixed5", "deg5_n18", "cubic_n24"])
def test_fp64_residual_general(hc, ctx, name):
    """Mixed mode with the FP64 Newton right-hand side (fp64_residual) on the
    general-degree kinds, total degree: the same root sets as the oracle."""
    n, spec = SPECS[name]
    S, coef, gam = hc_inputs.support_instances(n, spec, 2, seed=6600 + n)
    sysh = ctx.load_system(S)
    ep, st, info = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision="mixed", fp64_residual=1))
    oep, ost, _ = oracle.track(S, coef, gam)
    for i in range(2):
        check_parity(ep[i], st[i], oep[i], ost[i], hc)
    assert np.all(info["residual"][st == hc.HC_T_SUCCESS] <= 1e-10)


def test_start_points_of_any_degree(hc, ctx):
    """The device's total-degree start points (roots of unity, mixed radix over
    the equations) equal hc_total_degree_start's, so supplying them changes
    nothing."""
    n, spec = SPECS["deg54"]
    S, coef, gam = hc_inputs.support_instances(n, spec, 1, seed=6200)
    sysh = ctx.load_system(S)
    start = sysh.total_degree_start()
    assert start.shape == (20, 2)
    np.testing.assert_allclose(start[:, 0] ** 5, 1.0, atol=1e-14)
    np.testing.assert_allclose(start[:, 1] ** 4, 1.0, atol=1e-14)
    a = ctx.track(sysh, coef, gam)
    ps_a = a[0][0][a[1][0] == hc.HC_T_SUCCESS]
    b = ctx.track(sysh, coef, gam, start=start)
    ps_b = b[0][0][b[1][0] == hc.HC_T_SUCCESS]
    assert rel_match(ps_a, ps_b) <= 1e-12


def test_batch_with_every_kind_equals_single_calls(hc, ctx):
    """One batch over dense, quadratic term-list and both general-degree kinds
    returns, job by job, what a call on that job alone returns."""
    import torch
    dev = torch.device("cuda:0")
    opts = hc.default_opts(precision="mixed")
    systems = [hc_inputs.dense_quadratic_instances(4, 2, seed=6300),
               hc_inputs.dense_quadratic_instances(10, 1, seed=6301),
               hc_inputs.support_instances(*SPECS["mixed5"], 3, seed=6302),
               hc_inputs.support_instances(*SPECS["deg5_n18"], 2, seed=6303),
               hc_inputs.support_instances(*SPECS["cubic3"], 2, seed=6304)]
    jobs, refs = [], []
    for S, coef, gam in systems:
        sysh = ctx.load_system(S)
        ns = sysh.bezout
        n_inst = coef.shape[0]
        p = torch.from_numpy(coef).to(dev)
        g = torch.from_numpy(gam).to(dev)
        ref = [torch.empty((n_inst, ns, S.n), dtype=torch.complex128, device=dev),
               torch.empty((n_inst, ns), dtype=torch.int32, device=dev),
               torch.empty((n_inst, ns, 32), dtype=torch.uint8, device=dev)]
        ctx.track_device(sysh, p, g, ref[0], ref[1], ref[2], n_start=ns, opts=opts)
        torch.cuda.synchronize()
        refs.append([r.cpu().numpy() for r in ref])
        jobs.append(dict(sys=sysh, p_target=p, gamma=g, n_start=ns, endpoints=torch.zeros_like(ref[0]),
                         status=torch.zeros_like(ref[1]), info=torch.zeros_like(ref[2])))
    ctx.track_batch_device(jobs, opts=opts)
    torch.cuda.synchronize()
    for j, r in zip(jobs, refs):
        np.testing.assert_array_equal(j["endpoints"].cpu().numpy(), r[0])
        np.testing.assert_array_equal(j["status"].cpu().numpy(), r[1])
        np.testing.assert_array_equal(j["info"].cpu().numpy(), r[2])


def test_chunked_launches_general(hc, ctx):
    n, spec = SPECS["deg5_n18"]
    S, coef, gam = hc_inputs.support_instances(n, spec, 2, seed=6400)
    sysh = ctx.load_system(S)
    a = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision="mixed"))
    b = ctx.track(sysh, coef, gam, opts=hc.default_opts(precision="mixed", steps_per_launch=5))
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[0], b[0])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_with_32_row_kind(hc, ctx, precision):
    """The batch tracker (one device queue over jobs of several term-list kinds)
    on jobs of the 32-row kind (n = 24 and 32) beside a g16 job: every job ends
    with the statuses of a call on it alone and the oracle's root sets.  The
    batch escalates inline, the single call of the 32-row kind in a second
    launch; both run the same FP64 stages, so the endpoints agree to rounding."""
    import torch
    dev = torch.device("cuda:0")
    opts = hc.default_opts(precision=precision)
    jobs, refs, oin = [], [], []
    for k, name in enumerate(["cubic_n24", "mixed5", "quad_n32"]):
        n, spec = SPECS[name]
        S, coef, gam = hc_inputs.support_instances(n, spec, 2, seed=6700 + k)
        sysh = ctx.load_system(S)
        ns = sysh.bezout
        p = torch.from_numpy(coef).to(dev)
        g = torch.from_numpy(gam).to(dev)
        ep = torch.empty((2, ns, n), dtype=torch.complex128, device=dev)
        st = torch.empty((2, ns), dtype=torch.int32, device=dev)
        ctx.track_device(sysh, p, g, ep, st, None, opts=opts)
        torch.cuda.synchronize()
        refs.append((ep.cpu().numpy(), st.cpu().numpy()))
        oin.append((S, coef, gam))
        jobs.append(dict(sys=sysh, p_target=p, gamma=g, n_start=ns, endpoints=torch.zeros_like(ep),
                         status=torch.zeros_like(st)))
    ctx.track_batch_device(jobs, opts=opts)
    torch.cuda.synchronize()
    for j, (rep, rst), (S, coef, gam) in zip(jobs, refs, oin):
        ep, st = j["endpoints"].cpu().numpy(), j["status"].cpu().numpy()
        np.testing.assert_array_equal(st, rst)
        ok = st == hc.HC_T_SUCCESS
        np.testing.assert_allclose(ep[ok], rep[ok], rtol=1e-12, atol=1e-12)
        oep, ost, _ = oracle.track(S, coef, gam)
        for i in range(2):
            check_parity(ep[i], st[i], oep[i], ost[i], hc)


def test_general_load_errors(hc, ctx):
    deg9 = hc_inputs.support_system(2, [(9, [0]), (1, [0, 1])])
    with pytest.raises(hc.HcError):
        ctx.load_system(deg9)  # a term of degree 9 > 8
    cubic = hc_inputs.support_system(3, [(3, [0, 1, 2])] * 3)
    with pytest.raises(hc.HcError):
        ctx.load_system(cubic, layout=hc.HC_LAYOUT_DENSE)  # dense tables: degree <= 2
    with pytest.raises(hc.HcError):
        ctx.load_system(hc_inputs.support_system(33, linear_rows(33, 33)))  # n > HC_MAX_N
    sysh = ctx.load_system(hc_inputs.support_system(*SPECS["deg5_n18"]))
    _, coef, gam = hc_inputs.support_instances(*SPECS["deg5_n18"], 1, seed=6500)
    with pytest.raises(hc.HcError):
        ctx.track(sysh, coef, gam, opts=hc.default_opts(lanes_per_path=16))  # n = 18 needs 32 lanes
