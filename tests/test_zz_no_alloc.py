"""hc_track_device_noalloc (the fixed-workspace twin of hc_track_device) on the
GPU, through the C ABI: on the same inputs and launch configuration its
endpoints, statuses and counters equal hc_track_device's bit for bit.  Two
calls in a row share the device's fixed workspace, the second on a smaller
input (fewer instances and paths, another system), so leftovers of the first
must not leak into it; a call larger than the workspace is refused."""
import numpy as np
import pytest

import hc_inputs
import hc_inputs.vision as V

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


def _buffers(torch, n_inst, n_start, n):
    dev = torch.device("cuda:0")
    return (torch.full((n_inst, n_start, n), complex(float("nan"), 0.0), dtype=torch.complex128, device=dev),
            torch.full((n_inst, n_start), -7, dtype=torch.int32, device=dev),
            torch.zeros((n_inst, n_start, 32), dtype=torch.uint8, device=dev))


def _run_both(ctx, torch, sysh, p, g, n_inst, n_start, n, opts, start=None, p_start=None):
    """The same call through hc_track_device and hc_track_device_noalloc."""
    out = []
    for noalloc in (False, True):
        ep, st, info = _buffers(torch, n_inst, n_start, n)
        ctx.track_device(sysh, p, g, ep, st, info, start=start, p_start=p_start, n_start=n_start, opts=opts,
                         noalloc=noalloc)
        torch.cuda.synchronize()
        out.append((ep.cpu().numpy(), st.cpu().numpy(), info.cpu().numpy()))
    return out


def _assert_same(a, b):
    np.testing.assert_array_equal(a[0].view(np.float64), b[0].view(np.float64))
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_noalloc_equals_track_device_two_calls(hc, ctx, precision):
    import torch
    dev = torch.device("cuda:0")
    opts = hc.default_opts(precision=precision)
    # call 1: dense n = 8, 64 systems x 256 total-degree paths
    S, coef, gam = hc_inputs.dense_quadratic_instances(8, 64, seed=8100)
    sysh = ctx.load_system(S)
    p, g = torch.from_numpy(coef).to(dev), torch.from_numpy(gam).to(dev)
    ref, got = _run_both(ctx, torch, sysh, p, g, 64, 256, 8, opts)
    assert np.mean(ref[1] == hc.HC_T_SUCCESS) > 0.95
    _assert_same(ref, got)
    # call 2, smaller: 4-view triangulation (term lists, parameter homotopy),
    # 6 instances x 296 paths, in the workspace the first call left behind
    T = V.triangulation_system(4)
    c0, sols = V.start_instance(4)
    _, tcoef, _ = V.triangulation_instances(6, seed=8101)
    tsys = ctx.load_system(T, kind=hc.HC_PARAMETER)
    ref2, got2 = _run_both(ctx, torch, tsys, torch.from_numpy(tcoef).to(dev), None, 6, len(sols), T.n, opts,
                           start=torch.from_numpy(sols).to(dev), p_start=torch.from_numpy(c0).to(dev))
    assert np.mean(ref2[1] == hc.HC_T_SUCCESS) > 0.9
    _assert_same(ref2, got2)
    # and the small dense call again after the triangulation one
    ref3, got3 = _run_both(ctx, torch, sysh, p[:3], g[:3], 3, 100, 8, opts)
    _assert_same(ref3, got3)
    ctx.free_system(tsys)
    ctx.free_system(sysh)


def test_noalloc_refuses_oversized_call(hc, ctx):
    """A call whose workspace exceeds the fixed array is an error (raised on
    the host before any launch), and the context stays usable."""
    import torch
    dev = torch.device("cuda:0")
    S, coef, gam = hc_inputs.dense_quadratic_instances(8, 1, seed=8102)
    sysh = ctx.load_system(S)
    n_inst = hc.HC_NOALLOC_SCRATCH_BYTES // (256 * (16 * 8 + 40)) + 1
    p = torch.from_numpy(np.repeat(coef, n_inst, axis=0)).to(dev)
    g = torch.from_numpy(np.repeat(gam, n_inst)).to(dev)
    ep, st, info = _buffers(torch, n_inst, 256, 8)
    with pytest.raises(hc.HcError) as e:
        ctx.track_device(sysh, p, g, ep, st, info, noalloc=True)
    assert "workspace" in str(e.value)
    assert int(st[0, 0]) == -7
    ref, got = _run_both(ctx, torch, sysh, p[:2], g[:2], 2, 256, 8, hc.default_opts(precision="mixed"))
    _assert_same(ref, got)
    ctx.free_system(sysh)
