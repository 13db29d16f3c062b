"""CPU-side checks of the C-ABI library: it loads, exports every declared entry
point, and its host-only logic (default options, section-6 term tables) is right.
No GPU compute is called here."""
import ctypes
import json
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hc.h")


@pytest.fixture(scope="module")
def hc():
    import paper_2112_03444_amd as hc
    if not os.path.exists(hc.hc.LIB_PATH):
        pytest.skip("libhc.so not built (run __graft_entry__.build())")
    return hc


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(hc):
    names = declared_functions()
    assert "hc_track" in names and "hc_load_system" in names and "hc_track_device" in names
    out = subprocess.check_output(["nm", "-D", "--defined-only", hc.hc.LIB_PATH], text=True)
    exported = set(re.findall(r"\bT (hc_[a-z_0-9]+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(hc.hc.LIB_PATH)
    for n in names:
        assert getattr(L, n) is not None


def test_struct_layouts_match_header(hc, tmp_path):
    """The binding's ctypes structures have the C compiler's sizes and field
    offsets for the header's structs."""
    structs = {"hc_opts": hc.Opts, "hc_system_desc": hc.hc.SystemDesc, "hc_job": hc.hc.Job,
               "hc_profile": hc.hc.Profile, "hc_request": hc.hc.Request, "hc_server_opts": hc.hc.ServerOpts,
               "hc_server_stats": hc.hc.ServerStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hc.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = {}
    for line in subprocess.check_output([str(exe)], text=True).splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
    assert hc.INFO_DTYPE.itemsize == 32


def test_default_opts(hc):
    o = hc.default_opts()
    assert (o.h0, o.h_min, o.h_max, o.beta_inc, o.beta_dec) == (0.05, 1e-7, 0.1, 2.0, 0.5)
    assert (o.tau64, o.tau32, o.pred_tol, o.tau_refine) == (1e-6, 3e-4, 1e-2, 1e-14)
    assert (o.inf_bound, o.eta_max, o.t_end) == (1e7, 1e-10, 0.0)
    assert (o.n_inc, o.max_newton, o.max_steps, o.max_refine) == (5, 3, 5000, 10)
    assert o.precision == hc.HC_FP64 and o.steps_per_launch == 0 and o.fp64_residual == 0
    assert o.crossing_check == 1


def test_paper_term_table_example(hc):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_term_tables.json")))
    ents = [[(s, a - 1, e) for (s, a, e) in g["entries"][k]["terms"]] for k in ("A", "B")]
    out = hc.homogenize(g["n"], ents, g["K"], g["M"])
    for k, tab in zip(("A", "B"), out):
        want = np.array(g["entries"][k]["table_1based"])
        got = tab.copy()
        got[:, 1:] += 1  # 0-based -> the paper's 1-based indices
        np.testing.assert_array_equal(got, want)


def test_homogenize_rejects_bad_input(hc):
    with pytest.raises(hc.HcError):
        hc.homogenize(2, [[(1, 0, [2, 1])]], 1, 2)  # degree 3 > M
    with pytest.raises(hc.HcError):
        hc.homogenize(2, [[(1, 0, [1, 0]), (1, 1, [0, 1])]], 1, 2)  # 2 terms > K


def test_homogenize_cubic_and_padding(hc):
    out = hc.homogenize(3, [[(3, 7, [1, 0, 2])], []], 2, 4)
    np.testing.assert_array_equal(out[0, 0], [3, 7, 0, 2, 2, 3])  # x1 x3 x3 + aux
    np.testing.assert_array_equal(out[0, 1], [0, 0, 0, 0, 0, 0])
    np.testing.assert_array_equal(out[1], np.zeros((2, 6)))
