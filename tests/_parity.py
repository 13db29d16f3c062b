"""Set-level parity helpers shared by the GPU tests.

Per instance the GPU's finite solutions (status SUCCESS) and the oracle's must
be equal in number and pair up one to one: every oracle root is matched to a
distinct GPU root within the relative bar (max-norm distance over max(1, |x|)).
A duplicated GPU root plus a missed one fails, since the pairing must be a
bijection.
"""
import numpy as np

import oracle

REL = 1e-9


def rel_dist(x, y):
    """Relative max-norm distance of the rows of x to the row y."""
    return np.max(np.abs(x - y), axis=-1) / max(1.0, float(np.max(np.abs(y))))


def match_one_to_one(fg, fo):
    """Worst distance of a one-to-one pairing of the rows of fg and fo: the
    oracle roots are taken in turn, each paired with the nearest GPU root not
    yet taken.  inf if the counts differ."""
    if len(fg) != len(fo):
        return np.inf
    free = np.ones(len(fg), bool)
    worst = 0.0
    for y in fo:
        d = np.where(free, rel_dist(fg, y), np.inf)
        j = int(np.argmin(d))
        worst = max(worst, float(d[j]))
        free[j] = False
    return worst


def check_sets(ep_g, st_g, ep_o, st_o, success_gpu, rel=REL):
    """Equal finite counts and a one-to-one match within rel; returns the worst
    distance."""
    fg = ep_g[st_g == success_gpu]
    fo = ep_o[st_o == oracle.SUCCESS]
    assert len(fg) == len(fo), (np.bincount(st_g, minlength=7), np.bincount(st_o, minlength=7))
    w = match_one_to_one(fg, fo)
    assert w <= rel, w
    return w
