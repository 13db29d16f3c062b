"""The set-parity helper of the GPU tests, on the CPU: a one-to-one pairing
must reject a duplicated root that hides a missed one, even when the counts
agree and every root lies near some root of the other set."""
import numpy as np
import pytest

import _parity


def test_identical_and_permuted_sets_match():
    rng = np.random.default_rng(1)
    a = rng.standard_normal((8, 3)) + 1j * rng.standard_normal((8, 3))
    assert _parity.match_one_to_one(a, a) == 0.0
    assert _parity.match_one_to_one(a[::-1] * (1 + 1e-12), a) < 1e-11


def test_duplicate_plus_missed_root_fails():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((8, 3)) + 1j * rng.standard_normal((8, 3))
    b = a.copy()
    b[5] = b[4]                     # root 5 missed, root 4 found twice
    assert _parity.match_one_to_one(b, a) > 1e-3
    st = np.zeros(8, np.int32)
    with pytest.raises(AssertionError):
        _parity.check_sets(b, st, a, st, 0)


def test_count_mismatch_fails():
    a = np.ones((3, 2), complex)
    st_g = np.array([0, 0, 2], np.int32)
    st_o = np.zeros(3, np.int32)
    with pytest.raises(AssertionError):
        _parity.check_sets(a, st_g, a, st_o, 0)
