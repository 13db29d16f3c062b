"""Pins of the trifocal-pose workload (section 4: three views, shared unknown
focal length, 4 points) and of its start instance, on the CPU: the expanded
system against the projection model it comes from, the planted ground truth
of noise-free scenes, the symmetries (quaternion signs, focal flip), and the
stored monodromy start set."""
import numpy as np
import pytest

import hc_inputs.trifocal as TF
import oracle
import oracle.monodromy as M


def quat_rotation(q):
    """Rotation matrix of a quaternion by the Euler-Rodrigues formula, written
    from (a, b, c, d) directly (no polynomial expansion)."""
    a, b, c, d = q
    return np.array([[a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
                     [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
                     [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d]])


def model_residuals(x, pts):
    """The 18 equations from the matrix form of the model: for each view k and
    point p, A = rho_p R_k d_1 + f t_k and (x_k A_3 - f A_1, y_k A_3 - f A_2),
    then |q_12|^2 - 1, |q_13|^2 - 1."""
    f = x[TF.I_F]
    out = []
    for k in (2, 3):
        q = x[TF.I_Q[k]:TF.I_Q[k] + 4]
        t = x[TF.I_T[k]:TF.I_T[k] + 3]
        R = quat_rotation(q)
        for p in range(4):
            rho = 1.0 if p == 0 else x[TF.I_RHO[p]]
            d1 = np.array([pts[0, p, 0], pts[0, p, 1], f])
            A = rho * (R @ d1) + f * t
            out += [pts[k - 1, p, 0] * A[2] - f * A[0], pts[k - 1, p, 1] * A[2] - f * A[1]]
    for k in (2, 3):
        q = x[TF.I_Q[k]:TF.I_Q[k] + 4]
        out.append(q @ q - 1.0)
    return np.array(out)


def test_structure():
    S = TF.trifocal_system()
    assert (S.n, S.n_terms) == (18, 234)
    assert np.bincount(S.term_eq).tolist() == [14] * 16 + [5, 5]
    assert S.term_exp.sum(axis=1).max() == 5
    # every monomial is even in each quaternion: q -> -q is a symmetry
    for k in (2, 3):
        assert np.all(S.term_exp[:, TF.I_Q[k]:TF.I_Q[k] + 4].sum(axis=1) % 2 == 0)


def test_system_is_the_projection_model():
    """F(x) from the expanded term tables equals the matrix-form model at random
    complex points."""
    S, coef, sc = TF.trifocal_instances(3, seed=21)
    rng = np.random.default_rng(2)
    for i in range(3):
        for _ in range(3):
            x = rng.standard_normal(18) + 1j * rng.standard_normal(18)
            F = oracle.eval_system(S, coef[i], x)
            F = F[0] if isinstance(F, tuple) else F
            ref = model_residuals(x, sc["pts"][i])
            assert np.max(np.abs(F - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_planted_ground_truth_and_sign_orbit_solve_noise_free_scenes():
    S, coef, sc = TF.trifocal_instances(4, seed=22, sigma=0.0)
    for i in range(4):
        gt = sc["gt"][i]
        assert abs(gt[TF.I_F] * TF.F0 - sc["f"][i]) < 1e-9
        for x in TF.symmetry_orbit(gt):
            assert oracle.residual(S, coef[i], x.astype(complex)) < 1e-14


def test_symmetries_map_the_system_to_plus_minus_itself():
    """At any complex point, q -> -q leaves every equation's value unchanged and
    the focal flip negates the 16 projection equations and keeps the norms (so
    both map solutions to solutions)."""
    S, coef, _ = TF.trifocal_instances(2, seed=24)
    rng = np.random.default_rng(4)
    sign = np.array([-1.0] * 16 + [1.0, 1.0])
    for i in range(2):
        x = rng.standard_normal(18) + 1j * rng.standard_normal(18)
        F = oracle.eval_system(S, coef[i], x)
        F = F[0] if isinstance(F, tuple) else F
        for y in TF.sign_orbit(x):
            G = oracle.eval_system(S, coef[i], y)
            G = G[0] if isinstance(G, tuple) else G
            np.testing.assert_allclose(G, F, rtol=1e-13, atol=1e-13 * np.abs(F).max())
        G = oracle.eval_system(S, coef[i], TF.focal_flip(x))
        G = G[0] if isinstance(G, tuple) else G
        np.testing.assert_allclose(G, sign * F, rtol=1e-13, atol=1e-13 * np.abs(F).max())
    assert TF.symmetry_orbit(np.zeros((3, 18))).shape == (8, 3, 18)


def test_quaternion_extraction_round_trip():
    rng = np.random.default_rng(3)
    for _ in range(20):
        R = TF._rotation(rng.normal(0, 1.0, 3))
        q = TF.rotation_to_quaternion(R)
        assert abs(np.linalg.norm(q) - 1) < 1e-14
        np.testing.assert_allclose(quat_rotation(q), R, atol=1e-14)


@pytest.fixture(scope="module")
def start():
    return TF.start_instance()


def test_start_set_is_regular_distinct_and_sign_closed(start):
    """The stored monodromy set: every point a root of the start instance with
    tiny backward error, pairwise distinct, and closed under the eight-element
    symmetry group (so its size is a multiple of 8)."""
    from scipy.spatial import cKDTree
    S = TF.trifocal_system()
    p0, sols = start
    c0 = TF.coefficients(p0)
    assert sols.shape[1] == 18 and len(sols) % 8 == 0
    assert max(oracle.residual(S, c0, x) for x in sols) < 1e-12
    # max-norm distances over real and imaginary parts, relative to max(1, |x|)
    emb = lambda z: np.concatenate([z.real, z.imag], axis=-1)  # noqa: E731
    scale = np.maximum(1.0, np.max(np.abs(sols), axis=1))
    tree = cKDTree(emb(sols))
    d2, _ = tree.query(emb(sols), k=2, p=np.inf)      # nearest other solution
    assert np.all(d2[:, 1] / scale > 1e-6)
    for img in TF.symmetry_orbit(sols):               # every image is a stored solution
        d, j = tree.query(emb(img), k=1, p=np.inf)
        assert np.all(d / scale[j] <= 1e-12)


def test_noise_free_ground_truth_is_among_the_oracle_endpoints(start):
    """Tracking the start set to a noise-free scene along the two legs reaches
    the planted pose and all eight of its symmetry images."""
    S = TF.trifocal_system()
    p0, sols = start
    _, _, sc = TF.trifocal_instances(1, seed=23, sigma=0.0)
    w = TF.waypoints(p0, sc["pts"][0])
    e1, s1, _ = oracle.track(S, TF.coefficients(w[1])[None], start=sols, coef0=TF.coefficients(w[0]),
                             kind=oracle.LINEAR)
    ep, st, _ = oracle.track(S, TF.coefficients(w[2])[None], start=e1[0][s1[0] == oracle.SUCCESS],
                             coef0=TF.coefficients(w[1]), kind=oracle.LINEAR)
    ok = ep[0][st[0] == oracle.SUCCESS]
    for x in TF.symmetry_orbit(sc["gt"][0]):
        d = np.max(np.abs(ok - x), axis=1)
        assert d.min() < 1e-8, d.min()


def test_start_set_complete_by_an_independent_run(start):
    """Completeness of the stored set (no trace test applies to these fibers):
    an independent monodromy run of the oracle -- its own fabricated start pair
    (seed 5), its own parameter point and loops, to the same stall rule -- stops
    at the same count, and each set carried along the two legs to the other
    run's parameter point lands only on roots of the other set (every path that
    does not fail tracking reaches a distinct root of the other set).  Written by
    `python -m oracle.monodromy trifocal-check` and `trifocal-compare`."""
    import os
    S = TF.trifocal_system()
    p0, sols = start
    z = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trifocal_check.npz"))
    rep = {str(k): int(v) for k, v in zip(z["compare_keys"], z["compare"])}
    chk = z["solutions"]
    assert len(chk) == len(sols) == rep["n_start"] == rep["n_check"]
    assert not np.allclose(z["params0"], p0)                      # another parameter point
    assert max(oracle.residual(S, TF.coefficients(z["params0"]), x) for x in chk) < 1e-12
    assert len(M.distinct_rows(chk, M.TRIFOCAL_MERGE_TOL)) == len(chk)
    # carried sets: nothing outside the other set; what is missing is exactly
    # the paths lost on the way
    assert rep["carried_not_in_start"] == 0 and rep["carried_not_in_check"] == 0
    assert rep["check_carried"] + rep["start_roots_not_reached"] == len(sols)
    assert rep["start_carried"] + rep["check_roots_not_reached"] == len(chk)
    assert rep["start_roots_not_reached"] <= 0.05 * len(sols) and rep["check_roots_not_reached"] <= 0.05 * len(chk)
