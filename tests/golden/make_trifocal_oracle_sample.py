"""Writes tests/golden/trifocal_oracle_sample.npz: the FP64 oracle's endpoints of
sampled instances of the trifocal_batch1024 workload along the family's
two-leg parameter path (view 1's coordinates first, then views 2 and 3), from
the stored monodromy start set.  Calls only oracle/ (and the input generators);
the GPU tests and the benchmark's trifocal leg compare against it, since the
oracle needs about a minute per instance.

    python tests/golden/make_trifocal_oracle_sample.py [--threads=N]

Stored: instances (their indices in the batch), n_start, sols_sha (sha256 of
the start set's bytes: a start set written later makes the file stale),
endpoints [k, N, 18] and status [k, N] of leg 2 (a path whose leg 1 failed
counts as NONFINITE), the first-order forward-error bound of every leg-2
endpoint (fe_bound [k, N], see forward_error_bound) and the oracle's tracking
FLOPs per instance (both legs; 4 stages per step attempt and one per
corrector iteration at the contract's per-stage count).
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import hc_inputs.trifocal as TF  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "trifocal_oracle_sample.npz")
SAMPLE = [0, 511, 1023]
U = 2.0 ** -53


def forward_error_bound(S, c1, x):
    """First-order bound of the forward error of an FP64 root x of F(.; c1),
    relative to max(1, |x|_inf): ||J^-1||_2 u ||(sum_k |c_ik| |m_k(x)|)_i||_2 /
    max(1, |x|_inf) -- the evaluation's rounding (u times that sum per equation,
    up to a constant of the evaluation) carried through the inverse Jacobian."""
    _, J = oracle.eval_system(S, c1, x)
    inv = 1.0 / np.linalg.svd(J, compute_uv=False)[-1]
    m = np.prod(np.power(x[None, :], S.term_exp), axis=1)
    den = np.zeros(S.n)
    np.add.at(den, S.term_eq, np.abs(c1) * np.abs(m))
    return inv * U * np.linalg.norm(den) / max(1.0, np.max(np.abs(x)))


def w_lu(n):
    f = sum(8 * (n - k - 1) * (n - k) + 6 * (n - k - 1) + 2 * (n - k) + 8 for k in range(n))
    return f + sum(8 * (n - k - 1) + 6 for k in range(n))


def main():
    threads = None
    for a in sys.argv[1:]:
        if a.startswith("--threads="):
            threads = int(a.split("=", 1)[1])
    S = TF.trifocal_system()
    p0, sols = TF.start_instance()
    _, _, sc = TF.trifocal_workload("trifocal_batch1024")
    e = np.asarray(S.term_exp)
    w_stage = 20 * e.shape[0] + 12 * int((e > 0).sum()) + w_lu(S.n)
    eps, sts, fes, flops = [], [], [], []
    t0 = time.time()
    for i in SAMPLE:
        w = TF.waypoints(p0, sc["pts"][i])
        c0, cm, ce = TF.coefficients(w[0]), TF.coefficients(w[1]), TF.coefficients(w[2])
        e1, s1, i1 = oracle.track(S, cm[None], start=sols, coef0=c0, kind=oracle.LINEAR, n_threads=threads)
        ok = s1[0] == oracle.SUCCESS
        e2, s2, i2 = oracle.track(S, ce[None], start=e1[0][ok], coef0=cm, kind=oracle.LINEAR, n_threads=threads)
        ep = np.full((len(sols), S.n), np.nan + 0j)
        st = np.full(len(sols), oracle.NONFINITE, np.int32)
        ep[ok], st[ok] = e2[0], s2[0]
        fe = np.full(len(sols), np.nan)
        for b in np.flatnonzero(st == oracle.SUCCESS):
            fe[b] = forward_error_bound(S, ce, ep[b])
        fl = 0.0
        for inf in (i1[0], i2[0]):
            att = inf["steps"].astype(np.float64) + inf["rejects"]
            fl += float(np.sum((4.0 * att + inf["newton_its"]) * w_stage + 16.0 * S.n * att))
        eps.append(ep)
        sts.append(st)
        fes.append(fe)
        flops.append(fl)
        print(f"instance {i}: {int(np.sum(st == oracle.SUCCESS))} finite, {time.time() - t0:.0f} s", flush=True)
    np.savez(OUT, instances=np.array(SAMPLE), n_start=len(sols),
             sols_sha=np.frombuffer(hashlib.sha256(sols.tobytes()).digest(), np.uint8),
             endpoints=np.stack(eps), status=np.stack(sts), fe_bound=np.stack(fes),
             useful_flops_per_instance=float(np.mean(flops)))
    print(OUT, hashlib.sha256(open(OUT, "rb").read()).hexdigest())


if __name__ == "__main__":
    main()
