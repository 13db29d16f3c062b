#!/usr/bin/env python3
"""Throughput of batched homotopy-continuation path tracking on one MI355X.

Workload (the throughput configuration): 512 random dense quadratic systems in
n = 8 unknowns (45 monomials per equation, coefficients i.i.d. CN(0,1)), each
solved from the total-degree start system x_i^2 - 1 = 0 with its own random
unit-modulus gamma: 256 paths per system, 131,072 paths per step.  A "step" is
one full hc_track_device call: kernel-table preparation, path initialisation,
tracking (RK4 predictor + Newton corrector + adaptive step) and FP64 endpoint
refinement, with inputs already resident in HBM.

Prints ONE JSON line.  `value` is mixed-precision (FP32 tracking, FP64 end zone
and refinement) paths per second; FP64 figures, the per-instance FP64
comparator, the latency of the single small instance and the CPU oracle
baseline ride along in the same line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}   # MI355X published vector peaks
# HBM bytes per tracking launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch, scaled by the
# reading of a 512 MiB device copy in the same run), for the kernel versions profiled in profiles/; they are
# not measured live, and a kernel changed since its counters were taken has no entry.
PROFILED_TRAFFIC_BYTES = {"k_track_grp<8,8,float,false>": 171.2e6, "k_track_grp<8,8,double,false>": 453.1e6}


def w_lu(n: int) -> int:
    """FLOPs of LU with partial pivoting on [A | b] plus back substitution
    (complex add 2, mul 6, multiply-add 8, reciprocal 8, |re|+|im| compare 2)."""
    f = sum(8 * (n - k - 1) * (n - k) + 6 * (n - k - 1) + 2 * (n - k) + 8 for k in range(n))
    return f + sum(8 * (n - k - 1) + 6 for k in range(n))


# ---- the useful-FLOP count of the contract: per stage (one evaluation of [H_x | rhs] plus one solve)

def w_stage_dense(n: int, T: int) -> int:
    """Dense quadratic tables: 8nT (F) + 3n(n+1) (monomials) + 8n^2(n+1) (F_x,
    affine per entry) + the solve."""
    return 8 * n * T + 3 * n * (n + 1) + 8 * n * n * (n + 1) + w_lu(n)


def w_stage_param(system) -> int:
    """Linear parameter homotopy on term lists: 20 per term of H (the blend and
    two contractions) + 12 per term of the Jacobian (the blend and one
    multiply-add) + the solve."""
    e = np.asarray(system.term_exp)
    return 20 * e.shape[0] + 12 * int((e > 0).sum()) + w_lu(int(system.n))


def useful_flops(info, n: int, w_stage: int) -> float:
    """FLOPs the FP64 oracle's paths do in tracking (its own counters): per step
    attempt 4 RK4 stages and the RK combine (16n), per corrector iteration one
    stage; the endpoint refinement runs in another kernel and is not counted."""
    att = info["steps"].astype(np.float64) + info["rejects"]
    return float(np.sum((4.0 * att + info["newton_its"]) * w_stage + 16.0 * n * att))


# ---- the kernels' own count (what the tracker executes per stage), reported beside

def w_eval_kernel(n: int) -> int:
    """FLOPs to build [H_x | rhs] for a dense quadratic total-degree homotopy as the
    kernel does: per equation n^2 complex multiply-adds for the Jacobian row, 2n
    for L.x and x.J (F by Euler's identity), 2n to scale the row by t and 37 for
    G, G', gamma, the diagonal and the right-hand side."""
    return n * (8 * n * n + 18 * n + 37)


def w_stage_kernel(n: int) -> int:
    return w_eval_kernel(n) + w_lu(n)


def w_term(d: int, blend: int) -> int:
    """Kernel FLOPs of one term of degree d: the coefficient blend, the monomial
    and the products of all but one factor by prefix and suffix products
    (3d - 5 complex multiplies for d >= 2), F += c m (8) and one multiply-add per
    factor into the Jacobian row (8 d); a linear term needs no products (its
    Jacobian entry is c, an add), a constant only the add into F."""
    if d == 0:
        return blend + 2
    if d == 1:
        return blend + 8 + 2
    return blend + 6 * (3 * d - 5) + 8 + 8 * d


def term_kind(system) -> int:
    """The library's term-list kernel kind for a system (the smallest solver that
    holds it): 5, 3, 0 for degree <= 2 and n <= 10, 14, 16; 1, 4, 2 for higher
    degree and n <= 16, 18, 20."""
    n, d = int(system.n), int(np.asarray(system.term_exp).sum(axis=1).max())
    if d <= 2:
        return 5 if n <= 10 else 3 if n <= 14 else 0 if n <= 16 else 4 if n <= 18 else 2
    return 1 if n <= 16 else 4 if n <= 18 else 2


def w_eval_terms_kernel(system, param: bool) -> int:
    """Kernel FLOPs of one evaluation of [H_x | rhs] from term lists: per term
    w_term (parameter homotopy: 8 for the blend and c1 - c0), plus 37 per
    equation for G, gamma and the blend under total degree."""
    deg = np.asarray(system.term_exp).sum(axis=1)
    blend = 8 if param else 0
    w = int(sum(w_term(int(d), blend) for d in deg))
    if not param:
        w += 37 * int(system.n)
    return w


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def time_batch(ctx, sysh, p, g, ep, st, info, opts, steps, warmup, torch):
    for _ in range(warmup):
        ctx.track_device(sysh, p, g, ep, st, info, opts=opts)
    torch.cuda.synchronize()
    profs = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.track_device(sysh, p, g, ep, st, info, opts=opts)
        profs.append(ctx.last_profile().as_dict())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, profs


def roofline(profs, kind, kernel, w_contract, w_kernel, useful_per_step=None, useful_source=None):
    """Roofline of the dominant kernel of one mode: the tracking launch (in mixed
    precision one launch of the FP32 tracker whose escalated paths run their
    FP64 stages inside it, or, on the term-list kinds that escalate in a second
    launch, the FP32 launch plus that FP64 launch).  achieved = useful FLOPs per launch / the launch's
    mean duration from HIP events on its stream.  Useful FLOPs are the FP64
    oracle's tracking work on this workload (useful_per_step, the same figure for
    both precisions; `useful_source` says how it was counted), else the stages
    the GPU ran x the contract's per-stage count.  The kernel's own count of what
    it executes per stage is reported beside (achieved_kernel_count)."""
    key = "fp32" if kind == "fp32" else "fp64"
    ms = float(np.mean([p[f"ms_track_{key}"] for p in profs]))
    launches = max(float(np.mean([p[f"launches_{key}"] for p in profs])), 1.0)
    stages = float(np.mean([p[f"stages_{key}"] + (p["stages_fp64"] if key == "fp32" else 0.0) for p in profs]))
    # mixed precision with escalation in a second launch (term-list kinds): the
    # FP64 launch's time belongs to the same tracking work (its stages are
    # counted above); with inline escalation that interval is empty
    ms64 = float(np.mean([p["ms_track_fp64"] for p in profs])) if key == "fp32" else 0.0
    per_launch_s = (ms + ms64) / launches * 1e-3
    if useful_per_step is not None:
        flops, src = float(useful_per_step), useful_source or "oracle"
    else:
        flops, src = stages * w_contract, "GPU-executed stages x the contract's per-stage count"
    achieved = flops / launches / per_launch_s / 1e12
    peak = PEAK_TFLOPS[key]
    traffic = PROFILED_TRAFFIC_BYTES.get(kernel)
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
           "frac": round(achieved / peak, 4), "traffic": traffic,
           "traffic_source": "rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel version, profiles/ (not live)"
           if traffic is not None else None,
           "kernel": kernel, "kernel_ms_per_launch": round(ms / launches, 4), "launches_per_step": launches,
           "fp64_pass_ms_per_step": round(ms64, 4),
           "flops_source": src, "flops_per_stage": w_contract, "useful_flops_per_launch": flops / launches,
           "gpu_stages_per_launch": stages / launches, "flops_per_stage_kernel": w_kernel,
           "achieved_kernel_count": round(stages * w_kernel / launches / per_launch_s / 1e12, 3)}
    return out


def has_duplicate(f, tol=1e-8):
    """Whether two rows of f lie within tol (relative max-norm) of each other."""
    if len(f) < 2:
        return False
    d = np.abs(f[:, None, :] - f[None, :, :]).max(-1) / np.maximum(1.0, np.abs(f).max(-1))[None, :]
    d[np.arange(len(f)), np.arange(len(f))] = np.inf
    return bool(d.min() <= tol)


def set_parity(ep_g, st_g, ep_o, st_o, ok_gpu=0):
    """Endpoint error of the GPU's finite solutions against the FP64 oracle's,
    instance by instance: a one-to-one pairing (nearest oracle root by k-d tree,
    greedy when two GPU roots pick the same one), relative max-norm distance over
    max(1, |x|).  Returns the worst distance, the instances whose finite counts
    differ, and the failure rates of both sides.  An instance where two of the
    oracle's finite endpoints coincide lost a root to path jumping on the oracle's
    side (it has no crossing check): it is counted apart, as are instances whose
    GPU endpoints repeat a root."""
    from scipy.spatial import cKDTree
    worst, mismatch, o_dup, g_dup = 0.0, 0, 0, 0
    for i in range(len(ep_o)):
        fg = ep_g[i][st_g[i] == ok_gpu]
        fo = ep_o[i][st_o[i] == 0]
        if has_duplicate(fg):
            g_dup += 1
        if has_duplicate(fo):
            o_dup += 1
            continue
        if len(fg) != len(fo):
            mismatch += 1
            continue
        if len(fo) == 0:
            continue
        emb = lambda z: np.concatenate([z.real, z.imag], axis=1)  # noqa: E731
        _, j = cKDTree(emb(fg)).query(emb(fo), k=1, p=np.inf)
        if len(np.unique(j)) != len(j):
            free = np.ones(len(fg), bool)
            j = np.zeros(len(fo), int)
            for k, y in enumerate(fo):
                d = np.where(free, np.max(np.abs(fg - y), axis=1), np.inf)
                j[k] = int(np.argmin(d))
                free[j[k]] = False
        d = np.max(np.abs(fg[j] - fo), axis=1) / np.maximum(1.0, np.max(np.abs(fo), axis=1))
        worst = max(worst, float(d.max()))
    return {"instances": len(ep_o), "max_rel_err": worst, "finite_count_mismatches": mismatch,
            "oracle_path_jump_instances": o_dup, "gpu_duplicate_instances": g_dup,
            "gpu_failure_rate": float(np.mean(st_g[:len(ep_o)] != ok_gpu)),
            "oracle_failure_rate": float(np.mean(st_o != 0))}


def trifocal_slack(S) -> float:
    """Factor on an FP64 root's first-order forward-error bound for the distance
    of two correct FP64 computations of it: 2 (2 sqrt(2) (d + 1) + T_i) for terms
    of degree <= d in T_i terms per equation (the evaluation's rounding, twice)."""
    d = int(np.asarray(S.term_exp).sum(axis=1).max())
    T = int(np.bincount(np.asarray(S.term_eq)).max())
    return 2.0 * (2.0 * np.sqrt(2.0) * (d + 1) + T)


def conditioned_parity(ep_g, st_g, ep_o, st_o, fe_o, slack, rel=1e-9):
    """For badly conditioned roots (trifocal): per instance the one-to-one
    pairing's distances against each oracle root's own bar max(rel, slack x its
    forward-error bound + 2e-14); returns the roots past rel, those past their
    own bar, and the worst distance over the bound."""
    from scipy.spatial import cKDTree
    past_rel = past_bar = 0
    worst = 0.0
    for i in range(len(ep_o)):
        fg = ep_g[i][st_g[i] == 0]
        ok = st_o[i] == 0
        fo, fe = ep_o[i][ok], fe_o[i][ok]
        if len(fg) != len(fo) or len(fo) == 0:
            continue
        emb = lambda z: np.concatenate([z.real, z.imag], axis=1)  # noqa: E731
        _, j = cKDTree(emb(fg)).query(emb(fo), k=1, p=np.inf)
        d = np.max(np.abs(fg[j] - fo), axis=1) / np.maximum(1.0, np.max(np.abs(fo), axis=1))
        bar = slack * fe + 2e-14
        past_rel += int(np.sum(d > rel))
        past_bar += int(np.sum(d > np.maximum(rel, bar)))
        worst = max(worst, float(np.max(d / bar)))
    return {"slack": round(slack, 2), "roots_past_1e-9": past_rel, "roots_past_own_bar": past_bar,
            "worst_distance_over_bound": worst}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(S, coef, gam, single_inst=8):
    """The FP64 oracle (built -O3 -march=native) on the whole workload with every
    host core, and on its first `single_inst` instances with one thread.  Also
    returns the oracle's endpoints, statuses and counters for the parity and
    useful-FLOP figures."""
    import oracle
    lib = oracle.use_native_build()
    threads = oracle.default_threads()    # every core of this process's CPU share
    t0 = time.perf_counter()
    oep, ost, oinfo = oracle.track(S, coef, gam, n_threads=threads)
    dt = time.perf_counter() - t0
    n_start = oep.shape[1]
    paths = len(coef) * n_start
    t0 = time.perf_counter()
    oracle.track(S, coef[:single_inst], gam[:single_inst], n_threads=1)
    dt1 = time.perf_counter() - t0
    res = {"value": round(paths / dt, 1), "unit": "tracks/s", "cores": threads, "kind": "oracle",
           "sample": f"all {len(coef)} instances ({paths} paths, FP64) on {threads} threads in {dt:.1f} s; "
                     f"one thread: first {single_inst} instances in {dt1:.1f} s",
           "solves_per_s": round(len(coef) / dt, 2),
           "single_thread_tracks_per_s": round(single_inst * n_start / dt1, 1),
           "cpu_model": cpu_model(), "build": oracle.NATIVE_FLAGS, "library": os.path.basename(lib),
           "success_frac": round(float(np.mean(ost == 0)), 5)}
    return res, (oep, ost, oinfo)


def oracle_sample(S, coef, start, c0, k):
    """The oracle on the first k instances of a parameter-homotopy workload (all
    host cores): endpoints, statuses, counters and the wall time."""
    import oracle
    t0 = time.perf_counter()
    oep, ost, oinfo = oracle.track(S, coef[:k], start=start, coef0=c0, kind=oracle.LINEAR)
    return oep, ost, oinfo, time.perf_counter() - t0


def run_param_modes(ctx, hc, torch, sysh, p, ps, start, ep, st, info, steps, warmup, S, kernel_fmt,
                    w_contract, w_kernel, useful_per_step, useful_source, osamp, n_inst, n_start, osamp_eg=None):
    """FP64 and mixed runs of one parameter-homotopy batch: timing, statuses,
    roofline, endpoint error on the oracle's sampled instances; with osamp_eg
    (the oracle's end-game endpoints of the same sample) also mixed precision
    with the end-game ("mixed_endgame")."""
    out = {}
    modes = ("fp64", "mixed") + (("mixed_endgame",) if osamp_eg is not None else ())
    for mode in modes:
        oep, ost = osamp_eg if mode == "mixed_endgame" else osamp
        opts = hc.default_opts(precision="fp64" if mode == "fp64" else "mixed",
                               endgame=1 if mode == "mixed_endgame" else 0)
        for _ in range(warmup):
            ctx.track_device(sysh, p, None, ep, st, info, start=start, p_start=ps, opts=opts)
        torch.cuda.synchronize()
        profs = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.track_device(sysh, p, None, ep, st, info, start=start, p_start=ps, opts=opts)
            profs.append(ctx.last_profile().as_dict())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        stn = st.cpu().numpy()
        inf = info.cpu().numpy().view(hc.INFO_DTYPE).reshape(n_inst, n_start)
        k = len(oep)
        out[mode] = {"ms_per_step": dt * 1e3, "tracks_per_s": n_inst * n_start / dt, "solves_per_s": n_inst / dt,
                     "success_frac": float(np.mean(stn == hc.HC_T_SUCCESS)),
                     "status_counts": np.bincount(stn.ravel(), minlength=8).tolist(),
                     "escalated": int(inf["escalated"].sum()),
                     "mean_steps": float(inf["steps"].mean() + inf["rejects"].mean()),
                     "endpoint_error_vs_oracle": set_parity(ep[:k].cpu().numpy(), stn[:k], oep, ost),
                     "profile": {q: float(np.mean([r[q] for r in profs])) for q in profs[0]},
                     "roofline": roofline(profs, "fp64" if mode == "fp64" else "fp32",
                                          kernel_fmt.format("double" if mode == "fp64" else "float"),
                                          w_contract, w_kernel, useful_per_step, useful_source)}
        if mode == "mixed_endgame":
            out[mode]["cycle_counts"] = np.bincount(inf["cycle"].ravel(), minlength=3).tolist()
        log(f"bench: {mode}: {dt * 1e3:.1f} ms/step, {n_inst * n_start / dt:.3e} tracks/s")
    out["mixed_over_fp64"] = round(out["mixed"]["tracks_per_s"] / out["fp64"]["tracks_per_s"], 3)
    return out


def vision_leg(ctx, hc, torch, steps, warmup, n_views=4, sample=16):
    """N-view triangulation batch (4096 instances; 4 views: 296 paths each, 3
    views: 94; parameter homotopy from the monodromy start set) in both
    precisions; the oracle runs the first `sample` instances."""
    import hc_inputs.vision as V
    dev = torch.device("cuda:0")
    S = V.triangulation_system(n_views)
    c0, sols = V.start_instance(n_views)
    _, coef, _ = V.vision_workload(f"triang{n_views}_batch4096")
    n_inst, n_start, n = coef.shape[0], sols.shape[0], S.n
    oep, ost, oinfo, odt = oracle_sample(S, coef, sols, c0, sample)
    osamp_eg = None
    if n_views == 3:
        # the end-game leg (3 views: ~6% of the paths stop short of infinity without it)
        import oracle
        e, s_, _, _ = oracle.track(S, coef[:sample], start=sols, coef0=c0, kind=oracle.LINEAR, endgame=True)
        osamp_eg = (e, s_)
    w_c = w_stage_param(S)
    useful = useful_flops(oinfo, n, w_c) / sample * n_inst
    p = torch.from_numpy(coef).to(dev)
    ps = torch.from_numpy(c0).to(dev)
    start = torch.from_numpy(sols).to(dev)
    ep = torch.empty((n_inst, n_start, n), dtype=torch.complex128, device=dev)
    st = torch.empty((n_inst, n_start), dtype=torch.int32, device=dev)
    info = torch.empty((n_inst, n_start, 32), dtype=torch.uint8, device=dev)
    sysh = ctx.load_system(S, kind=hc.HC_PARAMETER)
    out = {"workload": f"triang{n_views}_batch4096: {n_inst} noisy {n_views}-view triangulation instances "
                       f"(n={n}, {S.n_terms} terms; each camera pair's pose perturbed as the paper's 4-view "
                       f"experiment does, so the critical points are isolated), parameter homotopy from a "
                       f"{n_start}-solution monodromy start set ({n_inst * n_start:,} paths)",
           "oracle_sample": f"first {sample} instances, {odt:.1f} s"}
    out.update(run_param_modes(ctx, hc, torch, sysh, p, ps, start, ep, st, info, steps, warmup, S,
                               "k_track_terms<" + str(term_kind(S)) + ",{},true>", w_c,
                               w_eval_terms_kernel(S, True) + w_lu(n), useful,
                               f"oracle counters of the first {sample} instances, scaled to {n_inst}",
                               (oep, ost), n_inst, n_start, osamp_eg))
    ctx.free_system(sysh)
    return out


def p3p_leg(ctx, hc, torch, steps, warmup, sample=1024):
    """P3P batch (65536 noisy instances x 8 total-degree paths, dense tables with
    n = 3) in both precisions, on device buffers; the oracle runs the first
    `sample` instances."""
    import oracle
    import hc_inputs.p3p as P
    dev = torch.device("cuda:0")
    S, coef, gam, _ = P.p3p_workload("p3p_batch65536")
    n_inst, n_start, n = coef.shape[0], 8, S.n
    oep, ost, oinfo = oracle.track(S, coef[:sample], gam[:sample])
    T = 1 + n + n * (n + 1) // 2
    w_c = w_stage_dense(n, T)
    useful = useful_flops(oinfo, n, w_c) / sample * n_inst
    p = torch.from_numpy(coef).to(dev)
    g = torch.from_numpy(gam).to(dev)
    ep = torch.empty((n_inst, n_start, n), dtype=torch.complex128, device=dev)
    st = torch.empty((n_inst, n_start), dtype=torch.int32, device=dev)
    info = torch.empty((n_inst, n_start, 32), dtype=torch.uint8, device=dev)
    sysh = ctx.load_system(S)
    out = {"workload": f"p3p_batch65536: {n_inst} noisy P3P instances (3 quadratics in the depths, 13 terms), "
                       f"total-degree homotopy, {n_inst * n_start:,} paths; oracle on the first {sample}"}
    for mode in ("fp64", "mixed"):
        opts = hc.default_opts(precision=mode)
        dt, profs = time_batch(ctx, sysh, p, g, ep, st, info, opts, steps, warmup, torch)
        stn = st.cpu().numpy()
        out[mode] = {"ms_per_step": dt * 1e3, "tracks_per_s": n_inst * n_start / dt, "solves_per_s": n_inst / dt,
                     "success_frac": float(np.mean(stn == hc.HC_T_SUCCESS)),
                     "status_counts": np.bincount(stn.ravel(), minlength=7).tolist(),
                     "endpoint_error_vs_oracle": set_parity(ep[:sample].cpu().numpy(), stn[:sample], oep, ost),
                     "roofline": roofline(profs, "fp32" if mode == "mixed" else "fp64",
                                          f"k_track_grp<3,4,{'float' if mode == 'mixed' else 'double'},false>",
                                          w_c, w_eval_terms_kernel(S, False) + w_lu(n), useful,
                                          f"oracle counters of the first {sample} instances, scaled")}
        log(f"bench: P3P {mode}: {dt * 1e3:.2f} ms/step, {n_inst / dt:.3e} solves/s")
    ctx.free_system(sysh)
    return out


def fivept_leg(ctx, hc, torch, steps, warmup, sample=32):
    """5-point relative pose + depth batch (1024 noisy instances x 40 paths from
    the monodromy start set, general-degree term lists, n = 16) in both
    precisions, on device buffers; the oracle runs the first `sample`."""
    import hc_inputs.fivept as F
    dev = torch.device("cuda:0")
    S = F.fivept_system()
    p0, sols = F.start_instance()
    c0 = F.coefficients(p0)
    _, coef, _ = F.fivept_workload("fivept_batch1024")
    n_inst, n_start, n = coef.shape[0], sols.shape[0], S.n
    oep, ost, oinfo, odt = oracle_sample(S, coef, sols, c0, sample)
    w_c = w_stage_param(S)
    useful = useful_flops(oinfo, n, w_c) / sample * n_inst
    p = torch.from_numpy(coef).to(dev)
    ps = torch.from_numpy(c0).to(dev)
    start = torch.from_numpy(sols).to(dev)
    ep = torch.empty((n_inst, n_start, n), dtype=torch.complex128, device=dev)
    st = torch.empty((n_inst, n_start), dtype=torch.int32, device=dev)
    info = torch.empty((n_inst, n_start, 32), dtype=torch.uint8, device=dev)
    sysh = ctx.load_system(S, kind=hc.HC_PARAMETER)
    out = {"workload": f"fivept_batch1024: {n_inst} noisy 5-point relative pose + depth instances (n=16, "
                       f"{S.n_terms} terms of degree <= 3), parameter homotopy from a {n_start}-solution "
                       f"monodromy start set ({n_inst * n_start:,} paths); oracle on the first {sample}"}
    out.update(run_param_modes(ctx, hc, torch, sysh, p, ps, start, ep, st, info, steps, warmup, S,
                               "k_track_terms<" + str(term_kind(S)) + ",{},true>", w_c,
                               w_eval_terms_kernel(S, True) + w_lu(n), useful,
                               f"oracle counters of the first {sample} instances, scaled", (oep, ost), n_inst,
                               n_start))
    ctx.free_system(sysh)
    return out


TRIFOCAL_ORACLE_SAMPLE = os.path.join(ROOT, "tests", "golden", "trifocal_oracle_sample.npz")


def trifocal_leg(ctx, hc, torch, steps, warmup, n_inst=1024, n_inst_fp64=256):
    """Trifocal pose batch (instances of trifocal_batch1024, each solved from the
    monodromy start set along the family's two-leg parameter path) on device
    buffers; one step = both legs.  Mixed precision on n_inst instances (the
    full batch by default), FP64 on the first n_inst_fp64.  The endpoint error
    and the useful FLOPs come from the oracle's two-leg endpoints of sampled
    instances stored by tests/golden/make_trifocal_oracle_sample.py (the oracle
    takes about a minute per instance).  The warmup runs on 8 instances."""
    import hc_inputs.trifocal as TF
    dev = torch.device("cuda:0")
    S = TF.trifocal_system()
    p0, sols = TF.start_instance()
    _, _, sc = TF.trifocal_workload("trifocal_batch1024", n_inst=n_inst)
    n_start, n = sols.shape[0], S.n
    mids = np.stack([TF.coefficients(TF.waypoints(p0, p1)[1]) for p1 in sc["pts"]])
    ends = np.stack([TF.coefficients(p1) for p1 in sc["pts"]])
    c0 = torch.from_numpy(TF.coefficients(p0)).to(dev)
    cm = torch.from_numpy(mids).to(dev)
    ce = torch.from_numpy(ends).to(dev)
    start = torch.from_numpy(sols).to(dev)
    ep1 = torch.empty((n_inst, n_start, n), dtype=torch.complex128, device=dev)
    st1 = torch.empty((n_inst, n_start), dtype=torch.int32, device=dev)
    info1 = torch.empty((n_inst, n_start, 32), dtype=torch.uint8, device=dev)
    ep = torch.empty_like(ep1)
    st = torch.empty_like(st1)
    info = torch.empty_like(info1)
    nan = torch.full_like(ep1, complex(float("nan"), 0.0))
    sysh = ctx.load_system(S, kind=hc.HC_PARAMETER)
    w_c = w_stage_param(S)
    gold = None
    if os.path.exists(TRIFOCAL_ORACLE_SAMPLE):
        z = np.load(TRIFOCAL_ORACLE_SAMPLE)
        if z["n_start"] == n_start and np.array_equal(z["sols_sha"], np.frombuffer(
                __import__("hashlib").sha256(sols.tobytes()).digest(), np.uint8)):
            gold = z
    out = {"workload": f"trifocal_batch1024: noisy trifocal-pose instances (n=18, 234 terms of degree <= 5), "
                       f"two-leg parameter path from a {n_start}-solution monodromy start set; mixed on "
                       f"{n_inst} instances ({n_inst * n_start:,} paths per leg), FP64 on the first {n_inst_fp64}"}
    for mode, ni in (("mixed", n_inst), ("fp64", n_inst_fp64)):
        opts = hc.default_opts(precision=mode)

        def solve(profs, k):
            ctx.track_device(sysh, cm[:k], None, ep1[:k], st1[:k], info1[:k], start=start, p_start=c0, opts=opts)
            if profs is not None:
                profs.append(ctx.last_profile().as_dict())
            s2 = torch.where((st1[:k] == hc.HC_T_SUCCESS)[..., None], ep1[:k], nan[:k])
            ctx.track_device(sysh, ce[:k], None, ep[:k], st[:k], info[:k], start=s2, p_start=cm[:k], opts=opts)
            if profs is not None:
                profs.append(ctx.last_profile().as_dict())

        for _ in range(warmup):
            solve(None, min(8, ni))
        torch.cuda.synchronize()
        profs = []
        t0 = time.perf_counter()
        for _ in range(steps):
            solve(profs, ni)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        stn = st[:ni].cpu().numpy()
        legs = {}
        for name, inf_t in (("leg1", info1), ("leg2", info)):
            inf = inf_t[:ni].cpu().numpy().view(hc.INFO_DTYPE).reshape(ni, n_start)
            legs[name] = {"steps": float(inf["steps"].mean()), "rejects": float(inf["rejects"].mean()),
                          "newton_its": float(inf["newton_its"].mean()),
                          "escalated_frac": float(inf["escalated"].mean())}
        useful = src = None
        res = {"instances": ni, "ms_per_step": dt * 1e3, "tracks_per_s": ni * n_start / dt,
               "solves_per_s": ni / dt, "success_frac": float(np.mean(stn == hc.HC_T_SUCCESS)),
               "finite_per_instance": float(np.mean(np.sum(stn == hc.HC_T_SUCCESS, axis=1))),
               "status_counts": np.bincount(stn.ravel(), minlength=7).tolist(), "legs": legs}
        if gold is not None:
            sel = [k for k, i in enumerate(gold["instances"]) if int(i) < ni]
            idx = [int(gold["instances"][k]) for k in sel]
            if idx:
                epn = ep[:ni].cpu().numpy()
                res["endpoint_error_vs_oracle"] = set_parity(epn[idx], stn[idx], gold["endpoints"][sel],
                                                             gold["status"][sel])
                res["endpoint_error_vs_oracle"]["instances_checked"] = idx
                res["endpoint_error_vs_oracle"]["conditioned"] = conditioned_parity(
                    epn[idx], stn[idx], gold["endpoints"][sel], gold["status"][sel], gold["fe_bound"][sel],
                    trifocal_slack(S))
            # per leg, the oracle's tracking FLOPs of its sampled instances, scaled
            # to this run's instances; a "launch" here is one leg
            # one call = one leg: half the two legs' work per call on average
            useful = float(gold["useful_flops_per_instance"]) * ni / 2
            src = f"oracle counters of instances {list(gold['instances'])} (both legs), scaled to {ni}"
        res["roofline"] = roofline(profs, "fp32" if mode == "mixed" else "fp64",
                                   f"k_track_terms<{term_kind(S)},{'float' if mode == 'mixed' else 'double'},true>", w_c,
                                   w_eval_terms_kernel(S, True) + w_lu(n), useful, src)
        out[mode] = res
        log(f"bench: trifocal {mode} ({ni} instances): {dt * 1e3:.1f} ms/step, {ni * n_start / dt:.3e} tracks/s "
            f"per leg")
    ctx.free_system(sysh)
    return out


def lu_leg(ctx, hc, torch, sizes=(4, 8, 12, 16, 20), batches=(1000, 1 << 18), reps=50):
    """Standalone batched complex FP32 solves (the fused LU of [A | b] plus back
    substitution), the setting of the paper's batched-solver experiment (1000
    matrices of 4x4 to 20x20), and a 2^18 batch for throughput; against
    torch.linalg.solve (the ROCm library's batched LU factorisation and solve)
    on the same data.  Times from HIP events on the launch stream, mean of
    `reps` calls.  Algorithmic HBM bytes per system: A and b read, x written, the
    info word written."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(77)
    out = {}
    for batch in batches:
        for n in sizes:
            A = torch.from_numpy(((rng.standard_normal((batch, n, n)) + 1j * rng.standard_normal((batch, n, n)))
                                  / np.sqrt(2)).astype(np.complex64)).to(dev)
            b = torch.from_numpy(((rng.standard_normal((batch, n)) + 1j * rng.standard_normal((batch, n)))
                                  / np.sqrt(2)).astype(np.complex64)).to(dev)
            x = torch.empty_like(b)
            info = torch.empty((batch,), dtype=torch.int32, device=dev)

            def timed(fn):
                fn()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    fn()
                e1.record()
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / reps

            ms = timed(lambda: ctx.solve_batched_device(A, b, x, info))
            ms_lib = timed(lambda: torch.linalg.solve(A, b.unsqueeze(-1)))
            err = float((torch.linalg.solve(A, b.unsqueeze(-1)).squeeze(-1) - x).abs().max())
            bytes_ = batch * (8 * n * n + 8 * n + 8 * n + 4)
            flops = batch * w_lu(n)
            out[f"n{n}_batch{batch}"] = {"us": round(ms * 1e3, 2), "us_library": round(ms_lib * 1e3, 2),
                                         "speedup": round(ms_lib / ms, 2), "max_abs_diff": err,
                                         "GB_per_s": round(bytes_ / (ms * 1e-3) / 1e9, 1),
                                         "TFLOP_per_s": round(flops / (ms * 1e-3) / 1e12, 3)}
            log(f"bench: batched LU n={n} batch={batch}: {ms * 1e3:.1f} us vs library {ms_lib * 1e3:.1f} us")
    out["note"] = ("roofline: hbm, peak 8000 GB/s (bytes per system 8n^2 + 16n + 4); flops W_LU(n) per system "
                   "against the 157.3 TFLOP/s FP32 vector peak")
    return out


def eval_leg(ctx, hc, torch, repeats=(1, 32), reps=20):
    """The evaluation step alone on the dense8_batch512 shape (512 instances of
    the dense n = 8 quadratic family, 256 points each): F and its Jacobian in
    FP32 by the two engines of hc_eval_dense_device, one Jacobian row per lane
    on the vector ALUs (the trackers' evaluation) and the [n^2 x (n + 1)] x
    [(n + 1) x points] matrix-core contraction.  repeat = 1 is bound by the
    outputs' HBM traffic (8 n (n + 2) bytes per point, read 8 n); repeat = 32
    evaluates every point 32 times to time the arithmetic.  FLOPs per point and
    evaluation: 8 n^3 + 16 n^2 (the rows' n^2 complex products of coefficients
    and unknowns, the linear terms' and Euler's 2n per row).  HIP events on the
    launch stream, mean of `reps` calls."""
    import hc_inputs
    S, coef, _ = hc_inputs.workload("dense8_batch512")
    n, n_inst, n_pts = S.n, coef.shape[0], 256
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(11)
    xr = rng.standard_normal((n_inst, n_pts, n, 2)).astype(np.float32)
    x = torch.from_numpy((xr[..., 0] + 1j * xr[..., 1]).astype(np.complex64)).to(dev)
    p = torch.from_numpy(coef).to(dev)
    sysh = ctx.load_system(S, layout=hc.HC_LAYOUT_DENSE)
    F = torch.empty((n_inst, n_pts, n), dtype=torch.complex64, device=dev)
    J = torch.empty((n_inst, n_pts, n, n), dtype=torch.complex64, device=dev)
    w = 8 * n ** 3 + 16 * n ** 2
    out = {"workload": f"dense8_batch512 shape: {n_inst} instances x {n_pts} points, n={n}, FP32",
           "flops_per_point": w}
    for engine, name, peak in ((hc.HC_EVAL_ROWS, "rows_valu", PEAK_TFLOPS["fp32"]),
                               (hc.HC_EVAL_MFMA, "mfma", PEAK_TFLOPS["fp32"])):
        for rep in repeats:
            def call():
                ctx.eval_dense_device(sysh, p, x, engine=engine, repeat=rep, F=F, J=J)
            call()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                call()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            tf = n_inst * n_pts * rep * w / (ms * 1e-3) / 1e12
            gbs = n_inst * n_pts * 8 * (n * (n + 2) + n) / (ms * 1e-3) / 1e9
            out[f"{name}_repeat{rep}"] = {"us": round(ms * 1e3, 2), "TFLOP_per_s": round(tf, 2),
                                          "frac_of_peak": round(tf / peak, 4), "peak": peak,
                                          "GB_per_s": round(gbs, 1)}
            log(f"bench: evaluation {name} repeat {rep}: {ms * 1e3:.1f} us, {tf:.1f} TFLOP/s")
    Fr, Jr = ctx.eval_dense_device(sysh, p, x, engine=hc.HC_EVAL_ROWS)
    Fm, Jm = ctx.eval_dense_device(sysh, p, x, engine=hc.HC_EVAL_MFMA)
    torch.cuda.synchronize()
    out["max_rel_diff_engines"] = float(((Jr - Jm).abs() / Jr.abs().clamp(min=1.0)).max())
    out["note"] = ("peak: the published 157.3 TFLOP/s FP32 for both the vector ALUs (no packed FP32 "
                   "instructions here; plain FP32 FMAs still issue above half of it) and the matrix cores; "
                   "GB/s counts x read, F and J written")
    return out


def _serving_trace(rate, total, seed):
    """Open-loop Poisson arrival times over `total` seconds and each request's
    draw (kind, n, instance index), the same for every serving run."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=int(rate * total * 1.2) + 16)
    arrivals = np.cumsum(gaps)
    arrivals = arrivals[arrivals < total]
    kinds = rng.random(len(arrivals))
    ns = rng.integers(5, 11, size=len(arrivals))
    picks = rng.integers(0, 64, size=len(arrivals))
    return arrivals, kinds, ns, picks


def _serving_inputs(ctx, hc):
    import hc_inputs
    import hc_inputs.vision as V
    systems = {n: ctx.load_system(hc_inputs.dense_quadratic_system(n)) for n in range(5, 11)}
    pool = {n: hc_inputs.dense_quadratic_instances(n, 64, seed=900 + n) for n in range(5, 11)}
    tri = ctx.load_system(V.triangulation_system(), kind=hc.HC_PARAMETER)
    tri_c0, tri_sols = V.start_instance()
    _, tri_coef, _ = V.triangulation_instances(64, seed=950)
    return systems, pool, tri, tri_c0, tri_sols, tri_coef


SERVE_MIX = "40% dense n=8 (256 paths), 40% 4-view triangulation (296 paths), 20% dense n in 5..10 (2^n paths)"


def serve_mix(ctx, hc, rate=2000.0, warm_s=1.0, meas_s=5.0, seed=5, precision="mixed"):
    """Open-loop Poisson arrivals at `rate` requests/s into the serving loop
    (continuous batching).  Mix: 40% one dense n = 8 system with 256 paths (the
    throughput workload's request), 40% one 4-view triangulation instance (296
    paths from the start set kept resident on the device), 20% one dense system
    with n uniform in 5..10 and 2^n paths."""
    systems, pool, tri, tri_c0, tri_sols, tri_coef = _serving_inputs(ctx, hc)
    srv = hc.Server(ctx, max_inflight=4, max_batch_requests=256, opts=hc.default_opts(precision=precision))
    tri_set = srv.add_start_set(tri, tri_sols, p_start=tri_c0)
    arrivals, kinds, ns, picks = _serving_trace(rate, warm_s + meas_s, seed)
    tickets = []
    reset_done = False
    t0 = time.perf_counter()
    for k, ta in enumerate(arrivals):
        while time.perf_counter() - t0 < ta:
            pass
        if not reset_done and ta >= warm_s:
            srv.reset_stats()
            reset_done = True
        if 0.4 <= kinds[k] < 0.8:
            tickets.append(srv.submit(tri, tri_coef[picks[k]], start_set=tri_set))
        else:
            n = 8 if kinds[k] < 0.4 else int(ns[k])
            _, coef, gam = pool[n]
            tickets.append(srv.submit(systems[n], coef[picks[k]], gam[picks[k]]))
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    return {"offered_rate": rate, "measured_s": meas_s, "requests": int(st["latencies"]),
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3), "max_ms": round(st["max_ms"], 3),
            "solves_per_s": round(st["completed"] / st["wall_s"], 1),
            "tracks_per_s": round(st["tracks_completed"] / st["wall_s"], 1), "batches": int(st["batches"]),
            "mix": f"{SERVE_MIX}; {precision} precision; 4 batches in flight, <= 256 requests per batch; the "
                   f"triangulation start set resident on the device"}


def serve_per_request(ctx, hc, rate=2000.0, warm_s=0.5, meas_s=1.5, seed=5):
    """The comparator of the serving loop: the same arrival trace served by plain
    per-request FP64 launches (one hc_track call per request, host buffers, in
    arrival order, no batching).  Latency = completion - arrival; requests that
    arrive while the device is busy wait in the queue."""
    systems, pool, tri, tri_c0, tri_sols, tri_coef = _serving_inputs(ctx, hc)
    arrivals, kinds, ns, picks = _serving_trace(rate, warm_s + meas_s, seed)
    o64 = hc.default_opts(precision="fp64")
    lat, paths = [], 0
    t0 = time.perf_counter()
    for k, ta in enumerate(arrivals):
        while time.perf_counter() - t0 < ta:
            pass
        if 0.4 <= kinds[k] < 0.8:
            ctx.track(tri, tri_coef[picks[k]], start=tri_sols, p_start=tri_c0, opts=o64)
            npaths = tri_sols.shape[0]
        else:
            n = 8 if kinds[k] < 0.4 else int(ns[k])
            _, coef, gam = pool[n]
            ctx.track(systems[n], coef[picks[k]], gam[picks[k]], opts=o64)
            npaths = 2 ** n
        if ta >= warm_s:
            lat.append(time.perf_counter() - t0 - ta)
            paths += npaths
    wall = time.perf_counter() - t0 - warm_s
    lat = np.array(lat) * 1e3
    return {"offered_rate": rate, "measured_s": meas_s, "requests": len(lat),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "max_ms": round(float(lat.max()), 3), "solves_per_s": round(len(lat) / wall, 1),
            "tracks_per_s": round(paths / wall, 1),
            "mix": f"{SERVE_MIX}; FP64; one hc_track call per request in arrival order"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip every leg beyond the dense8_batch512 batch")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a known-size kernel that calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters in a profiled run)")
    ap.add_argument("--trifocal-instances", type=int, default=1024,
                    help="instances of the trifocal leg's mixed batch (the full batch is 1024)")
    ap.add_argument("--skip", default="",
                    help="comma-separated legs to skip: per_instance,host,latency,triangulation,triangulation3,p3p,"
                         "fivept,trifocal,lu,eval,serving,serving_per_request")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: paths are independent "
                                   "and the multi-GPU path is not part of this build (--gpus 1)"}))
        sys.exit(2)

    import torch

    import hc_inputs
    import paper_2112_03444_amd as hc

    dev = torch.device("cuda:0")
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_mib} MiB device to device")
        del src, dst
    S, coef, gam = hc_inputs.workload("dense8_batch512")
    n_inst, n_start, n = coef.shape[0], 256, S.n
    T = 1 + n + n * (n + 1) // 2
    p = torch.from_numpy(coef).to(dev)
    g = torch.from_numpy(gam).to(dev)
    ep = torch.empty((n_inst, n_start, n), dtype=torch.complex128, device=dev)
    st = torch.empty((n_inst, n_start), dtype=torch.int32, device=dev)
    info = torch.empty((n_inst, n_start, 32), dtype=torch.uint8, device=dev)

    ctx = hc.Context(0)
    sysh = ctx.load_system(S)
    ctx.set_profiling(True)
    res, profs_of, out_of = {}, {}, {}
    modes = ["fp64", "mixed"] if args.mode == "both" else [args.mode]
    for mode in modes:
        log(f"bench: {mode} batch, {args.warmup} warmup + {args.steps} timed steps")
        opts = hc.default_opts(precision=mode)
        dt, profs = time_batch(ctx, sysh, p, g, ep, st, info, opts, args.steps, args.warmup, torch)
        stn = st.cpu().numpy()
        inf = info.cpu().numpy().view(hc.INFO_DTYPE).reshape(n_inst, n_start)
        out_of[mode] = (ep.cpu().numpy(), stn)
        profs_of[mode] = profs
        res[mode] = {
            "ms_per_step": dt * 1e3,
            "tracks_per_s": n_inst * n_start / dt,
            "solves_per_s": n_inst / dt,
            "success_frac": float(np.mean(stn == hc.HC_T_SUCCESS)),
            "escalated": int(inf["escalated"].sum()),
            "mean_steps": float(inf["steps"].mean() + inf["rejects"].mean()),
            "profile": {k: float(np.mean([q[k] for q in profs])) for k in profs[0]},
        }
        log(f"bench: {mode}: {dt * 1e3:.2f} ms/step, {n_inst * n_start / dt:.3e} tracks/s")

    # the CPU oracle on the same workload: the baseline rate, and the reference
    # for the endpoint error and the useful-FLOP count of the GPU runs
    cpu, useful, useful_src = None, None, None
    if not args.no_cpu:
        log("bench: CPU oracle baseline (all host cores, the whole workload; one thread on 8 instances)")
        cpu, (oep, ost, oinfo) = cpu_baseline(S, coef, gam)
        useful = useful_flops(oinfo, n, w_stage_dense(n, T))
        useful_src = "FP64 oracle counters of the whole workload (4 stages per step attempt + corrector iterations)"
        for mode in modes:
            res[mode]["endpoint_error_vs_oracle"] = set_parity(out_of[mode][0], out_of[mode][1], oep, ost)
    for mode in modes:
        res[mode]["roofline"] = roofline(profs_of[mode], "fp32" if mode == "mixed" else "fp64",
                                         f"k_track_grp<8,8,{'float' if mode == 'mixed' else 'double'},false>",
                                         w_stage_dense(n, T), w_stage_kernel(n), useful, useful_src)

    extras = {}
    # the vector FMA rates the ALU roofline's peaks stand for, measured on this device
    extras["measured_peak_tflops"] = {"fp32_plain": round(ctx.measure_vector_peak(False), 2),
                                      "fp64": round(ctx.measure_vector_peak(True), 2)}
    log(f"bench: measured vector FMA peaks (TFLOP/s): {extras['measured_peak_tflops']}")
    # the tracking launches against the FMA rates measured on this device
    for mode, r in res.items():
        m = extras["measured_peak_tflops"]["fp32_plain" if mode == "mixed" else "fp64"]
        if m > 0:
            r["roofline"]["frac_of_measured_fma_rate"] = round(r["roofline"]["achieved"] / m, 4)
    skip = set(x for x in args.skip.split(",") if x)
    if not args.no_extras and "per_instance" not in skip:
        # paper-style comparator: plain FP64, one instance per call (one launch set each)
        log("bench: per-instance FP64 comparator (512 calls)")
        o64 = hc.default_opts(precision="fp64")
        ctx.set_profiling(False)
        ctx.track_device(sysh, p[:1], g[:1], ep[:1], st[:1], info[:1], opts=o64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n_inst):
            ctx.track_device(sysh, p[i:i + 1], g[i:i + 1], ep[i:i + 1], st[i:i + 1], info[i:i + 1], opts=o64)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        extras["per_instance_fp64"] = {"tracks_per_s": n_inst * n_start / dt, "ms_per_instance": dt / n_inst * 1e3}
    if not args.no_extras and "host" not in skip:
        # the host-buffer entry point on the same batch: coefficients and gammas
        # copied in, endpoints, status and info copied out over PCIe in each call
        log("bench: host-buffer entry point (mixed, copies included)")
        om = hc.default_opts(precision="mixed")
        ctx.set_profiling(False)
        ctx.track(sysh, coef, gam, opts=om)
        ts = []
        for _ in range(max(1, args.steps)):
            t0 = time.perf_counter()
            ctx.track(sysh, coef, gam, opts=om)
            ts.append(time.perf_counter() - t0)
        dt = float(np.mean(ts))
        extras["host_buffers_mixed"] = {"tracks_per_s": n_inst * n_start / dt, "ms_per_step": dt * 1e3,
                                        "bytes_in": int(coef.nbytes + gam.nbytes),
                                        "bytes_out": int(n_inst * n_start * (n * 16 + 4 + 32))}
        log(f"bench: host buffers: {dt * 1e3:.2f} ms/step, {n_inst * n_start / dt:.3e} tracks/s")
    if not args.no_extras and "latency" not in skip:
        o64 = hc.default_opts(precision="fp64")
        ctx.set_profiling(False)
        # latency of one small instance (n = 3, 8 paths, FP64)
        log("bench: single-instance latency (n=3, 8 paths, FP64), 1000 calls")
        S1, c1, g1 = hc_inputs.workload("dense3_single")
        sys1 = ctx.load_system(S1)
        p1 = torch.from_numpy(c1).to(dev)
        q1 = torch.from_numpy(g1).to(dev)
        e1 = torch.empty((1, 8, 3), dtype=torch.complex128, device=dev)
        s1 = torch.empty((1, 8), dtype=torch.int32, device=dev)
        lat = []
        for r in range(1050):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.track_device(sys1, p1, q1, e1, s1, None, opts=o64)
            torch.cuda.synchronize()
            if r >= 50:
                lat.append(time.perf_counter() - t0)
        lat = np.array(lat) * 1e3
        extras["latency_dense3_single_ms"] = {"p50": float(np.percentile(lat, 50)),
                                              "p99": float(np.percentile(lat, 99)),
                                              "repeats": len(lat)}
        # the same with the launch sequence replayed from a captured hipGraph
        log("bench: single-instance latency with hipGraph replay, 1000 calls")
        gs = torch.cuda.Stream()
        og = hc.default_opts(precision="fp64", use_graph=1)
        lat = []
        for r in range(1050):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.track_device(sys1, p1, q1, e1, s1, None, opts=og, stream=gs)
            gs.synchronize()
            if r >= 50:
                lat.append(time.perf_counter() - t0)
        lat = np.array(lat) * 1e3
        extras["latency_dense3_single_graph_ms"] = {"p50": float(np.percentile(lat, 50)),
                                                    "p99": float(np.percentile(lat, 99)),
                                                    "repeats": len(lat)}
    if not args.no_extras and "triangulation" not in skip:
        log("bench: 4-view triangulation batch")
        ctx.set_profiling(True)
        extras["triangulation"] = vision_leg(ctx, hc, torch, max(2, args.steps // 2), 1)
        ctx.set_profiling(False)
    if not args.no_extras and "p3p" not in skip:
        log("bench: P3P batch")
        ctx.set_profiling(True)
        extras["p3p"] = p3p_leg(ctx, hc, torch, args.steps, 1)
        ctx.set_profiling(False)
    if not args.no_extras and "fivept" not in skip:
        log("bench: 5-point relative pose + depth batch")
        ctx.set_profiling(True)
        extras["fivept"] = fivept_leg(ctx, hc, torch, max(2, args.steps // 2), 1)
        ctx.set_profiling(False)
    if not args.no_extras and "triangulation3" not in skip:
        log("bench: 3-view triangulation batch")
        ctx.set_profiling(True)
        extras["triangulation3"] = vision_leg(ctx, hc, torch, max(2, args.steps // 2), 1, n_views=3)
        ctx.set_profiling(False)
    if not args.no_extras and "trifocal" not in skip:
        log("bench: trifocal pose batch")
        ctx.set_profiling(True)
        extras["trifocal"] = trifocal_leg(ctx, hc, torch, 1, 1, n_inst=args.trifocal_instances,
                                          n_inst_fp64=min(256, args.trifocal_instances))
        ctx.set_profiling(False)
    if not args.no_extras and "lu" not in skip:
        log("bench: standalone batched LU solves")
        extras["batched_lu"] = lu_leg(ctx, hc, torch)
    if not args.no_extras and "eval" not in skip:
        log("bench: evaluation engines (vector rows vs matrix cores) on the dense8_batch512 shape")
        extras["eval_engines"] = eval_leg(ctx, hc, torch)
    if not args.no_extras and "serving" not in skip:
        log("bench: serving, Poisson arrivals at 2000 requests/s, 1 s warmup + 5 s, mixed and FP64")
        extras["serving"] = serve_mix(ctx, hc)
        extras["serving_fp64"] = serve_mix(ctx, hc, precision="fp64")
    if not args.no_extras and "serving_per_request" not in skip:
        log("bench: serving comparator, plain per-request FP64 launches on the same arrival trace (0.5 s + 1.5 s)")
        extras["serving_per_request_fp64"] = serve_per_request(ctx, hc)

    head = res["mixed"] if "mixed" in res else res["fp64"]
    out = {
        "metric": "tracks/s & solves/s (FP32+FP64-refine vs FP64) at 1 GPU; p99 solve latency",
        "value": round(head["tracks_per_s"], 1),
        "unit": "tracks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32+fp64" if "mixed" in res else "fp64",
        "data": "synthetic",
        "config": {"workload": "dense8_batch512: 512 random dense quadratic systems, n=8, "
                               "total-degree start, 256 paths each (131,072 paths)",
                   "n": n, "n_inst": n_inst, "paths_per_instance": n_start,
                   "precision": "mixed" if "mixed" in res else "fp64"},
        "solves_per_s": round(head["solves_per_s"], 2),
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "modes": {m: {k: v for k, v in r.items() if k != "roofline"} | {"roofline": r["roofline"]}
                  for m, r in res.items()},
    }
    if "mixed" in res and "fp64" in res:
        out["mixed_over_fp64"] = round(res["mixed"]["tracks_per_s"] / res["fp64"]["tracks_per_s"], 3)
    out.update(extras)
    if "per_instance_fp64" in extras:
        out["batched_mixed_over_per_instance_fp64"] = round(
            head["tracks_per_s"] / extras["per_instance_fp64"]["tracks_per_s"], 2)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
