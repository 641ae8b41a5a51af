#!/usr/bin/env python3
"""Throughput of the DA-FMM hot path on one MI355X, at 1e-7 relative error.

Default workload (plummer4m): N = 4,000,000 points from a Plummer sphere
(scale radius 0.05, truncated at r = 1, seed 2), charges U(-1,1), adaptive
octree with at most 64 points per leaf, potentials and fields.  The order p is
the lowest from 12 up whose relative L2 error of the potential against the
FP64 direct sum, on 4096 seeded sample targets, is at most 1e-7 (the paper's
error measure sigma of Sec. 3.5); it is 14 on this input.  One step is one pass
of the whole path over the input with positions and charges already in HBM:
fmm_plan (root, Morton keys, radix sort, boxes, U/V/W/X lists, sorted
particles, M2L tiles) followed by fmm_evaluate (P2M, M2M, M2L, P2L, L2L,
L2P/M2P, P2P, output).  `value` is the plain FP64 path; the mixed path
(FP32 P2P terms with compensated sums, FP32 M2L where the precision rule
allows it) is timed beside it with its own sigma.

The roofline entry is for the dominant kernel, the sign-class M2L: its
algorithmic work per launch is, for every target and every sign class of its
V list with a member, the contraction over parity-compatible (row, column)
classes of harmonic components plus the butterflies that combine the members
(m2l_work); the time is the M2L stage from HIP events on the evaluation
stream, averaged over the timed evaluations.  The dense counts (2 (p+1)^4 per
V pair on harmonic components, 2 n_p^2 on the full DA vectors) are reported
beside it.  The CPU baseline is the oracle's direct sum on the 4096 sample
targets (the exact reference at any accuracy), timed on the host cores.

The same line carries a short served run (continuous batching, Poisson
arrivals at half the saturated rate) with p50/p99 latency and the achieved
sigma per requested-accuracy bucket, the uniform 1e6-point workload at
p = 8 (uniform1m), and the second kernel, the softened Coulomb potential
1/sqrt(r^2 + eps^2), on those points (eps = 1e-3, softened1m) and on 1e6
Plummer points with an adaptive tree (eps = 1e-4, softened_plummer1m).

Other workloads (--workload): uniform1m, softened1m or softened_plummer1m alone, batch256 (256 independent
problems, one fmm_evaluate_batch), serve (the served stream at four arrival
rates), sweep (leaf size x order x N on Gaussian points), calib (a plain
256 MiB device copy, for the HBM byte-counter calibration).
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particles/s at 1e-7 rel. err (plain FP64 vs mixed); p50/p99 solve latency"
FP64_PEAK_TFLOPS, FP32_PEAK_TFLOPS = 78.6, 157.3
TARGET_SIGMA = 1e-7

# HBM bytes per launch of the dominant M2L kernel, from rocprofv3 FETCH_SIZE
# and WRITE_SIZE scaled by a plain-copy calibration (read x2.0, write x1.0;
# profiles/).  Each figure is valid only for the kernel sources it was
# measured on (kernel, shared header, tile order): a different fingerprint
# reports null.
M2L_TRAFFIC = {
    "uniform1m": {"fingerprint": "3c89b53399f58b31", "bytes": (1296.29 + 153.34) * 1e6},
    "plummer4m_p14": {"fingerprint": "3c89b53399f58b31", "bytes": (33599.88 + 998.38) * 1e6},
}
M2L_SOURCES = ("paper_2508_02626_amd/csrc/m2l.hip", "paper_2508_02626_amd/csrc/common.h",
               "paper_2508_02626_amd/csrc/m2l_tiles.hip")


def m2l_fingerprint():
    import hashlib
    h = hashlib.sha256()
    for f in M2L_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def m2l_traffic(workload):
    e = M2L_TRAFFIC.get(workload)
    return e["bytes"] if e and e["fingerprint"] == m2l_fingerprint() else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- work counts
def sym_class_counts(p):
    """Harmonic components (i, j, kz), kz in {0, 1}, |.| <= p, per parity class
    c = (i % 2) << 2 | (j % 2) << 1 | kz."""
    n = [0] * 8
    for d in range(p + 1):
        for kz in (0, 1):
            for i in range(d - kz + 1) if d - kz >= 0 else []:
                j = d - kz - i
                n[(i & 1) << 2 | (j & 1) << 1 | kz] += 1
    return n


def cart_class_counts(p):
    """Monomials x^i y^j z^k (i + j + k <= p) in each parity class (i, j, k mod 2):
    the row / column classes of the softened kernel's sign-class M2L."""
    n = [0] * 8
    for i in range(p + 1):
        for j in range(p + 1 - i):
            for k in range(p + 1 - i - j):
                n[(i & 1) << 2 | (j & 1) << 1 | (k & 1)] += 1
    return n


def m2l_work(t, p, cartesian=False):
    """Algorithmic flops of one M2L evaluation on sign classes.  For every
    target and every sign class (|k_x|, |k_y|, |k_z|) of its V list that has a
    member: 2 sum n_pi n_tau over row / column parity classes compatible on
    the zero axes of the class (the contraction with the representative's
    derivative table), plus the butterflies combining the members
    (|P| 2^|P| additions per column, P the axes with a +- pair).  The classes
    are those of the folded harmonic components (Coulomb kernel) or, with
    cartesian, of the full Taylor monomials (softened kernel).  Also returns
    the number of V pairs, for the dense counts."""
    vo, vs = t["V_off"].astype(np.int64), t["V_src"].astype(np.int64)
    nv = len(vs)
    if nv == 0:
        return 0.0, 0
    tg = np.repeat(np.arange(len(vo) - 1), np.diff(vo))
    lev, code = t["level"].astype(np.int64), t["morton"].astype(np.uint64)

    def coords(b):
        c = np.zeros((len(b), 3), np.int64)
        cb, lb = code[b], lev[b]
        for bit in range(int(lev.max())):
            on = bit < lb
            for d in range(3):
                c[:, d] |= np.where(on, ((cb >> np.uint64(3 * bit + 2 - d)) & np.uint64(1)).astype(np.int64), 0) << bit
        return c

    k = np.abs(coords(tg) - coords(vs))
    cls = np.unique(tg * 64 + k[:, 0] * 16 + k[:, 1] * 4 + k[:, 2]) % 64
    a = np.stack([cls // 16, (cls // 4) % 4, cls % 4], 1)
    zero = ((a == 0) * np.array([4, 2, 1])).sum(1)
    pair = ((a == 1) | (a == 2)).sum(1)
    n = cart_class_counts(p) if cartesian else sym_class_counts(p)
    nh = sum(n) if cartesian else (p + 1) ** 2
    macs = {z: sum(n[x] * n[y] for x in range(8) for y in range(8) if not ((x ^ y) & z)) for z in range(8)}
    flops = sum(2.0 * macs[int(z)] for z in zero) + float((pair * (2 ** pair) * nh).sum())
    return flops, nv


def p2p_pairs(t):
    """Particle pairs summed by P2P: for every leaf, its count times the
    particles of its U list (the pair of a particle with itself included)."""
    cnt = t["count"].astype(np.int64)
    uo, us = t["U_off"], t["U_src"]
    per_box = np.add.reduceat(cnt[us], uo[:-1]) if len(us) else np.zeros(len(cnt), np.int64)
    per_box = np.where(uo[1:] > uo[:-1], per_box, 0)
    return int((cnt * per_box).sum())


# Algorithmic FP64 operations of one P2P pair (potential and field):
# 3 differences, r^2 (3 mul + 2 add), 1/r (counted as 2: square root and
# division), q/r, q/r^3 (3 mul), 4 accumulations (1 add + 3 fused
# multiply-adds counted as 2) = 20.
P2P_FLOPS_PER_PAIR = 20


def stage_avg(stages):
    """ms per evaluation of each stage; the two P2P parts are reported together."""
    out = {k: v[0] / max(v[1], 1) for k, v in stages.items()}
    out["p2p"] = out.get("p2p", 0.0) + out.pop("p2p_part2", 0.0)
    return out


# ---------------------------------------------------------------- measurement
def timed_steps(make_plan, q, phi, fld, steps, warmup):
    """Mean seconds of one step (fmm_plan + fmm_evaluate) over `steps` after
    `warmup` untimed ones; the plan is destroyed at the end of every step."""
    import torch
    for _ in range(warmup):
        pl = make_plan()
        pl.evaluate(q, phi, fld)
        pl.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pl = make_plan()
        pl.evaluate(q, phi, fld)
        pl.close()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def timed_evaluations(pl, q, phi, fld, steps):
    """Mean seconds of one fmm_evaluate on a built plan, with HIP-event stage
    times (ms per evaluation)."""
    import torch
    pl.evaluate(q, phi, fld)
    torch.cuda.synchronize()
    pl.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        pl.evaluate(q, phi, fld)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    st = pl.read_timing()
    pl.set_timing(False)
    return dt, stage_avg(st)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sample_targets(n, count, seed=7):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False))


def m2l_roofline(tree, p, m2l_ms, kernel, workload, peak):
    flops, nv = m2l_work(tree, p)
    nc = (p + 1) * (p + 2) * (p + 3) // 6
    achieved = flops / (m2l_ms * 1e-3) / 1e12
    dense_h = 2.0 * (p + 1) ** 4 * nv
    dense_full = 2.0 * nc * nc * nv
    return {"kernel": kernel, "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": m2l_traffic(workload), "traffic_unit": "HBM bytes per launch",
            "flops_per_launch": flops, "ms_per_launch": m2l_ms, "v_pairs": nv,
            "work": "sign-class contraction on harmonic components (unpadded) + member butterflies",
            "dense_harmonic_flops_per_launch": dense_h,
            "dense_harmonic_equivalent_tflops": dense_h / (m2l_ms * 1e-3) / 1e12,
            "dense_full_flops_per_launch": dense_full,
            "dense_full_equivalent_tflops": dense_full / (m2l_ms * 1e-3) / 1e12}


def p2p_roofline(tree, p2p_ms, kernel):
    pairs = p2p_pairs(tree)
    achieved = P2P_FLOPS_PER_PAIR * pairs / (p2p_ms * 1e-3) / 1e12
    return {"kernel": kernel, "bound": "alu", "pairs_per_launch": pairs, "ms_per_launch": p2p_ms,
            "pairs_per_s": pairs / (p2p_ms * 1e-3), "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s (FP64 vector)", "frac": achieved / FP64_PEAK_TFLOPS}


def base_record(args):
    return {"metric": METRIC, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "data": "synthetic"}


# ---------------------------------------------------------------- plummer4m
def bench_plummer(args):
    """The metric's workload: 4e6 Plummer points, adaptive s = 64, at the
    lowest order that reaches sigma <= 1e-7, FP64 and mixed."""
    import torch
    import oracle
    from paper_2508_02626_amd import fmm, inputs
    n = args.n or 4_000_000
    xh, qh = inputs.plummer(n, 2)
    x = torch.tensor(xh, device="cuda:0")
    q = torch.tensor(qh, device="cuda:0")
    phi = torch.empty(n, dtype=torch.float64, device="cuda:0")
    fld = torch.empty(n, 3, dtype=torch.float64, device="cuda:0")
    idx = sample_targets(n, args.sigma_targets)
    log("bench plummer4m: direct sum on %d sample targets (host)" % len(idx))
    t0 = time.perf_counter()
    dphi, dfld = oracle.direct(xh, qh, idx)
    t_direct = time.perf_counter() - t0
    log("bench plummer4m: direct sum %.1f s on %d threads" % (t_direct, oracle.num_threads()))

    def sigma_of(ph, fl):
        return rel(ph[idx], dphi), rel(fl[idx], dfld)

    # order: the lowest from 12 up that reaches the target
    scan = {}
    orders = [args.order] if args.order else list(range(12, 17))
    for p in orders:
        pl = fmm.Plan(x, p, leaf_size=64)
        pl.evaluate(q, phi, fld)
        pl.close()
        scan[p] = sigma_of(phi.cpu().numpy(), fld.cpu().numpy())
        log("bench plummer4m: p=%d sigma phi %.3e field %.3e" % (p, *scan[p]))
        if scan[p][0] <= TARGET_SIGMA:
            break
    p = max(scan) if args.order else next((o for o in sorted(scan) if scan[o][0] <= TARGET_SIGMA), max(scan))
    res = {}
    for mode in (["fp64"] if args.no_mixed else ["fp64", "mixed"]):
        mk = lambda: fmm.Plan(x, p, leaf_size=64, precision=mode)
        step_s = timed_steps(mk, q, phi, fld, args.steps, args.warmup)
        pl = mk()
        eval_s, stages = timed_evaluations(pl, q, phi, fld, args.steps)
        r = dict(step_s=step_s, eval_s=eval_s, stages=stages, sizes=pl.sizes())
        if mode == "fp64":
            r["tree"] = pl.export_tree()
        pl.close()
        r["phi"], r["fld"] = phi.cpu().numpy(), fld.cpu().numpy()
        r["sigma"], r["sigma_f"] = sigma_of(r["phi"], r["fld"])
        log("bench plummer4m: p=%d %s step %.2f ms eval %.2f ms sigma %.3e" %
            (p, mode, 1e3 * step_s, 1e3 * eval_s, r["sigma"]))
        res[mode] = r
    f = res["fp64"]
    kern = "k_m2l_symh<%d,*>" % p if p >= 12 else "k_m2l_sym<%d,double>" % p
    out = base_record(args)
    out.update({
        "value": n / f["step_s"], "ms_per_step": 1e3 * f["step_s"], "dtype": "f64",
        "config": {"workload": "Plummer sphere: N=%d, scale radius 0.05, truncated at r=1 (seed 2), q~U(-1,1), "
                               "adaptive octree s=64, order p=%d (lowest order from 12 with sampled sigma <= 1e-7), "
                               "potential+field" % (n, p),
                   "n": n, "order": p, "leaf_size": 64, "step": "fmm_plan + fmm_evaluate", "sizes": f["sizes"]},
        "accuracy": {"sigma_phi_vs_direct": f["sigma"], "sigma_field_vs_direct": f["sigma_f"],
                     "targets_sampled": len(idx), "target": TARGET_SIGMA, "meets_target": f["sigma"] <= TARGET_SIGMA,
                     "sigma_phi_by_order": {str(o): s[0] for o, s in scan.items()}},
        "eval_only": {"value": n / f["eval_s"], "ms": 1e3 * f["eval_s"]},
        "stage_ms": f["stages"],
        "roofline": m2l_roofline(f["tree"], p, f["stages"]["m2l"], kern, "plummer4m_p%d" % p, FP64_PEAK_TFLOPS),
        "p2p": p2p_roofline(f["tree"], f["stages"]["p2p"], "k_p2p<0>"),
    })
    if "mixed" in res:
        m = res["mixed"]
        out["mixed"] = {"value": n / m["step_s"], "ms_per_step": 1e3 * m["step_s"],
                        "speedup_vs_fp64": f["step_s"] / m["step_s"],
                        "eval_only_value": n / m["eval_s"], "eval_ms": 1e3 * m["eval_s"],
                        "sigma_phi_vs_direct": m["sigma"], "sigma_field_vs_direct": m["sigma_f"],
                        "meets_target": m["sigma"] <= TARGET_SIGMA,
                        "rel_l2_vs_fp64_path_phi": rel(m["phi"], f["phi"]),
                        "rel_l2_vs_fp64_path_field": rel(m["fld"], f["fld"]),
                        "dtype": "f64 with f32 P2P terms (compensated sums) and the FP32 M2L of this order's rule",
                        "stage_ms": m["stages"]}
    if not args.no_rotation:
        # the rotation-based M2L of Sec. 3.4 (vector unit) beside the sign-class
        # contraction (matrix cores), same plan and order
        mk = lambda: fmm.Plan(x, p, leaf_size=64, m2l="rotation")
        rsteps = max(1, args.steps // 2)
        step_s = timed_steps(mk, q, phi, fld, rsteps, 1)
        pl = mk()
        eval_s, stages = timed_evaluations(pl, q, phi, fld, rsteps)
        pl.close()
        rphi, rfld = phi.cpu().numpy(), fld.cpu().numpy()
        rs, rsf = sigma_of(rphi, rfld)
        flops, nv = m2l_work(f["tree"], p)
        S = (p + 1) * (2 * p + 1) * (2 * p + 3) // 3
        SA = (p + 1) * (p + 2) * (2 * p + 3) // 6
        rot_flops = 2.0 * (2 * S + (2 * SA - (p + 1) ** 2)) * nv  # per pair: F and B per degree, A per mode
        log("bench plummer4m: p=%d rotation M2L %.2f ms (sign-class %.2f ms), step %.2f ms" %
            (p, stages["m2l"], f["stages"]["m2l"], 1e3 * step_s))
        out["m2l_rotation"] = {
            "kernel": "k_m2l_rot<%d>" % p, "ms_per_launch": stages["m2l"],
            "sign_class_ms_per_launch": f["stages"]["m2l"],
            "flops_per_launch": rot_flops, "achieved": rot_flops / (stages["m2l"] * 1e-3) / 1e12,
            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s (FP64 vector)",
            "frac": rot_flops / (stages["m2l"] * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "value": n / step_s, "ms_per_step": 1e3 * step_s, "eval_ms": 1e3 * eval_s,
            "sigma_phi_vs_direct": rs, "sigma_field_vs_direct": rsf,
            "rel_l2_vs_sign_class_phi": rel(rphi, f["phi"]), "rel_l2_vs_sign_class_field": rel(rfld, f["fld"]),
            "work": "per V pair: 2 sum_n (2n+1)^2 (rotations) + 2 sum_m (p+1-|m|)^2 (axial) flops"}
    cores = oracle.num_threads()
    out["cpu_baseline"] = {"value": len(idx) / t_direct, "unit": "particles/s", "cores": cores, "kind": "oracle",
                           "seconds": t_direct,
                           "sample": "oracle direct O(N^2) sum (FP64, exact at any accuracy) for %d seeded sample "
                                     "targets against all %d sources of this workload" % (len(idx), n)}
    return out


# ---------------------------------------------------------------- uniform1m
def bench_uniform(args, with_cpu=True):
    """1e6 uniform points in [0,1)^3 (seed 1), uniform depth 5 on [0,1]^3,
    p = 8, FP64 and mixed."""
    import torch
    import oracle
    from paper_2508_02626_amd import fmm, inputs
    n, depth, p = 1_000_000, 5, 8
    xh, qh = inputs.uniform(n, 1)
    x = torch.tensor(xh, device="cuda:0")
    q = torch.tensor(qh, device="cuda:0")
    phi = torch.empty(n, dtype=torch.float64, device="cuda:0")
    fld = torch.empty(n, 3, dtype=torch.float64, device="cuda:0")
    idx = sample_targets(n, 2000)
    dphi, dfld = oracle.direct(xh, qh, idx)
    res = {}
    for mode in (["fp64"] if args.no_mixed else ["fp64", "p2p32", "m2l32", "mixed"]):
        mk = lambda: fmm.Plan(x, p, uniform_depth=depth, root=[0, 0, 0, 1], precision=mode)
        step_s = timed_steps(mk, q, phi, fld, args.steps, args.warmup)
        pl = mk()
        eval_s, stages = timed_evaluations(pl, q, phi, fld, args.steps)
        r = dict(step_s=step_s, eval_s=eval_s, stages=stages)
        if mode == "fp64":
            r["tree"] = pl.export_tree()
        pl.close()
        r["phi"], r["fld"] = phi.cpu().numpy(), fld.cpu().numpy()
        r["sigma"], r["sigma_f"] = rel(r["phi"][idx], dphi), rel(r["fld"][idx], dfld)
        log("bench uniform1m: %s step %.3f ms eval %.3f ms sigma %.3e" % (mode, 1e3 * step_s, 1e3 * eval_s, r["sigma"]))
        res[mode] = r
    f = res["fp64"]
    out = {"value": n / f["step_s"], "ms_per_step": 1e3 * f["step_s"], "dtype": "f64",
           "config": {"workload": "uniform cube: N=%d uniform in [0,1)^3 (seed 1), q~U(-1,1), uniform octree depth 5 "
                                  "on [0,1]^3, order p=8, potential+field" % n, "n": n, "order": p},
           "accuracy": {"sigma_phi_vs_direct": f["sigma"], "sigma_field_vs_direct": f["sigma_f"],
                        "targets_sampled": len(idx)},
           "eval_only": {"value": n / f["eval_s"], "ms": 1e3 * f["eval_s"]},
           "stage_ms": f["stages"],
           "roofline": m2l_roofline(f["tree"], p, f["stages"]["m2l"], "k_m2l_sym<8,double>", "uniform1m",
                                    FP64_PEAK_TFLOPS),
           "p2p": p2p_roofline(f["tree"], f["stages"]["p2p"], "k_p2p<0>")}
    for mode in ("p2p32", "m2l32", "mixed"):
        if mode not in res:
            continue
        m = res[mode]
        e = {"value": n / m["step_s"], "ms_per_step": 1e3 * m["step_s"], "eval_ms": 1e3 * m["eval_s"],
             "sigma_phi_vs_direct": m["sigma"], "sigma_field_vs_direct": m["sigma_f"],
             "rel_l2_vs_fp64_path_phi": rel(m["phi"], f["phi"]),
             "rel_l2_vs_fp64_path_field": rel(m["fld"], f["fld"]), "stage_ms": m["stages"]}
        if mode in ("m2l32", "mixed"):
            mm = m["stages"]["m2l"]
            e["m2l_kernel"], e["m2l_ms"] = "k_m2l_sym<8,float>", mm
            e["m2l_roofline"] = m2l_roofline(f["tree"], p, mm, "k_m2l_sym<8,float>", "-", FP32_PEAK_TFLOPS)
        if mode in ("p2p32", "mixed"):
            e["p2p"] = p2p_roofline(f["tree"], m["stages"]["p2p"], "k_p2p<1>")
        out[mode if mode == "mixed" else "only_" + mode] = e
    if with_cpu:
        t0 = time.perf_counter()
        tree = oracle.Tree(xh, root=[0, 0, 0, 1], uniform_depth=depth)
        tree.fmm(p, qh)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": n / dt, "unit": "particles/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "seconds": dt,
                               "sample": "oracle DA-FMM (TPSA operators, memoised translations) on the whole "
                                         "workload: %d points, uniform depth 5, p=8, potential+field" % n}
    return out


# ---------------------------------------------------------------- softened kernel
def bench_softened(args, plummer=False):
    """The second kernel, 1/sqrt(r^2 + eps^2), FP64: 1e6 uniform points in
    [0,1)^3 (seed 1), uniform depth 5 on [0,1]^3, p = 8, eps = 1e-3 (a tenth of
    the mean spacing); or (plummer) 1e6 Plummer points (scale radius 0.05,
    seed 2), adaptive s = 64, p = 8, eps = 1e-4.  Its M2L contracts the full
    Taylor components (the kernel is not harmonic) on sign classes (it is even
    in every coordinate): the work of m2l_work(cartesian=True) per launch;
    2 n_p^2 flops per V pair without the classes."""
    import torch
    import oracle
    from paper_2508_02626_amd import fmm, inputs
    n, depth, p, eps = 1_000_000, 5, 8, (1e-4 if plummer else 1e-3)
    xh, qh = inputs.plummer(n, 2) if plummer else inputs.uniform(n, 1)
    x = torch.tensor(xh, device="cuda:0")
    q = torch.tensor(qh, device="cuda:0")
    phi = torch.empty(n, dtype=torch.float64, device="cuda:0")
    fld = torch.empty(n, 3, dtype=torch.float64, device="cuda:0")
    idx = sample_targets(n, 2000)
    dphi, dfld = oracle.direct_soft(xh, qh, eps, idx)
    if plummer:
        mk = lambda: fmm.Plan(x, p, leaf_size=64, kernel="softened", softening=eps)
    else:
        mk = lambda: fmm.Plan(x, p, uniform_depth=depth, root=[0, 0, 0, 1], kernel="softened", softening=eps)
    step_s = timed_steps(mk, q, phi, fld, args.steps, args.warmup)
    pl = mk()
    eval_s, stages = timed_evaluations(pl, q, phi, fld, args.steps)
    tree = pl.export_tree()
    pl.close()
    ph, fl = phi.cpu().numpy(), fld.cpu().numpy()
    sig, sig_f = rel(ph[idx], dphi), rel(fl[idx], dfld)
    log("bench softened %s: step %.3f ms eval %.3f ms sigma %.3e" % ("plummer1m" if plummer else "1m", 1e3 * step_s,
                                                                    1e3 * eval_s, sig))
    flops, nv = m2l_work(tree, p, cartesian=True)
    nc = (p + 1) * (p + 2) * (p + 3) // 6
    m2l_ms = stages["m2l"]
    achieved = flops / (m2l_ms * 1e-3) / 1e12
    return {"value": n / step_s, "ms_per_step": 1e3 * step_s, "dtype": "f64",
            "config": {"workload": ("softened Coulomb kernel 1/sqrt(r^2+eps^2), eps=1e-4: N=%d Plummer points (scale "
                                    "radius 0.05, truncated at r=1, seed 2), q~U(-1,1), adaptive octree s=64, order "
                                    "p=8, potential+field" % n) if plummer else
                                   ("softened Coulomb kernel 1/sqrt(r^2+eps^2), eps=1e-3: N=%d uniform in [0,1)^3 "
                                    "(seed 1), q~U(-1,1), uniform octree depth 5 on [0,1]^3, order p=8, "
                                    "potential+field" % n), "n": n, "order": p, "softening": eps},
            "accuracy": {"sigma_phi_vs_direct": sig, "sigma_field_vs_direct": sig_f, "targets_sampled": len(idx)},
            "eval_only": {"value": n / eval_s, "ms": 1e3 * eval_s},
            "stage_ms": stages,
            "roofline": {"kernel": "k_m2l_soft_sym<8>", "bound": "mfma", "achieved": achieved,
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                         "flops_per_launch": flops, "ms_per_launch": m2l_ms, "v_pairs": nv,
                         "dense_full_flops_per_launch": 2.0 * nc * nc * nv,
                         "work": "sign-class contraction of the full Taylor components: per (target, class with "
                                 "a member) 2 sum n_pi n_tau over compatible parity classes, plus the member "
                                 "butterflies"}}


# ---------------------------------------------------------------- served
def served_run(nreq, fracs, sigma_per_bucket=6, sigma_targets=256):
    """Poisson stream through the continuous-batching server: N log-uniform in
    [1e3, 1e6], uniform or Plummer, rel. error in {1e-4, 1e-7, 1e-9} -> p in
    {4, 8, 12}.  Saturated throughput first, then the given arrival rates
    (fractions of it), p50/p99 latency per rate, and the achieved sigma of the
    first `sigma_per_bucket` requests of every accuracy bucket (sampled direct
    sum)."""
    import oracle
    from paper_2508_02626_amd import inputs, serve
    warm = max(nreq // 10, 5)
    reqs = [inputs.served_request(i) for i in range(nreq + warm)]
    ntot = sum(len(q) for _, q, _ in reqs[warm:])
    srv = serve.Server(hbm_budget_bytes=64 << 30, slots=4)
    futs = [srv.submit(x, q, e) for x, q, e in reqs[:warm]]
    [f.result() for f in futs]
    t0 = time.perf_counter()
    futs = [srv.submit(x, q, e) for x, q, e in reqs[warm:]]
    sat = [f.result() for f in futs]
    sat_s = time.perf_counter() - t0
    rate_sat = nreq / sat_s
    log("bench serve: saturated %.1f req/s, %.3e particles/s" % (rate_sat, ntot / sat_s))
    rates = {}
    for frac in fracs:
        lam = frac * rate_sat
        arr = inputs.poisson_arrivals(nreq, lam, seed=5)
        futs = []
        t0 = time.perf_counter()
        for (x, q, e), ta in zip(reqs[warm:], arr):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            futs.append(srv.submit(x, q, e))
        lat = [f.result()[2] for f in futs]
        span = time.perf_counter() - t0
        st = serve.latency_stats(lat)
        st.update({"arrival_rate_req_s": lam, "throughput_particles_s": ntot / span})
        rates["%.2f" % frac] = st
        log("bench serve: rate %.2f x sat: p50 %.1f ms p99 %.1f ms" % (frac, st["p50_ms"], st["p99_ms"]))
    srv.close()
    # achieved accuracy per bucket, from the saturated run's results
    buckets = {}
    for (x, q, e), (phi, fld, _) in zip(reqs[warm:], sat):
        b = buckets.setdefault(e, {"num": 0.0, "den": 0.0, "num_f": 0.0, "den_f": 0.0, "requests": 0})
        if b["requests"] >= sigma_per_bucket:
            continue
        idx = sample_targets(len(q), sigma_targets, seed=11)
        dp, df = oracle.direct(x, q, idx)
        b["num"] += float(np.sum((phi[idx] - dp) ** 2)); b["den"] += float(np.sum(dp ** 2))
        b["num_f"] += float(np.sum((fld[idx] - df) ** 2)); b["den_f"] += float(np.sum(df ** 2))
        b["requests"] += 1
    acc = {}
    for e, b in sorted(buckets.items(), reverse=True):
        acc["%g" % e] = {"order": serve.order_for(e), "precision": serve.precision_for(e),
                         "sigma_phi_vs_direct": float(np.sqrt(b["num"] / b["den"])),
                         "sigma_field_vs_direct": float(np.sqrt(b["num_f"] / b["den_f"])),
                         "meets_request": bool(np.sqrt(b["num"] / b["den"]) <= e),
                         "requests_sampled": b["requests"], "targets_per_request": sigma_targets}
    return {"saturated": dict(serve.latency_stats([s[2] for s in sat]), requests_per_s=rate_sat,
                              throughput_particles_s=ntot / sat_s),
            "latency_by_load": rates, "accuracy_by_bucket": acc, "requests": nreq, "particles": ntot,
            "config": "served Poisson stream: %d requests (+%d warm-up, seeds 10000+i), N log-uniform in "
                      "[1e3,1e6], uniform or Plummer, rel. error {1e-4,1e-7,1e-9} -> p {4,8,12} (mixed precision "
                      "only for 1e-4), adaptive s=64, 4 slots, 64 GiB admission budget" % (nreq, warm)}


def bench_serve(args):
    s = served_run(args.requests, (0.25, 0.5, 0.75, 0.9))
    out = base_record(args)
    out.update({"value": s["saturated"]["throughput_particles_s"],
                "ms_per_step": 1e3 / s["saturated"]["requests_per_s"],
                "dtype": "f64 (1e-7, 1e-9 buckets) / mixed (1e-4 bucket)",
                "config": {"workload": s["config"], "requests": s["requests"]},
                "saturated": s["saturated"], "latency_by_load": s["latency_by_load"],
                "accuracy_by_bucket": s["accuracy_by_bucket"], "roofline": None})
    return out


# ---------------------------------------------------------------- batch256
def bench_batch(args):
    """256 problems (N log-uniform in [1e3, 2e5], half uniform, half 8-cluster
    mixtures, p in {4,6,8}), adaptive s=64, mixed precision: plans + one
    fmm_evaluate_batch per step, against evaluating the plans one by one."""
    import torch
    from paper_2508_02626_amd import fmm, inputs
    probs = [inputs.batch_problem(i) for i in range(256)]
    xs = [torch.tensor(x, device="cuda:0") for x, _, _ in probs]
    qs = [torch.tensor(q, device="cuda:0") for _, q, _ in probs]
    ntot = sum(len(q) for _, q, _ in probs)

    def plans():
        return fmm.plan_batch(xs, [p for _, _, p in probs], leaf_size=64, precision="mixed", threads=8)

    def run(batched):
        ps = plans()
        if batched:
            fmm.evaluate_batch(ps, qs)
        else:
            for pl, q in zip(ps, qs):
                pl.evaluate(q)
        return ps

    times = {}
    for batched in (True, False):
        for _ in range(args.warmup):
            for pl in run(batched):
                pl.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for pl in run(batched):
                pl.close()
        torch.cuda.synchronize()
        times[batched] = (time.perf_counter() - t0) / args.steps
    ps = plans()
    torch.cuda.synchronize()
    ev = {}
    for batched in (True, False):
        fmm.evaluate_batch(ps, qs) if batched else [pl.evaluate(q) for pl, q in zip(ps, qs)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            if batched:
                fmm.evaluate_batch(ps, qs)
            else:
                for pl, q in zip(ps, qs):
                    pl.evaluate(q)
        torch.cuda.synchronize()
        ev[batched] = (time.perf_counter() - t0) / args.steps
    for pl in ps:
        pl.close()
    log("bench batch: step %.1f ms (one by one %.1f ms), evaluate %.1f ms (one by one %.1f ms)" %
        (1e3 * times[True], 1e3 * times[False], 1e3 * ev[True], 1e3 * ev[False]))
    out = base_record(args)
    out.update({
        "value": ntot / times[True], "ms_per_step": 1e3 * times[True], "dtype": "f64 with f32 P2P and f32 MFMA M2L",
        "config": {"workload": "256 independent problems, N log-uniform in [1e3,2e5] (seeds 1000+i), half "
                               "uniform cube, half 8-cluster mixtures (sigma 0.02), p in {4,6,8}, adaptive s=64, "
                               "mixed precision; step = one fmm_plan_batch (8 host threads) + one fmm_evaluate_batch",
                   "n_total": ntot},
        "one_by_one": {"value": ntot / times[False], "ms_per_step": 1e3 * times[False]},
        "eval_only": {"batched_ms": 1e3 * ev[True], "one_by_one_ms": 1e3 * ev[False],
                      "batched_value": ntot / ev[True]},
        "roofline": None,
    })
    return out


# ---------------------------------------------------------------- sweep
def bench_sweep(args):
    """Leaf-size and order sweep and the scaling with N, on the distribution
    of the paper's sweeps (3-D Gaussian, unit standard deviation, adaptive
    tree), plain FP64 path, one step = fmm_plan + fmm_evaluate.  For every N
    and p the leaf size with the shortest step is reported (the experiment
    behind the paper's optimal-s table); then the step time over N at
    p in {2, 6, 10} with that leaf size, and the slope of its log-log fit."""
    import torch
    import oracle
    from paper_2508_02626_amd import fmm, inputs
    sizes_n = [100_000, 1_000_000, 10_000_000]
    orders = [2, 4, 6, 8, 10]
    leaf = [16, 32, 64, 128, 256, 512]
    reps = max(1, min(args.steps, 3))

    def timed(x, q, p, s):
        def step():
            pl = fmm.Plan(x, p, leaf_size=s, precision="fp64")
            pl.evaluate(q)
            return pl
        step().close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step().close()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    table, best = {}, {}
    for n in sizes_n:
        xh, qh = inputs.gaussian(n, 3)
        x = torch.tensor(xh, device="cuda:0")
        q = torch.tensor(qh, device="cuda:0")
        table[n], best[n] = {}, {}
        for p in orders:
            row = {s: 1e3 * timed(x, q, p, s) for s in leaf}
            table[n][p] = row
            best[n][p] = min(row, key=row.get)
            log("bench sweep: N=%d p=%d best s=%d (%.2f ms)" % (n, p, best[n][p], row[best[n][p]]))
        del x, q
    xh, qh = inputs.gaussian(1_000_000, 3)
    x = torch.tensor(xh, device="cuda:0")
    q = torch.tensor(qh, device="cuda:0")
    idx = sample_targets(len(qh), 500)
    dp, _ = oracle.direct(xh, qh, idx)
    sigma = {}
    for p in orders:
        pl = fmm.Plan(x, p, leaf_size=best[1_000_000][p], precision="fp64")
        phi, fld = pl.evaluate(q)
        pl.close()
        sigma[p] = rel(phi.cpu().numpy()[idx], dp)
    del x, q
    scan = [10_000, 30_000, 100_000, 300_000, 1_000_000, 3_000_000, 10_000_000]
    linear = {}
    for p in (2, 6, 10):
        ms = []
        for n in scan:
            near = min(sizes_n, key=lambda m: abs(np.log(m / n)))
            xh, qh = inputs.gaussian(n, 4)
            x = torch.tensor(xh, device="cuda:0")
            q = torch.tensor(qh, device="cuda:0")
            ms.append(1e3 * timed(x, q, p, best[near][p]))
            del x, q
        ln, lt = np.log(scan), np.log(ms)
        big, huge = np.array(scan) >= 100_000, np.array(scan) >= 1_000_000
        linear[p] = {"n": scan, "ms": ms, "slope": float(np.polyfit(ln, lt, 1)[0]),
                     "slope_n_ge_1e5": float(np.polyfit(ln[big], lt[big], 1)[0]),
                     "slope_n_ge_1e6": float(np.polyfit(ln[huge], lt[huge], 1)[0])}
        log("bench sweep: p=%d slope %.3f (N>=1e5: %.3f)" % (p, linear[p]["slope"], linear[p]["slope_n_ge_1e5"]))
    n_top, p_top = sizes_n[-1], orders[-1]
    t_top = table[n_top][p_top][best[n_top][p_top]]
    out = base_record(args)
    out.update({
        "steps": reps, "warmup": 1,
        "value": n_top / (t_top * 1e-3), "ms_per_step": t_top, "dtype": "f64",
        "config": {"workload": "3-D Gaussian (unit std, seeds 3 and 4), q~U(-1,1), adaptive octree, plain FP64, "
                               "potential+field; value = N=1e7, p=10 at its best leaf size",
                   "n": sizes_n, "orders": orders, "leaf_sizes": leaf},
        "step_ms": {str(n): {str(p): {str(s): v for s, v in r.items()} for p, r in t.items()}
                    for n, t in table.items()},
        "best_leaf_size": {str(n): {str(p): s for p, s in b.items()} for n, b in best.items()},
        "sigma_phi_vs_direct_n1e6": {str(p): v for p, v in sigma.items()},
        "scaling_with_n": {str(p): v for p, v in linear.items()},
        "roofline": None,
    })
    return out


def bench_calib(args):
    """A plain device-to-device copy of 256 MiB, twice: the reference for the
    HBM byte counters (FETCH_SIZE, WRITE_SIZE) of rocprofv3."""
    import torch
    nbytes = 256 << 20
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"workload": "calib", "bytes_copied_per_launch": nbytes, "launches": 2}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=0, help="points of the plummer4m workload (default 4e6)")
    ap.add_argument("--order", type=int, default=0, help="plummer4m: fixed order instead of the scan")
    ap.add_argument("--sigma-targets", type=int, default=4096)
    ap.add_argument("--workload", default="plummer4m",
                    choices=["plummer4m", "uniform1m", "softened1m", "softened_plummer1m", "batch256", "serve",
                             "sweep", "calib"])
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--serve-requests", type=int, default=120, help="requests of the served run in the default line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-uniform", action="store_true")
    ap.add_argument("--no-rotation", action="store_true")
    ap.add_argument("--no-softened", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs a solve on a single GPU "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload == "plummer4m":
        out = bench_plummer(args)
        if args.no_cpu_baseline:
            out.pop("cpu_baseline", None)
        if not args.no_serve:
            s = served_run(args.serve_requests, (0.5,))
            out["served"] = {"p50_ms": s["latency_by_load"]["0.50"]["p50_ms"],
                             "p99_ms": s["latency_by_load"]["0.50"]["p99_ms"],
                             "arrival_rate_req_s": s["latency_by_load"]["0.50"]["arrival_rate_req_s"],
                             "throughput_particles_s": s["latency_by_load"]["0.50"]["throughput_particles_s"],
                             "saturated": s["saturated"], "accuracy_by_bucket": s["accuracy_by_bucket"],
                             "config": s["config"] + "; arrivals at 0.5 x the saturated rate"}
        if not args.no_uniform:
            out["uniform1m"] = bench_uniform(args, with_cpu=not args.no_cpu_baseline)
        if not args.no_softened:
            out["softened1m"] = bench_softened(args)
            out["softened_plummer1m"] = bench_softened(args, plummer=True)
    elif args.workload in ("softened1m", "softened_plummer1m"):
        out = base_record(args)
        out.update(bench_softened(args, plummer=args.workload == "softened_plummer1m"))
    elif args.workload == "uniform1m":
        out = base_record(args)
        out.update(bench_uniform(args, with_cpu=not args.no_cpu_baseline))
    else:
        out = {"batch256": bench_batch, "serve": bench_serve, "sweep": bench_sweep,
               "calib": bench_calib}[args.workload](args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
