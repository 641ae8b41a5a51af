#!/usr/bin/env python3
"""Throughput of the DA-FMM hot path on one MI355X.

Workload: N = 1,000,000 points uniform in [0,1)^3 (seed 1), charges U(-1,1),
uniform octree of depth 5 on the root cube [0,1]^3, truncation order p = 8,
potentials and fields.  One step is one pass of the whole path over this input
with the positions and charges already in HBM: fmm_plan (root, Morton keys,
radix sort, boxes, U/V/W/X lists, sorted particles, M2L slot tables) followed
by fmm_evaluate (P2M, M2M, M2L, P2L, L2L, L2P/M2P, P2P, output).  The step is
timed for the plain FP64 path (reported as `value`) and for the mixed path
(FP32 P2P with FP64 accumulation, FP32-MFMA M2L), reported beside it.

The roofline entry is for the dominant kernel, M2L on sign classes: its
algorithmic work is, per target and per sign class of its V list with a
member, the contraction over parity-compatible (row, column) classes plus the
butterflies that combine the members (m2l_work); time from HIP events on the
evaluation stream over the timed steps.  The dense harmonic count, 2 (p+1)^4
flops per V-list pair, is reported beside it.  The CPU baseline times
the plain oracle on the same workload once (a few seconds on the host cores).

Other workloads (--workload): plummer4m (4e6 Plummer points, adaptive s=64,
p=10), batch256 (256 independent problems, one fmm_evaluate_batch), serve
(Poisson request stream through the continuous-batching server, p50/p99),
sweep (leaf size x order x N on Gaussian points, and the scaling with N).
Each prints one JSON line of the same form.

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
N_DEFAULT, DEPTH, ORDER, SEED = 1_000_000, 5, 8, 1
FP64_PEAK_TFLOPS, FP32_PEAK_TFLOPS = 78.6, 157.3

# HBM bytes per launch of k_m2l_sym<8,double> on this workload, from rocprofv3
# FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration (read x2.0,
# write x1.0; profiles/uniform1m_hbm_traffic.txt).  Valid only for the kernel
# sources it was measured on (kernel, shared header, tile order): a different
# fingerprint reports null.
M2L_TRAFFIC = {"fingerprint": "2e96bb397b2bc4cb", "bytes": (1342.94 + 83.36) * 1e6}
M2L_SOURCES = ("paper_2508_02626_amd/csrc/m2l.hip", "paper_2508_02626_amd/csrc/common.h",
               "paper_2508_02626_amd/csrc/m2l_tiles.hip")


def m2l_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in M2L_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return M2L_TRAFFIC["bytes"] if h.hexdigest()[:16] == M2L_TRAFFIC["fingerprint"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_mode(x, q, precision, steps, warmup, n):
    import torch
    from paper_2508_02626_amd import fmm
    phi = torch.empty(n, dtype=torch.float64, device=x.device)
    fld = torch.empty(n, 3, dtype=torch.float64, device=x.device)

    def step():
        pl = fmm.Plan(x, ORDER, uniform_depth=DEPTH, root=[0, 0, 0, 1], precision=precision)
        pl.evaluate(q, phi, fld)
        return pl

    for _ in range(warmup):
        step().close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step().close()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / steps
    # stage breakdown and evaluate-only rate on one plan, HIP events per stage
    pl = fmm.Plan(x, ORDER, uniform_depth=DEPTH, root=[0, 0, 0, 1], precision=precision)
    pl.evaluate(q, phi, fld)
    torch.cuda.synchronize()
    pl.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        pl.evaluate(q, phi, fld)
    torch.cuda.synchronize()
    eval_s = (time.perf_counter() - t0) / steps
    stages = pl.read_timing()
    sizes = pl.sizes()
    tree = pl.export_tree()
    sizes["p2p_pairs"] = p2p_pairs(tree)
    m2l_flops = m2l_work(tree, ORDER)[0]
    pl.close()
    return dict(step_s=step_s, eval_s=eval_s, stages=stages, sizes=sizes, m2l_flops=m2l_flops,
                phi=phi.cpu().numpy(), fld=fld.cpu().numpy())


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


def m2l_work(t, p):
    """Algorithmic flops of one M2L launch on sign classes.  For every target
    and every sign class (|k_x|, |k_y|, |k_z|) of its V list that has a
    member: 2 sum n_pi n_tau over row / column parity classes compatible on
    the zero axes of the class (the contraction with the representative's
    derivative table), plus the butterflies combining the members
    (|P| 2^|P| additions per column, P the axes with a +- pair).  Also returns
    the V pairs, for the dense harmonic count 2 (p+1)^4 per pair."""
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
    n = sym_class_counts(p)
    nh = (p + 1) ** 2
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


def cpu_baseline(xh, qh):
    """The oracle DA-FMM on the whole workload (same points, tree and order)."""
    import oracle
    t0 = time.perf_counter()
    tree = oracle.Tree(xh, root=[0, 0, 0, 1], uniform_depth=DEPTH)
    tree.fmm(ORDER, qh)
    dt = time.perf_counter() - t0
    return {"value": len(qh) / dt, "unit": "particles/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": dt,
            "sample": "oracle DA-FMM (TPSA operators, memoised translations) on the whole workload: "
                      "%d points, uniform depth %d on [0,1]^3, p=%d, potential+field" % (len(qh), DEPTH, ORDER)}


def sampled_sigma(xh, qh, phi, fld, count=2000, seed=7):
    import oracle
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(len(qh), size=min(count, len(qh)), replace=False))
    dp, df = oracle.direct(xh, qh, idx)
    s_phi = float(np.linalg.norm(phi[idx] - dp) / np.linalg.norm(dp))
    s_fld = float(np.linalg.norm(fld[idx] - df) / np.linalg.norm(df))
    return s_phi, s_fld, len(idx)


# Algorithmic FP64 operations of one P2P pair (potential and field):
# 3 differences, r^2 (3 mul + 2 add), 1/r (counted as 2: square root and
# division), q/r, q/r^3 (3 mul), 4 accumulations (1 add + 3 fused
# multiply-adds counted as 2) = 20.
P2P_FLOPS_PER_PAIR = 20


def p2p_roofline(r):
    ms = stage_avg(r["stages"])["p2p"]
    pairs = r["sizes"]["p2p_pairs"]
    achieved = P2P_FLOPS_PER_PAIR * pairs / (ms * 1e-3) / 1e12
    return {"kernel": "k_p2p<0>", "bound": "alu", "pairs_per_launch": pairs, "ms_per_launch": ms,
            "pairs_per_s": pairs / (ms * 1e-3), "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s (FP64 vector)", "frac": achieved / FP64_PEAK_TFLOPS}


def base_record(args):
    return {"metric": METRIC, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "data": "synthetic"}


def stage_avg(stages):
    """ms per evaluation of each stage; the two P2P parts are reported together."""
    out = {k: v[0] / max(v[1], 1) for k, v in stages.items()}
    out["p2p"] = out.get("p2p", 0.0) + out.pop("p2p_part2", 0.0)
    return out


def bench_plummer(args):
    """4e6 Plummer points (a=0.05, r<=1, seed 2), adaptive s=64, p=10."""
    import torch
    from paper_2508_02626_amd import fmm, inputs
    n = args.n if args.n != N_DEFAULT else 4_000_000
    xh, qh = inputs.plummer(n, 2)
    x = torch.tensor(xh, device="cuda:0")
    q = torch.tensor(qh, device="cuda:0")
    p = 10
    res = {}
    for mode in ("fp64", "mixed"):
        def step():
            pl = fmm.Plan(x, p, leaf_size=64, precision=mode)
            pl.evaluate(q)
            return pl
        for _ in range(args.warmup):
            step().close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step().close()
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / args.steps
        pl = fmm.Plan(x, p, leaf_size=64, precision=mode)
        phi, fld = pl.evaluate(q)
        torch.cuda.synchronize()
        pl.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            pl.evaluate(q, phi, fld)
        torch.cuda.synchronize()
        eval_s = (time.perf_counter() - t0) / args.steps
        st, sizes = pl.read_timing(), pl.sizes()
        if mode == "fp64":
            tree = pl.export_tree()
            sizes["p2p_pairs"] = p2p_pairs(tree)
            sizes["m2l_flops"] = m2l_work(tree, p)[0]
        pl.close()
        ph, fh = phi.cpu().numpy(), fld.cpu().numpy()
        sp, sf, nt = sampled_sigma(xh, qh, ph, fh, count=1000)
        log("bench plummer: %s step %.2f ms eval %.2f ms sigma %.3e" % (mode, 1e3 * step_s, 1e3 * eval_s, sp))
        res[mode] = dict(step_s=step_s, eval_s=eval_s, stages=stage_avg(st), sizes=sizes, sigma=sp, sigma_f=sf,
                         phi=ph, fld=fh)
    # the same problem at the order that reaches a relative error of 1e-7
    hi = {}
    ph = 14
    for mode in ("fp64", "mixed"):
        pl = fmm.Plan(x, ph, leaf_size=64, precision=mode)
        phi, fld = pl.evaluate(q)
        pl.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps // 2)):
            pl = fmm.Plan(x, ph, leaf_size=64, precision=mode)
            pl.evaluate(q, phi, fld)
            pl.close()
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / max(1, args.steps // 2)
        sp, sf, nt = sampled_sigma(xh, qh, phi.cpu().numpy(), fld.cpu().numpy(), count=1000)
        log("bench plummer: p=%d %s step %.2f ms sigma %.3e" % (ph, mode, 1e3 * step_s, sp))
        hi[mode] = {"value": n / step_s, "ms_per_step": 1e3 * step_s, "sigma_phi_vs_direct": sp,
                    "sigma_field_vs_direct": sf}
    f, m = res["fp64"], res["mixed"]
    flops = f["sizes"]["m2l_flops"]
    dense = 2.0 * (p + 1) ** 4 * f["sizes"]["V"]
    m2l_ms = f["stages"]["m2l"]
    out = base_record(args)
    out.update({
        "value": n / f["step_s"], "ms_per_step": 1e3 * f["step_s"], "dtype": "f64",
        "config": {"workload": "Plummer sphere: N=%d, scale 0.05, truncated at r=1 (seed 2), q~U(-1,1), "
                               "adaptive octree s=64, p=10, potential+field" % n, "n": n, "order": p,
                   "tree": "adaptive s=64", "step": "fmm_plan + fmm_evaluate", "sizes": f["sizes"]},
        "accuracy": {"sigma_phi_vs_direct": f["sigma"], "sigma_field_vs_direct": f["sigma_f"],
                     "targets_sampled": 1000},
        "eval_only": {"value": n / f["eval_s"], "ms": 1e3 * f["eval_s"]},
        "stage_ms": f["stages"],
        "roofline": {"kernel": "k_m2l_sym<10,double>", "bound": "mfma", "achieved": flops / (m2l_ms * 1e-3) / 1e12,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / (m2l_ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, "traffic": None,
                     "flops_per_launch": flops, "ms_per_launch": m2l_ms,
                     "work": "sign-class contraction (unpadded) + member butterflies",
                     "dense_harmonic_flops_per_launch": dense,
                     "dense_equivalent_tflops": dense / (m2l_ms * 1e-3) / 1e12},
        "p2p": {"kernel": "k_p2p<0>", "pairs_per_launch": f["sizes"]["p2p_pairs"],
                "pairs_per_s": f["sizes"]["p2p_pairs"] / (1e-3 * f["stages"]["p2p"]),
                "achieved": P2P_FLOPS_PER_PAIR * f["sizes"]["p2p_pairs"] / (1e-3 * f["stages"]["p2p"]) / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s (FP64 vector)"},
        "mixed": {"value": n / m["step_s"], "ms_per_step": 1e3 * m["step_s"], "eval_ms": 1e3 * m["eval_s"],
                  "sigma_phi_vs_direct": m["sigma"], "sigma_field_vs_direct": m["sigma_f"],
                  "rel_l2_vs_fp64_path_phi": float(np.linalg.norm(m["phi"] - f["phi"]) / np.linalg.norm(f["phi"])),
                  "rel_l2_vs_fp64_path_field": float(np.linalg.norm(m["fld"] - f["fld"]) / np.linalg.norm(f["fld"])),
                  "dtype": "f64 with f32 P2P terms (M2L stays FP64 at p=10)", "stage_ms": m["stages"]},
        "order_for_1e-7": {"order": ph, "fp64": hi["fp64"], "mixed": hi["mixed"]},
    })
    return out


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
    # evaluate-only, plans built once
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


def bench_serve(args):
    """Poisson stream through the continuous-batching server: N log-uniform in
    [1e3, 1e6], uniform or Plummer, rel. error in {1e-4, 1e-7, 1e-9} -> p in
    {4, 8, 12}; saturated throughput first, then arrival rates 0.25/0.5/0.75/0.9
    of it; p50/p99 latency per rate."""
    import torch
    from paper_2508_02626_amd import inputs, serve
    nreq, warm = args.requests, max(args.requests // 10, 5)
    reqs = [inputs.served_request(i) for i in range(nreq + warm)]
    ntot = sum(len(q) for _, q, _ in reqs[warm:])
    srv = serve.Server(hbm_budget_bytes=64 << 30, slots=4)
    # saturated: everything submitted at once
    futs = [srv.submit(x, q, e) for x, q, e in reqs[:warm]]
    [f.result() for f in futs]
    t0 = time.perf_counter()
    futs = [srv.submit(x, q, e) for x, q, e in reqs[warm:]]
    lat_sat = [f.result()[2] for f in futs]
    sat_s = time.perf_counter() - t0
    rate_sat = nreq / sat_s
    log("bench serve: saturated %.1f req/s, %.3e particles/s" % (rate_sat, ntot / sat_s))
    rates = {}
    for frac in (0.25, 0.5, 0.75, 0.9):
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
    out = base_record(args)
    out.update({
        "value": ntot / sat_s, "ms_per_step": 1e3 * sat_s / nreq, "dtype": "f64 (p=12) / mixed (p<=8)",
        "config": {"workload": "served Poisson stream: %d requests (+%d warm-up), N log-uniform in [1e3,1e6], "
                               "uniform or Plummer, rel. error {1e-4,1e-7,1e-9} -> p {4,8,12}, adaptive s=64, "
                               "4 slots, 64 GiB admission budget" % (nreq, warm), "requests": nreq},
        "saturated": dict(serve.latency_stats(lat_sat), requests_per_s=rate_sat),
        "latency_by_load": rates,
        "roofline": None,
    })
    return out


def bench_sweep(args):
    """Leaf-size and order sweep and the scaling with N, on the distribution
    of the paper's sweeps (3-D Gaussian, unit standard deviation, adaptive
    tree), plain FP64 path, one step = fmm_plan + fmm_evaluate.  For every N
    and p the leaf size with the shortest step is reported (the experiment
    behind the paper's optimal-s table); then the step time over N at
    p in {2, 6, 10} with that leaf size, and the slope of its log-log fit."""
    import torch
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
    # accuracy of each order against the direct sum at N = 1e6, best leaf size
    xh, qh = inputs.gaussian(1_000_000, 3)
    x = torch.tensor(xh, device="cuda:0")
    q = torch.tensor(qh, device="cuda:0")
    sigma = {}
    for p in orders:
        pl = fmm.Plan(x, p, leaf_size=best[1_000_000][p], precision="fp64")
        phi, fld = pl.evaluate(q)
        pl.close()
        sigma[p] = sampled_sigma(xh, qh, phi.cpu().numpy(), fld.cpu().numpy(), count=500)[0]
    del x, q
    # scaling with N at the best leaf size of the nearest swept N
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=N_DEFAULT)
    ap.add_argument("--workload", default="uniform1m", choices=["uniform1m", "plummer4m", "batch256", "serve", "sweep"])
    ap.add_argument("--requests", type=int, default=300)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs a solve on a single GPU "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2508_02626_amd import inputs
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.workload != "uniform1m":
        fn = {"plummer4m": bench_plummer, "batch256": bench_batch, "serve": bench_serve,
              "sweep": bench_sweep}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return
    n = args.n
    xh, qh = inputs.uniform(n, SEED)
    x = torch.tensor(xh, device="cuda:0")
    q = torch.tensor(qh, device="cuda:0")
    log("bench: n=%d depth=%d p=%d steps=%d warmup=%d" % (n, DEPTH, ORDER, args.steps, args.warmup))
    res = {}
    for mode in (["fp64"] if args.no_mixed else ["fp64", "mixed"]):
        r = run_mode(x, q, mode, args.steps, args.warmup, n)
        r["sigma_phi"], r["sigma_field"], r["sigma_targets"] = sampled_sigma(xh, qh, r["phi"], r["fld"])
        log("bench: %s step %.3f ms eval %.3f ms sigma %.3e" % (mode, 1e3 * r["step_s"], 1e3 * r["eval_s"],
                                                                r["sigma_phi"]))
        res[mode] = r
    f = res["fp64"]
    nv = f["sizes"]["V"]
    m2l_ms = f["stages"]["m2l"][0] / max(f["stages"]["m2l"][1], 1)
    flops = f["m2l_flops"]
    dense = 2.0 * (ORDER + 1) ** 4 * nv
    achieved = flops / (m2l_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": n / f["step_s"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * f["step_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "uniform cube: N=%d uniform in [0,1)^3 (seed %d), q~U(-1,1), uniform octree "
                               "depth 5 on [0,1]^3, order p=8, potential+field" % (n, SEED),
                   "n": n, "order": ORDER, "tree": "uniform depth 5", "step": "fmm_plan + fmm_evaluate"},
        "accuracy": {"sigma_phi_vs_direct": f["sigma_phi"], "sigma_field_vs_direct": f["sigma_field"],
                     "targets_sampled": f["sigma_targets"]},
        "eval_only": {"value": n / f["eval_s"], "ms": 1e3 * f["eval_s"]},
        "stage_ms": stage_avg(f["stages"]),
        "roofline": {"kernel": "k_m2l_sym<8,double>", "bound": "mfma", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": m2l_traffic(), "traffic_unit": "bytes per launch",
                     "flops_per_launch": flops, "ms_per_launch": m2l_ms,
                     "work": "sign-class contraction (unpadded) + member butterflies",
                     "dense_harmonic_flops_per_launch": dense,
                     "dense_equivalent_tflops": dense / (m2l_ms * 1e-3) / 1e12},
        "p2p": p2p_roofline(f),
    }
    if "mixed" in res:
        m = res["mixed"]
        mm = m["stages"]["m2l"][0] / max(m["stages"]["m2l"][1], 1)
        out["mixed"] = {"rel_l2_vs_fp64_path_phi": float(np.linalg.norm(m["phi"] - f["phi"]) / np.linalg.norm(f["phi"])),
                        "rel_l2_vs_fp64_path_field": float(np.linalg.norm(m["fld"] - f["fld"]) / np.linalg.norm(f["fld"])),
                        "value": n / m["step_s"], "ms_per_step": 1e3 * m["step_s"],
                        "eval_only_value": n / m["eval_s"], "eval_ms": 1e3 * m["eval_s"],
                        "sigma_phi_vs_direct": m["sigma_phi"], "sigma_field_vs_direct": m["sigma_field"],
                        "dtype": "f64 with f32 P2P terms and f32 MFMA M2L",
                        "stage_ms": stage_avg(m["stages"]),
                        "m2l_kernel": "k_m2l_sym<8,float>", "m2l_ms": mm,
                        "m2l_tflops": flops / (mm * 1e-3) / 1e12, "m2l_peak_fp32": FP32_PEAK_TFLOPS,
                        "p2p_pairs_per_s": m["sizes"]["p2p_pairs"] / (1e-3 * stage_avg(m["stages"])["p2p"])}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(xh, qh)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
