#!/usr/bin/env python3
"""Benchmark of the tree-force hot path on one MI355X.

One step = tree_build + compute_moments + build_interaction_lists +
eval_forces + eval_forces_adjoint on one synthetic batch whose inputs are
already resident in HBM. Prints one JSON line.

value = particle interactions (P2P pairs + M2P sink-cell pairs of the
forward lists) per second of whole step time. The line also carries
forces/s, the per-kernel split, the adjoint/forward cost ratio, the RMS
force error against direct summation on sampled sinks, the roofline of the
dominant kernel (timed with HIP events on the library's stream) and the
CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle interactions/sec & forces/sec at ≤1e-3 RMS force err; "
          "adjoint/fwd cost")
FP32_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (n_leaf, n_group, direct_max, description)
    "zeldovich16m": (16, 96, 64, "2^24 particles, 256^3 grid displaced by a P(k)~k^-2 "
                                 "Gaussian field (RMS 0.3 cells), eps=2e-5, theta=0.5, p=8, "
                                 "forward + one adjoint VJP"),
    "clustered16m": (16, 256, 32, "2^24 particles, half in 512 Plummer halos, half uniform, "
                                 "eps=5e-5, theta=0.5, p=6"),
    "clustered4m": (16, 256, 32, "2^22 particles, half in 512 Plummer halos, half uniform, "
                                "eps=5e-5, theta=0.5, p=6"),
    "plummer1m": (16, 256, 16, "2^20 Plummer sphere a=1/16, eps=1e-4, theta=0.6, p=4"),
    "uniform4k": (16, 64, 0, "4096 uniform, eps=1e-3, theta=0.5, p=2"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_flops():
    """FP32 operations per interaction of the P2P and M2P kernels, counted
    from the code the generator emits (FMA = 2)."""
    sys.path.insert(0, os.path.join(ROOT, "paper_1310_4502_amd", "csrc"))
    import gen_expansions as ge
    return ge.flops_p2p(), {p: ge.flops_m2p(p) for p in range(9)}


def source_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_key)
    except Exception:
        return None
    if not rec:
        return None
    if rec.get("source_digest") != source_digest(rec.get("sources", [])):
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zeldovich16m", choices=sorted(WORKLOADS))
    ap.add_argument("--n-group", type=int, default=None)
    ap.add_argument("--n-leaf", type=int, default=None)
    ap.add_argument("--direct-max", type=int, default=None)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--periodic", action="store_true",
                    help="periodic boundaries: positions wrapped into the unit cube, which is "
                         "the periodic cell")
    ap.add_argument("--background", action="store_true",
                    help="periodic boundaries with background subtraction (implies "
                         "--periodic)")
    ap.add_argument("--bg-width", type=int, default=3,
                    help="background subtraction: side of each group's neighbourhood in group "
                         "sides (odd, 3 .. 9)")
    ap.add_argument("--err-tol", type=float, default=None,
                    help="error-bound lists with this absolute acceleration tolerance per "
                         "interaction (orders up to the workload's p) instead of theta lists")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 evaluation on the last tree (mixed/FP64 speed-up)")
    ap.add_argument("--cpu-groups", type=int, default=160,
                    help="sink groups evaluated by the CPU oracle sample")
    ap.add_argument("--err-sinks", type=int, default=256)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized buffer once (known traffic for the HBM "
                         "byte counters) and exit")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        a = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}))
        return

    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (got --gpus {args.gpus}): the force path of "
              "this library is single-GPU; see the sharding design notes.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1310_4502_amd import workloads as W
    from paper_1310_4502_amd.binding import HOT_FP64, HOT_MIXED, HotError, Tree

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n_leaf, n_group, direct_max, desc = WORKLOADS[args.workload]
    n_leaf = args.n_leaf or n_leaf
    n_group = args.n_group or n_group
    direct_max = direct_max if args.direct_max is None else args.direct_max
    if args.background and args.direct_max is None:
        # accepted cells summed pair by pair outside the neighbourhood would
        # each need an exact box field: with subtraction they stay expansions
        direct_max = 0
    prec = HOT_FP64 if args.precision == "fp64" else HOT_MIXED

    if args.background:
        args.periodic = True
    t0 = time.time()
    w = W.make(args.workload)
    log(f"workload {args.workload}: N={w.n} generated in {time.time() - t0:.1f}s")
    if args.periodic:
        if args.err_tol is not None and args.background:
            print("--background and --err-tol are exclusive", file=sys.stderr)
            sys.exit(2)
        w.pos = np.ascontiguousarray(w.pos % 1.0)
        w.box = (0.0, 0.0, 0.0, 1.0)
    pos = torch.from_numpy(w.pos).cuda()
    mass = torch.from_numpy(w.mass).cuda()
    abar = torch.from_numpy(W.cotangent(w.n, 404)).cuda()
    torch.cuda.synchronize()

    def step():
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        evs[3].record()
        t = Tree(pos, n_leaf, n_group, w.box)
        t.compute_moments(pos, mass, w.p)
        if args.background:
            t.build_interaction_lists_periodic_bs(w.theta, direct_max, args.bg_width)
        elif args.periodic and args.err_tol is not None:
            t.build_interaction_lists_periodic_err(mass, args.err_tol, w.p, direct_max)
        elif args.periodic:
            t.build_interaction_lists_periodic(w.theta, direct_max)
        elif args.err_tol is None:
            t.build_interaction_lists(w.theta, direct_max)
        else:
            t.build_interaction_lists_err(mass, args.err_tol, w.p, direct_max)
        ev0, ev1, ev2 = evs[:3]
        ev0.record()
        acc, _, st = t.eval_forces(pos, mass, w.eps, prec, stats=True)
        ev1.record()
        xbar, _ = t.eval_forces_adjoint(pos, mass, w.eps, abar, prec)
        ev2.record()
        return t, acc, xbar, st, evs

    for k in range(args.warmup):
        t, *_ = step()
        del t
        torch.cuda.synchronize()
        log(f"warmup step {k + 1}/{args.warmup} done")

    recs = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        t, acc, xbar, st, evs = step()
        recs.append((st.ms_p2p, st.ms_m2p, st.ms_total, st.p2p_pairs, st.m2p_pairs, evs))
        last = (t, acc, xbar)
        log(f"timed step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_step = 1000.0 * elapsed / args.steps
    ms_p2p = float(np.mean([r[0] for r in recs]))
    ms_m2p = float(np.mean([r[1] for r in recs]))
    ms_fwd_eval = float(np.mean([r[2] for r in recs]))
    ms_adj = float(np.mean([r[5][1].elapsed_time(r[5][2]) for r in recs]))
    step_ms = [r[5][3].elapsed_time(r[5][2]) for r in recs]
    # the forward path alone: tree build, moments, lists and eval_forces
    fwd_ms = float(np.mean([r[5][3].elapsed_time(r[5][1]) for r in recs]))
    p2p_pairs, m2p_pairs = recs[-1][3], recs[-1][4]
    inter = p2p_pairs + m2p_pairs
    tree, acc, xbar = last
    counts = tree.counts()

    # after the timed region, on the last step's tree: the adjoint again (its
    # transposed lists are now cached, so this excludes their construction) and
    # the FP64 evaluation on identical lists
    def timed(fn, reps=2):
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            r = fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return min(ts), r
    ms_adj_cached = None
    if xbar is not None:
        ms_adj_cached, _ = timed(lambda: tree.eval_forces_adjoint(pos, mass, w.eps, abar, prec))
    acc64, ms_eval64 = None, None
    if prec == HOT_MIXED and not args.no_fp64:
        ms_eval64, r64 = timed(lambda: tree.eval_forces(pos, mass, w.eps, HOT_FP64))
        acc64 = r64[0]
        log(f"fp64 eval on the same lists: {ms_eval64:.1f} ms")

    f_p2p, f_m2p = kernel_flops()
    if args.err_tol is None:
        m2p_flops = m2p_pairs * f_m2p[w.p]
        orders = None
    else:
        # per-entry orders: flops of each entry's order times its group's sinks
        _, _, mo, _ = tree.lists()
        q = tree.m2p_orders()
        gcount = tree.cells()["count"][tree.groups()].astype(np.int64)
        per_entry = np.repeat(gcount, np.diff(mo))
        fq = np.array([f_m2p[k] for k in range(9)], dtype=np.int64)
        m2p_flops = int((per_entry * fq[q]).sum())
        orders = np.bincount(q, minlength=w.p + 1).tolist()
    # dominant kernel: the longer of P2P and M2P in eval_forces
    if ms_m2p >= ms_p2p:
        dom, dom_ms, dom_flops = f"m2p_p{w.p}", ms_m2p, m2p_flops
    else:
        dom, dom_ms, dom_flops = "p2p", ms_p2p, p2p_pairs * f_p2p
    achieved = dom_flops / (dom_ms * 1e-3) / 1e12
    # the committed counter record covers the default (open, theta) lists only
    traffic = (traffic_from_profiles(dom) if args.err_tol is None and not args.periodic
               else None)
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": traffic, "kernel": dom,
                "flops_per_interaction": (round(m2p_flops / max(m2p_pairs, 1), 1)
                                          if dom.startswith("m2p") else f_p2p),
                "ms_per_launch": round(dom_ms, 3)}

    out = {
        "metric": METRIC,
        "value": inter / (ms_step * 1e-3),
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median_min_max": [float(np.median(step_ms)), float(np.min(step_ms)),
                                       float(np.max(step_ms))],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == HOT_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "n": w.n, "p": w.p,
                   "theta": w.theta if args.err_tol is None else None,
                   "err_tol": args.err_tol, "eps": w.eps, "n_leaf": n_leaf,
                   "n_group": n_group, "direct_max": direct_max, "precision": args.precision,
                   "boundary": (f"periodic, background subtracted (neighbourhood "
                                f"{args.bg_width} group sides)" if args.background else
                                "periodic" if args.periodic else "open")},
        "forces_per_s": w.n / (ms_step * 1e-3),
        "ms_forward_path": fwd_ms,
        "forces_per_s_forward_path": w.n / (fwd_ms * 1e-3),
        "forces_per_s_eval": w.n / (ms_fwd_eval * 1e-3),
        "p2p_pairs": p2p_pairs,
        "m2p_pairs": m2p_pairs,
        "ms_eval_forces": ms_fwd_eval,
        "ms_p2p": ms_p2p,
        "ms_m2p": ms_m2p,
        "ms_adjoint": ms_adj,
        "adjoint_over_eval": ms_adj / ms_fwd_eval if ms_adj and ms_fwd_eval > 0 else None,
        "ms_adjoint_lists_cached": ms_adj_cached,
        "adjoint_over_eval_lists_cached": (ms_adj_cached / ms_fwd_eval
                                           if ms_adj_cached and ms_fwd_eval > 0 else None),
        "ms_eval_forces_fp64": ms_eval64,
        "fp64_over_mixed_eval": ms_eval64 / ms_fwd_eval if ms_eval64 else None,
        "interactions_per_s_eval": inter / (ms_fwd_eval * 1e-3),
        "p2p_gflops_28flop_convention": p2p_pairs * 28 / (ms_p2p * 1e-3) / 1e9,
        "tree": {k: counts[k] for k in ("n_cells", "n_groups", "n_leaves", "max_level",
                                        "n_p2p", "n_m2p", "n_items", "n_boxes")},
        "roofline": roofline,
        "m2p_orders": orders,
        "cpu_baseline": None,
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"], errs = cpu_baseline(
            w, {"mixed": acc, "fp64": acc64}, n_leaf, n_group, direct_max, args.cpu_groups,
            args.err_sinks, args.err_tol, args.periodic,
            args.bg_width if args.background else None)
        key = "rms_err_vs_oracle_treecode" if args.periodic else "rms_err_vs_direct"
        out[key] = errs.get("mixed" if prec == HOT_MIXED else "fp64")
        if acc64 is not None:
            out[key + "_fp64"] = errs["fp64"]
        # per-particle relative errors of the evaluated precision
        pp = errs.get("per_particle_" + ("mixed" if prec == HOT_MIXED else "fp64"))
        if pp is not None:
            out[key.replace("rms_", "") + "_per_particle_median_p99"] = pp
    print(json.dumps(out), flush=True)


def cpu_baseline(w, accs, n_leaf, n_group, direct_max, n_groups_sample, n_err, err_tol=None,
                 periodic=False, bg_width=None):
    """The CPU oracle (FP64 scalar treecode, OpenMP) on a bounded sample of the
    same workload: its interaction rate over the sampled sinks' evaluation
    (tree build and moments excluded), plus the relative RMS error of each GPU
    result in `accs` against the oracle's direct summation on sampled sinks."""
    import numpy as np

    import oracle
    from paper_1310_4502_amd import workloads as W

    t0 = time.time()
    ot = oracle.Tree(w.pos, n_leaf, n_group, w.box)
    gof = ot.group_of()
    G = ot.counts()["n_groups"]
    groups = W.sample_indices(G, n_groups_sample, 77)
    if bg_width is not None:
        ot.build_lists_periodic_bs(w.theta, direct_max, width=bg_width, groups=groups)
    elif periodic and err_tol is not None:
        ot.build_lists_periodic_err(w.mass, err_tol, w.p, direct_max, groups=groups)
    elif periodic:
        ot.build_lists_periodic(w.theta, direct_max, groups=groups)
    elif err_tol is None:
        ot.build_lists(w.theta, direct_max, groups=groups)
    else:
        ot.build_lists_err(w.mass, err_tol, w.p, direct_max, groups=groups)
    po, pl, mo, ml = ot.lists()
    cells = np.unique(np.concatenate([ml[mo[g]:mo[g + 1]] for g in groups] + [np.zeros(1, int)]))
    ot.compute_moments(w.pos, w.mass, w.p, cells=cells)
    _, perm = ot.keys()
    sinks = np.sort(perm[np.isin(gof, groups)])
    log(f"cpu oracle: tree+lists+moments for {len(groups)} groups in {time.time() - t0:.1f}s")
    t1 = time.perf_counter()
    a_ot, _, cnt = ot.eval(w.pos, w.mass, w.eps, sinks=sinks, with_pot=False)
    dt = time.perf_counter() - t1
    inter = int(cnt[0] + cnt[1])
    cores = oracle.num_threads()
    log(f"cpu oracle: {len(sinks)} sinks, {inter} interactions in {dt:.1f}s on {cores} threads")
    # the same evaluation on one core, over the sinks of the first tenth of the sampled groups
    one = np.sort(perm[np.isin(gof, groups[:max(1, len(groups) // 10)])])
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    _, _, cnt1 = ot.eval(w.pos, w.mass, w.eps, sinks=one, with_pot=False)
    dt1 = time.perf_counter() - t1
    oracle.set_num_threads(cores)
    inter1 = int(cnt1[0] + cnt1[1])
    log(f"cpu oracle, one core: {len(one)} sinks, {inter1} interactions in {dt1:.1f}s")
    base = {"value": inter / dt, "unit": "interactions/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 scalar treecode (O-T) evaluation of {len(sinks)} sinks in "
                      f"{len(groups)} sampled groups of the same workload; tree build and "
                      f"moments not timed",
            "forces_per_s": len(sinks) / dt,
            "one_core": {"value": inter1 / dt1, "unit": "interactions/s",
                         "forces_per_s": len(one) / dt1, "sinks": len(one)}}
    errs = {}
    if periodic:
        # an Ewald direct sum over 2^24 sources is out of reach here: the
        # periodic result is compared with the oracle treecode on the same lists
        for k, acc in accs.items():
            if acc is not None:
                a = acc.cpu().numpy()[sinks]
                errs[k] = float(np.linalg.norm(a - a_ot) / np.linalg.norm(a_ot))
        log(f"periodic: rel RMS vs the oracle treecode on {len(sinks)} sinks: {errs}")
        return base, errs
    es = W.sample_indices(w.n, n_err, 102)
    t2 = time.time()
    ad, _ = oracle.direct(w.pos, w.mass, w.eps, sinks=es)
    for k, acc in accs.items():
        if acc is None:
            continue
        a = acc.cpu().numpy()[es]
        errs[k] = float(np.linalg.norm(a - ad) / np.linalg.norm(ad))
        rel = np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)
        errs["per_particle_" + k] = [float(np.median(rel)), float(np.percentile(rel, 99))]
    log(f"direct-sum check on {n_err} sinks in {time.time() - t2:.1f}s: rel RMS "
        f"{ {k: v for k, v in errs.items() if not k.startswith('per_particle')} }")
    return base, errs


if __name__ == "__main__":
    main()
