#!/usr/bin/env python3
"""Benchmark of the tree-force hot path on one MI355X.

One step = tree_build + compute_moments + build_interaction_lists +
eval_forces + eval_forces_adjoint on one synthetic batch whose inputs are
already resident in HBM. Prints one JSON line.

value = particle interactions (P2P pairs + M2P sink-cell pairs of the
forward lists) per second of whole step time. The line also carries
forces/s, the per-phase split (the library's phase timers: HIP events on its
stream), the adjoint/forward cost ratio, the RMS force error against direct
summation on sampled sinks, the roofline of each of the six interaction
kernels (forward pair and expansion, pair sink and source adjoint, expansion
sink and cell adjoint) at algorithmic flop counts, with the dominant one as
"roofline", a sub-record of the clustered 2^24 workload, and the CPU
oracle's rate on a bounded sample.
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


def nm(p):
    return (p + 1) * (p + 2) * (p + 3) // 6


def comb(n, k):
    from math import comb as c
    return c(n, k)


# Algorithmic FP32 operations per interaction (FMA = 2, reciprocal square
# root = 1), from the formulas each kernel evaluates, independent of how the
# code is written:
#  pair forward: r = x_j - x_i (3), r^2 + eps^2 (3 FMA), rsq, m s^-3/2 (3 mul),
#    a += f r (3 FMA): the count of 20 per pair;
#  expansion forward at order p: derivatives of G to order p + 1 by the Hermite
#    recursion, 2 C(p+5, 4); the contraction with the moments, 3 components of
#    n_m(p) FMAs, 6 n_m(p); powers and rsq, p + 4;
#  pair adjoint, sink side: r, s, rsq as above (10), s^-3/2, s^-5/2, m s^-3/2
#    (3 mul), r . abar (1 mul + 2 FMA = 5), the r r^T coefficient (2 mul), the
#    running sums of m s^-3/2 (1) and of the r r^T term (3 FMA): 28;
#  pair adjoint, source side: r, s, rsq (10), s^-1, s^-3/2 (2 mul), r . b (5),
#    its coefficient (2 mul), the Hessian row (3 x 2 FMA = 12), the mass
#    cotangent (1 FMA): 33;
#  expansion adjoint, sink side: derivatives to order p + 2, 2 C(p+6, 4); the
#    six Hessian entries contracted with the moments, 6 n_m(p) FMAs = 12 n_m(p);
#    the Hessian times abar (9 mul-adds as 3 x (1 mul + 2 FMA) = 15); powers
#    and rsq, p + 5;
#  expansion adjoint, cell side: derivatives to order p + 1, 2 C(p+5, 4); the
#    moment cotangent row, n_m(p) entries of 3 FMAs, 6 n_m(p); p + 4.
FLOPS_P2P = 20
FLOPS_P2P_SINK_ADJ = 28
FLOPS_P2P_SRC_ADJ = 33


def flops_m2p(p):
    return 2 * comb(p + 5, 4) + 6 * nm(p) + (p + 4)


def flops_m2p_sink_adj(p):
    return 2 * comb(p + 6, 4) + 12 * nm(p) + 15 + (p + 5)


def flops_m2p_cell_adj(p):
    return 2 * comb(p + 5, 4) + 6 * nm(p) + (p + 4)


def git_head():
    """The checked-out commit, where the tree is a git checkout (else None)."""
    import subprocess
    try:
        r = subprocess.run(["git", "-C", ROOT, "rev-parse", "HEAD"], capture_output=True,
                           text=True, timeout=10)
        return r.stdout.strip() or None if r.returncode == 0 else None
    except Exception:
        return None


def tree_digest():
    """Digest of the library sources, the binding and this script: names the
    code a line was measured on where no git metadata travels with the tree."""
    csrc = os.path.join("paper_1310_4502_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(os.path.join(ROOT, csrc))
                   if f.endswith((".hip", ".h", ".py")))
    files += ["include/hot.h", "paper_1310_4502_amd/binding.py", "bench.py"]
    return source_digest(files)


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
    ap.add_argument("--err-sinks", type=int, default=4096,
                    help="sampled sinks of the direct-sum error check (a quarter of them for "
                         "the clustered sub-record)")
    ap.add_argument("--no-sub-clustered", dest="sub_clustered", action="store_false",
                    help="skip the clustered 2^24 sub-record")
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

    from paper_1310_4502_amd.binding import HOT_FP64, HOT_MIXED

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    prec = HOT_FP64 if args.precision == "fp64" else HOT_MIXED
    if args.background:
        args.periodic = True
    if args.periodic and args.err_tol is not None and args.background:
        print("--background and --err-tol are exclusive", file=sys.stderr)
        sys.exit(2)
    n_leaf, n_group, direct_max, desc = WORKLOADS[args.workload]
    n_leaf = args.n_leaf or n_leaf
    n_group = args.n_group or n_group
    direct_max = direct_max if args.direct_max is None else args.direct_max
    if args.background and args.direct_max is None:
        # accepted cells summed pair by pair outside the neighbourhood would
        # each need an exact box field: with subtraction they stay expansions
        direct_max = 0
    cfg = dict(n_leaf=n_leaf, n_group=n_group, direct_max=direct_max, periodic=args.periodic,
               background=args.background, bg_width=args.bg_width, err_tol=args.err_tol,
               prec=prec)
    m = measure(args.workload, cfg, args.steps, args.warmup, not args.no_fp64)
    w = m.pop("_w")
    tree, acc, acc64 = m.pop("_tree"), m.pop("_acc"), m.pop("_acc64")
    ms_step = m["ms_per_step"]
    out = {
        "metric": METRIC,
        "value": m["interactions_per_step"] / (ms_step * 1e-3),
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median_min_max": m.pop("ms_per_step_median_min_max"),
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
    }
    out.update(m)
    out["git_head"] = git_head()
    out["source_digest"] = tree_digest()
    out["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        out["cpu_baseline"], errs = cpu_baseline(
            w, {"mixed": acc, "fp64": acc64}, n_leaf, n_group, direct_max, args.cpu_groups,
            args.err_sinks, args.err_tol, args.periodic,
            args.bg_width if args.background else None)
        key = "rms_err_vs_oracle_treecode" if args.periodic else "rms_err_vs_direct"
        out[key] = errs.get("mixed" if prec == HOT_MIXED else "fp64")
        out["err_sinks"] = errs.get("n_sinks")
        if acc64 is not None:
            out[key + "_fp64"] = errs["fp64"]
        # per-particle relative errors of the evaluated precision
        pp = errs.get("per_particle_" + ("mixed" if prec == HOT_MIXED else "fp64"))
        if pp is not None:
            out[key.replace("rms_", "") + "_per_particle_median_p99"] = pp
    del tree, acc, acc64
    if args.sub_clustered and args.workload != "clustered16m" and not args.periodic \
            and args.err_tol is None:
        # the clustered 2^24 set in its own configuration, same step, fewer steps
        cl, cd, cdm, cdesc = WORKLOADS["clustered16m"]
        ccfg = dict(n_leaf=cl, n_group=cd, direct_max=cdm, periodic=False, background=False,
                    bg_width=3, err_tol=None, prec=prec)
        torch.cuda.empty_cache()
        cm = measure("clustered16m", ccfg, 5, 2, not args.no_fp64)
        cw = cm.pop("_w")
        cacc, cacc64 = cm.pop("_acc"), cm.pop("_acc64")
        cm.pop("_tree")
        cm.pop("ms_per_step_median_min_max", None)
        cm["workload"] = f"clustered16m: {cdesc}"
        cm["config"] = {"n": cw.n, "p": cw.p, "theta": cw.theta, "eps": cw.eps, "n_leaf": cl,
                        "n_group": cd, "direct_max": cdm, "steps": 5, "warmup": 2}
        cm["interactions_per_s"] = cm["interactions_per_step"] / (cm["ms_per_step"] * 1e-3)
        if not args.no_cpu_baseline:
            cm["rms_err_vs_direct"], cm["rms_err_vs_direct_fp64"], cm["err_sinks"], pp = \
                direct_errors(cw, cacc, cacc64, args.err_sinks // 4)
            cm["err_vs_direct_per_particle_median_p99"] = pp
        out["clustered16m"] = cm
    print(json.dumps(out), flush=True)


def measure(name, cfg, steps, warmup, with_fp64):
    """Times `steps` whole steps of workload `name` after `warmup` ones and
    returns the figures of the line (plus the last tree and forces under
    keys starting with _)."""
    import numpy as np
    import torch

    from paper_1310_4502_amd import workloads as W
    from paper_1310_4502_amd.binding import HOT_FP64, HOT_MIXED, Tree, context

    prec = cfg["prec"]
    t0 = time.time()
    w = W.make(name)
    log(f"workload {name}: N={w.n} generated in {time.time() - t0:.1f}s")
    if cfg["periodic"]:
        w.pos = np.ascontiguousarray(w.pos % 1.0)
        w.box = (0.0, 0.0, 0.0, 1.0)
    pos = torch.from_numpy(w.pos).cuda()
    mass = torch.from_numpy(w.mass).cuda()
    abar = torch.from_numpy(W.cotangent(w.n, 404)).cuda()
    torch.cuda.synchronize()
    ctx = context(pos.device.index or 0)
    err_tol, dmax = cfg["err_tol"], cfg["direct_max"]

    def step():
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        evs[3].record()
        t = Tree(pos, cfg["n_leaf"], cfg["n_group"], w.box, ctx=ctx)
        t.compute_moments(pos, mass, w.p)
        if cfg["background"]:
            t.build_interaction_lists_periodic_bs(w.theta, dmax, cfg["bg_width"])
        elif cfg["periodic"] and err_tol is not None:
            t.build_interaction_lists_periodic_err(mass, err_tol, w.p, dmax)
        elif cfg["periodic"]:
            t.build_interaction_lists_periodic(w.theta, dmax)
        elif err_tol is None:
            t.build_interaction_lists(w.theta, dmax)
        else:
            t.build_interaction_lists_err(mass, err_tol, w.p, dmax)
        ev0, ev1, ev2 = evs[:3]
        ev0.record()
        acc, _, st = t.eval_forces(pos, mass, w.eps, prec, stats=True)
        ev1.record()
        xbar, _ = t.eval_forces_adjoint(pos, mass, w.eps, abar, prec)
        ev2.record()
        return t, acc, xbar, st, evs

    for k in range(warmup):
        t, *_ = step()
        del t
        torch.cuda.synchronize()
        log(f"{name}: warmup step {k + 1}/{warmup} done")

    ctx.set_timing(True)
    recs, phases = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(steps):
        t, acc, xbar, st, evs = step()
        # the phases of this step (waits for the stream: the step is over)
        phases.append(ctx.timings())
        recs.append((st.ms_total, st.p2p_pairs, st.m2p_pairs, evs))
        last = (t, acc, xbar)
        log(f"{name}: timed step {k + 1}/{steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ctx.set_timing(False)
    ms_step = 1000.0 * elapsed / steps
    ph = {k: float(np.mean([p[k] for p in phases if k in p]))
          for k in phases[0] if all(k in p for p in phases)}
    ms_fwd_eval = float(np.mean([r[0] for r in recs]))
    ms_adj = float(np.mean([r[3][1].elapsed_time(r[3][2]) for r in recs]))
    step_ms = [r[3][3].elapsed_time(r[3][2]) for r in recs]
    # the forward path alone: tree build, moments, lists and eval_forces
    fwd_ms = float(np.mean([r[3][3].elapsed_time(r[3][1]) for r in recs]))
    p2p_pairs, m2p_pairs = recs[-1][1], recs[-1][2]
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
    ms_adj_cached, _ = timed(lambda: tree.eval_forces_adjoint(pos, mass, w.eps, abar, prec))
    acc64, ms_eval64 = None, None
    if prec == HOT_MIXED and with_fp64:
        ms_eval64, r64 = timed(lambda: tree.eval_forces(pos, mass, w.eps, HOT_FP64))
        acc64 = r64[0]
        log(f"{name}: fp64 eval on the same lists: {ms_eval64:.1f} ms")

    # algorithmic flops of the expansion kernels: per entry at its order
    # (error-bound lists) or at p, times the sinks of its group
    if err_tol is None:
        q_pairs = {w.p: m2p_pairs}
        orders = None
    else:
        _, _, mo, _ = tree.lists()
        q = tree.m2p_orders()
        gcount = tree.cells()["count"][tree.groups()].astype(np.int64)
        per_entry = np.repeat(gcount, np.diff(mo))
        q_pairs = {int(k): int(per_entry[q == k].sum()) for k in np.unique(q)}
        orders = np.bincount(q, minlength=w.p + 1).tolist()
    kern = {
        "p2p": ("eval_p2p", p2p_pairs * FLOPS_P2P, FLOPS_P2P),
        "m2p": ("eval_m2p", sum(n * flops_m2p(k) for k, n in q_pairs.items()), None),
        "p2p_sink_adj": ("adj_p2p_sink", p2p_pairs * FLOPS_P2P_SINK_ADJ, FLOPS_P2P_SINK_ADJ),
        "p2p_src_adj": ("adj_p2p_source", p2p_pairs * FLOPS_P2P_SRC_ADJ, FLOPS_P2P_SRC_ADJ),
        "m2p_sink_adj": ("adj_m2p_sink", sum(n * flops_m2p_sink_adj(k)
                                            for k, n in q_pairs.items()), None),
        "m2p_cell_adj": ("adj_m2p_cell", sum(n * flops_m2p_cell_adj(k)
                                            for k, n in q_pairs.items()), None),
    }
    rooflines = {}
    for k, (phase, flops, per) in kern.items():
        if phase not in ph or ph[phase] <= 0:
            continue
        n_int = p2p_pairs if k.startswith("p2p") else m2p_pairs
        achieved = flops / (ph[phase] * 1e-3) / 1e12
        rooflines[k] = {"bound": "alu", "achieved": round(achieved, 3),
                        "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                        "flops_per_interaction": (per if per is not None else
                                                  round(flops / max(n_int, 1), 1)),
                        "interactions": int(n_int), "ms_per_launch": round(ph[phase], 3)}
        # HBM bytes per launch from the committed counter records, which cover
        # the default lists of the default workload only
        rooflines[k]["traffic"] = (
            traffic_from_profiles(f"{k}_p{w.p}" if k.startswith("m2p") else k)
            if (name == "zeldovich16m" and err_tol is None and not cfg["periodic"])
            else None)
    dom = max(rooflines, key=lambda k: rooflines[k]["ms_per_launch"])
    roofline = dict(rooflines[dom])
    roofline["kernel"] = dom
    res = {
        "ms_per_step": ms_step,
        "ms_per_step_median_min_max": [float(np.median(step_ms)), float(np.min(step_ms)),
                                       float(np.max(step_ms))],
        "interactions_per_step": inter,
        "forces_per_s": w.n / (ms_step * 1e-3),
        "ms_forward_path": fwd_ms,
        "forces_per_s_forward_path": w.n / (fwd_ms * 1e-3),
        "forces_per_s_eval": w.n / (ms_fwd_eval * 1e-3),
        "p2p_pairs": p2p_pairs,
        "m2p_pairs": m2p_pairs,
        "ms_eval_forces": ms_fwd_eval,
        "ms_p2p": ph.get("eval_p2p"),
        "ms_m2p": ph.get("eval_m2p"),
        "ms_phases": {k: round(v, 3) for k, v in ph.items()},
        "ms_adjoint": ms_adj,
        "adjoint_over_eval": ms_adj / ms_fwd_eval if ms_adj and ms_fwd_eval > 0 else None,
        "ms_adjoint_lists_cached": ms_adj_cached,
        "adjoint_over_eval_lists_cached": (ms_adj_cached / ms_fwd_eval
                                           if ms_adj_cached and ms_fwd_eval > 0 else None),
        "ms_eval_forces_fp64": ms_eval64,
        "fp64_over_mixed_eval": ms_eval64 / ms_fwd_eval if ms_eval64 else None,
        "interactions_per_s_eval": inter / (ms_fwd_eval * 1e-3),
        "p2p_gflops_28flop_convention": (p2p_pairs * 28 / (ph["eval_p2p"] * 1e-3) / 1e9
                                         if ph.get("eval_p2p") else None),
        "tree": {k: counts[k] for k in ("n_cells", "n_groups", "n_leaves", "max_level",
                                        "n_p2p", "n_m2p", "n_items", "n_boxes")},
        "roofline": roofline,
        "rooflines": rooflines,
        "m2p_orders": orders,
        "_w": w, "_tree": tree, "_acc": acc, "_acc64": acc64,
    }
    return res


def direct_errors(w, acc, acc64, n_err):
    """Relative RMS errors of the mixed and FP64 forces against the oracle's
    direct sum on n_err sampled sinks, and the mixed per-particle median and
    99th percentile."""
    import numpy as np

    import oracle
    from paper_1310_4502_amd import workloads as W
    es = W.sample_indices(w.n, n_err, 102)
    t2 = time.time()
    ad, _ = oracle.direct(w.pos, w.mass, w.eps, sinks=es)
    a = acc.cpu().numpy()[es]
    e = float(np.linalg.norm(a - ad) / np.linalg.norm(ad))
    rel = np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)
    e64 = None
    if acc64 is not None:
        e64 = float(np.linalg.norm(acc64.cpu().numpy()[es] - ad) / np.linalg.norm(ad))
    log(f"{w.name}: direct-sum check on {n_err} sinks in {time.time() - t2:.1f}s: {e}, fp64 {e64}")
    return e, e64, int(n_err), [float(np.median(rel)), float(np.percentile(rel, 99))]


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
    errs["n_sinks"] = int(n_err)
    log(f"direct-sum check on {n_err} sinks in {time.time() - t2:.1f}s: rel RMS "
        f"{ {k: v for k, v in errs.items() if k in ('mixed', 'fp64')} }")
    return base, errs


if __name__ == "__main__":
    main()
