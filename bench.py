#!/usr/bin/env python3
"""Benchmark of the MI355X machine code: volume-potential unknowns/s, FP64, forward + adjoint.

    python bench.py [--gpus 1] [--steps 10] [--warmup 3] [--no-cpu-baseline] [--no-batched]

Workload (one "step" = one forward apply and one adjoint apply, every stage of the box code):
the adaptive 20-Gaussian source on the size-matched quadtree (background level 7, Chebyshev-
tail rule eps = 1e-11, 2:1 balanced; 16,837 leaves = 4.31M unknowns for seed 0), p = 16. Inputs
are resident in HBM before the timed region; plan and table construction are outside it.

The launch shape (tile sizes, split policy, stream overlap) is the autotuner's choice unless
given on the command line; tuning runs before the timed region. `value` comes from K steps with
nothing else recorded; the roofline of the dominant kernel (the near-field stage and its
transpose) from HIP events around its launches in a second pass of K steps.

Printed: one JSON line with the metric, the roofline, the CPU oracle timed on this host, and the
batched forest (256 uneven trees, hipGraph replay, autotuned) versus 256 sequential applies.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "volume-potential unknowns/s FP64 (rel err ≤1e-11), fwd+adjoint, batched vs serial"
PEAK_FP64_MFMA = 78.6e12  # MI355X dense FP64 matrix peak, FLOP/s
PEAK_HBM = 8.0e12  # bytes/s


def kernel_source_hash():
    """Hash of the sources that decide what the leaf-stage launches do: the kernels and the
    plan and scheduling code that cut the work into launches."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.hpp", "plan.cpp", "api.cpp"):
        with open(os.path.join(ROOT, "paper_2501_17967_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(shape):
    """HBM bytes per launch of the leaf-stage kernel from the committed counter summary, or
    None when the summary is missing or was taken on other sources or another launch shape."""
    path = os.path.join(ROOT, "profiles", "leaf_stage_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_source_hash() or d.get("launch_shape") != shape:
        return None
    return d.get("bytes_per_launch")


def _timed(fn, reps):
    import torch

    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - a) / reps


def _oracle_cores():
    try:
        from threadpoolctl import threadpool_info

        return int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))
    except Exception:
        return len(os.sched_getaffinity(0))


def layer_leg(args, dev):
    """The glue layer potentials S[sigma] - D[tau] (Sec. 4.4) at every node of the star-cut
    adaptive tree, from 512 panels of 24 nodes on the star pulled inwards."""
    import numpy as np
    import torch

    from workloads import gen

    from paper_2501_17967_amd import LayerPlan

    timed = _timed
    cores = _oracle_cores()

    print("bench: layer potentials", file=sys.stderr, flush=True)
    lw = gen.config3(0, lcut=10)
    curve = gen.star_curve(n_panels=512, order=24, scale=0.95, seed=1)
    t0 = time.perf_counter()
    lp = LayerPlan(lw.centres, lw.levels, curve.nodes, curve.weights, curve.normals)
    torch.cuda.synchronize()
    t_lplan = time.perf_counter() - t0
    sig = torch.from_numpy(curve.sigma).to(dev)
    tau = torch.from_numpy(curve.tau).to(dev)
    V = torch.empty((lw.n_leaves, 256), dtype=torch.float64, device=dev)
    for _ in range(3):
        lp.apply(sig, tau, out=V)
    t_lay = timed(lambda: lp.apply(sig, tau, out=V), max(5, args.steps))
    lp.set_timing(True)
    lp.stage_times()
    for _ in range(3):
        lp.apply(sig, tau, out=V)
    lst = lp.stage_times()
    lp.set_timing(False)
    linf = lp.info()
    n_t = lw.n_leaves * 256
    names = {"up": "prep+P2M+M2M", "down": "M2L+P2L+L2L", "near": "P2P", "loct": "L2T+M2T"}
    lay = {"workload": "star-cut adaptive tree (200 Gaussians, lcut 10) x star curve 512 panels x 24 nodes",
           "targets": n_t, "curve_nodes": curve.n_nodes, "ms": 1e3 * t_lay, "targets_per_s": n_t / t_lay,
           "plan_s": t_lplan, "source_leaves": linf["n_source_leaves"], "active_boxes": linf["n_active_boxes"],
           "pairs_direct": linf["pairs_p2p"],
           "stage_ms": {names[k]: round(v[0] / 3, 4) for k, v in lst.items() if v[1]}}
    if lst["near"][1]:
        lay["direct_pairs_per_s"] = linf["pairs_p2p"] / (lst["near"][0] / 3 * 1e-3)
    if not args.no_cpu_baseline:
        # the oracle (direct sum over all curve nodes) on a bounded sample of the targets,
        # which also checks the sampled values
        from oracle import layer as olayer

        tg = olayer.leaf_targets(lw.centres, lw.levels)
        idx = np.random.default_rng(args.seed + 2).choice(n_t, 50000, replace=False)
        t0 = time.perf_counter()
        ref = olayer.layer_potential(tg[idx], curve.nodes, curve.weights, curve.normals, curve.sigma, curve.tau)
        t_cpu = time.perf_counter() - t0
        got = V.reshape(-1)[torch.from_numpy(idx).to(dev)].cpu().numpy()
        lay["rel_err_vs_oracle_sampled"] = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        lay["cpu_baseline"] = {"value": idx.size / t_cpu, "unit": "targets/s", "cores": int(cores), "kind": "oracle",
                               "sample": "%d random leaf nodes, direct sum over all %d curve nodes: %.1f s"
                                         % (idx.size, curve.n_nodes, t_cpu)}
    lp.close()
    return lay


def points_leg(args, dev):
    """u and grad u at the nodes of a curve inside the star-cut adaptive tree (the values the
    glue step needs on the fictitious curve), in one forward apply of the volume potential."""
    import numpy as np
    import torch

    from paper_2501_17967_amd import PointPlan
    from workloads import gen

    print("bench: off-grid points", file=sys.stderr, flush=True)
    pw = gen.config3(0, lcut=10)
    curve = gen.star_curve(n_panels=128, order=24, scale=0.95, seed=1)
    t0 = time.perf_counter()
    pp = PointPlan(pw.centres, pw.levels, curve.nodes, overlap=32)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    f = torch.from_numpy(pw.f).to(dev)
    u = torch.empty_like(f)
    for _ in range(3):
        pp.apply_points(f, out=u)
        pp.apply(f, out=u)
    reps = max(10, args.steps)
    t_pts = _timed(lambda: pp.apply_points(f, out=u), reps)
    t_app = _timed(lambda: pp.apply(f, out=u), reps)
    _, up, gp = pp.apply_points(f, out=u)
    torch.cuda.synchronize()
    inf = pp.info()
    res = {"workload": "star-cut adaptive tree (200 Gaussians, lcut 10), u and grad u at the 3,072 nodes of a "
                       "128-panel star curve", "points": curve.n_nodes, "pairs": inf["pairs_points"],
           "plan_s": t_plan, "ms_apply": 1e3 * t_app, "ms_apply_points": 1e3 * t_pts,
           "points_per_s": curve.n_nodes / max(t_pts - t_app, 1e-9)}
    if not args.no_cpu_baseline:
        from oracle import quad, tree

        idx = np.random.default_rng(args.seed + 3).choice(curve.n_nodes, 60, replace=False)
        T = tree.Tree(pw.centres, pw.levels)
        t0 = time.perf_counter()
        u_o, g_o = quad.potential_at_points(pw.centres, T.halfw, pw.f, curve.nodes[idx], grad=True)
        t_cpu = time.perf_counter() - t0
        ug = up.cpu().numpy()[idx]
        gg = gp.cpu().numpy()[idx]
        res["rel_err_vs_oracle_sampled"] = {"u": float(np.max(np.abs(ug - u_o)) / np.max(np.abs(u_o))),
                                            "grad": float(np.max(np.abs(gg - g_o)) / np.max(np.abs(g_o)))}
        res["cpu_baseline"] = {"value": idx.size / t_cpu, "unit": "points/s", "cores": _oracle_cores(), "kind": "oracle",
                               "sample": "%d random curve nodes, u and grad u by adaptive quadrature over all %d "
                                         "leaves: %.1f s" % (idx.size, pw.n_leaves, t_cpu)}
    pp.close()
    return res


def tree_leg(args, dev):
    """Adaptive quadtree construction (Sec. 4.2.1) of the size-matched 20-Gaussian workload on
    the GPU: the source is sampled by a torch expression on the device, the tail tests run in
    the library; against the oracle builder (NumPy) on the host, whose leaves must be the same."""
    import numpy as np
    import torch

    from paper_2501_17967_amd import build_tree
    from workloads import gen

    print("bench: quadtree construction", file=sys.stderr, flush=True)
    g = gen.sample_gaussians(np.random.default_rng(args.seed), 20, -0.9, 0.9, 1e-3, 1e-1)
    C = torch.tensor(g.centres, device=dev)
    S2 = torch.tensor(2.0 * g.sigmas ** 2, device=dev)
    A = torch.tensor(g.amps, device=dev)

    def f_dev(p):
        d2 = (p[:, None, 0] - C[None, :, 0]) ** 2 + (p[:, None, 1] - C[None, :, 1]) ** 2
        return (A[None, :] * torch.exp(-d2 / S2[None, :])).sum(dim=1)

    build_tree(f_dev, 1e-11, g.scale, 7, 24)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, lv = build_tree(f_dev, 1e-11, g.scale, 7, 24)
    t_gpu = time.perf_counter() - t0
    res = {"workload": "20 Gaussians (sigma log-U[1e-3, 1e-1]), eps 1e-11, min level 7: the size-matched tree",
           "leaves": int(lv.size), "max_level": int(lv.max()), "s": t_gpu, "leaves_per_s": lv.size / t_gpu}
    if not args.no_cpu_baseline:
        from oracle import quadtree as qt

        def f_np(p):
            out = np.zeros(p.shape[0])
            for cc, s, a in zip(g.centres, g.sigmas, g.amps):
                out += a * np.exp(-((p[:, 0] - cc[0]) ** 2 + (p[:, 1] - cc[1]) ** 2) / (2 * s * s))
            return out

        t0 = time.perf_counter()
        ref = qt.build(f_np, 1e-11, g.scale, 7, 24)
        t_cpu = time.perf_counter() - t0
        s = 2.0 ** (-lv.astype(float))
        got = {(int(a), int(x), int(y)) for a, x, y in zip(lv, np.round((c[:, 0] + 1) / (2 * s) - 0.5),
                                                             np.round((c[:, 1] + 1) / (2 * s) - 0.5))}
        res["same_leaves_as_oracle"] = got == set(ref)
        res["cpu_baseline"] = {"value": len(ref) / t_cpu, "unit": "leaves/s", "cores": 1, "kind": "oracle",
                               "sample": "the whole construction by the oracle builder: %.1f s" % t_cpu}
    return res


def strip_leg(args, dev):
    """Strip solve (Sec. 4.3) at the size of the paper's raindrop strip: 56 elements of 24 nodes
    along the panel by 16 across (21,504 unknowns), here between the star (56 panels of 16
    Gauss-Legendre nodes) and the star pulled inwards by 7 %. Plan (host factorization) outside
    the timed apply; against the oracle's dense row-equilibrated solve of the same system."""
    import numpy as np
    import torch

    from paper_2501_17967_amd import StripPlan
    from workloads import gen

    print("bench: strip solve", file=sys.stderr, flush=True)
    n, q, n_r = 56, 24, 16
    g = gen.star_curve(n_panels=n, order=16, scale=1.0).nodes.reshape(n, 16, 2)
    gt = gen.star_curve(n_panels=n, order=16, scale=0.93).nodes.reshape(n, 16, 2)
    f_np = lambda p: np.sin(3 * p[:, 0]) * np.exp(p[:, 1]) + 0.5
    t0 = time.perf_counter()
    sp = StripPlan(g, gt, q, n_r)
    torch.cuda.synchronize()
    t_plan_first = time.perf_counter() - t0
    sp.close()
    t0 = time.perf_counter()  # a second plan: host assembly, GPU inversion, host chain, GPU blocks
    sp = StripPlan(g, gt, q, n_r)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    f = torch.from_numpy(f_np(sp.nodes.reshape(-1, 2))).to(dev)
    v = torch.empty(sp.shape, dtype=torch.float64, device=dev)
    for _ in range(5):
        sp.apply(f, out=v)
    t_app = _timed(lambda: sp.apply(f, out=v), max(50, args.steps))
    N = n * q * n_r
    B, m = q * n_r, n_r - 2
    Bi = m * q
    # algorithmic HBM bytes of one apply: the interior blocks of the inverses (n Bi^2), the
    # right-hand-side functionals (n 2m Bi), the sweep and response matrices F, G, H, Pz, Pt
    # (6 n m^2), f and the row scales read twice (4 n Bi), v written (N), the sweep vectors
    bytes_apply = 8 * (n * Bi * Bi + 2 * m * n * Bi + 6 * n * m * m + 4 * n * Bi + N + 8 * n * m)
    res = {"workload": "strip of 56 elements at 24 x 16 (21,504 unknowns) between the star and the star pulled "
                       "inwards by 7 %", "unknowns": N, "plan_s": t_plan, "plan_s_first": t_plan_first, "ms_apply": 1e3 * t_app,
           "unknowns_per_s": N / t_app, "bytes_per_apply": bytes_apply,
           "hbm_frac_whole_apply": bytes_apply / t_app / PEAK_HBM}
    if not args.no_cpu_baseline:
        from oracle import strip

        t0 = time.perf_counter()
        ref, _ = strip.solve(g, gt, f_np, q=q, n_r=n_r)
        t_cpu = time.perf_counter() - t0
        vv = v.cpu().numpy()
        res["rel_err_vs_oracle"] = float(np.max(np.abs(vv - ref)) / np.max(np.abs(ref)))
        res["cpu_baseline"] = {"value": N / t_cpu, "unit": "unknowns/s", "cores": _oracle_cores(), "kind": "oracle",
                               "sample": "the whole strip by the oracle (assembly and dense solve): %.1f s" % t_cpu}
    sp.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-layer", action="store_true", help="skip the layer-potential evaluation leg")
    ap.add_argument("--layer-only", action="store_true",
                    help="run only the layer-potential leg and print its object (for profiling)")
    ap.add_argument("--no-points", action="store_true", help="skip the off-grid evaluation leg")
    ap.add_argument("--points-only", action="store_true",
                    help="run only the off-grid evaluation leg and print its object (for profiling)")
    ap.add_argument("--no-tree", action="store_true", help="skip the quadtree construction leg")
    ap.add_argument("--tree-only", action="store_true",
                    help="run only the quadtree construction leg and print its object (for profiling)")
    ap.add_argument("--no-strip", action="store_true", help="skip the strip-solve leg")
    ap.add_argument("--strip-only", action="store_true",
                    help="run only the strip-solve leg and print its object (for profiling)")
    ap.add_argument("--batched-trees", type=int, default=256)
    ap.add_argument("--tile-leaf", type=int, default=0, help="0: chosen by the autotuner")
    ap.add_argument("--tile-box", type=int, default=0, help="0: chosen by the autotuner")
    ap.add_argument("--split-min", type=int, default=None, help="default: chosen by the autotuner")
    ap.add_argument("--overlap", type=int, default=None, help="default: chosen by the autotuner")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run 5 device-to-device copies of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the box code runs on one GPU only (it has no multi-GPU path); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_mib": args.calibrate_copy_mib, "copies": 5}))
        return

    if args.layer_only:
        print(json.dumps({"layer_potential": layer_leg(args, torch.device("cuda:0"))}), flush=True)
        return
    if args.strip_only:
        print(json.dumps({"strip": strip_leg(args, torch.device("cuda:0"))}), flush=True)
        return
    if args.points_only:
        print(json.dumps({"points": points_leg(args, torch.device("cuda:0"))}), flush=True)
        return
    if args.tree_only:
        print(json.dumps({"tree": tree_leg(args, torch.device("cuda:0"))}), flush=True)
        return

    from paper_2501_17967_amd import Plan, autotune
    from workloads import gen

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = gen.config2(args.seed, size_matched=True)
    t_gen = time.perf_counter() - t0
    # launch shape: the autotuner's choice unless fixed on the command line (outside the timed region)
    t0 = time.perf_counter()
    if args.tile_leaf and args.tile_box and args.split_min is not None and args.overlap is not None:
        shape = {}
    else:
        shape, _ = autotune(w.centres, w.levels)
    t_tune = time.perf_counter() - t0
    if args.tile_leaf:
        shape["tile_leaf"] = args.tile_leaf
    if args.tile_box:
        shape["tile_box"] = args.tile_box
    if args.split_min is not None:
        shape["split_min"] = args.split_min
    if args.overlap is not None:
        shape["overlap"] = args.overlap
    print("bench: launch shape %s (autotuner %.1fs)" % (shape, t_tune), file=sys.stderr, flush=True)
    plan_shape = {"tile_leaf": 32, "tile_box": 32, "split_min": 0, "overlap": 0}
    plan_shape.update(shape)
    t0 = time.perf_counter()
    plan = Plan(w.centres, w.levels, **plan_shape)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    info = plan.info()
    N = w.unknowns
    print("bench: %s, %d leaves, %d unknowns, max level %d; gen %.1fs plan %.2fs"
          % (w.name, w.n_leaves, N, info["max_level"], t_gen, t_plan), file=sys.stderr, flush=True)

    f = torch.from_numpy(w.f).to(dev)
    rng = np.random.default_rng(args.seed + 1)
    ubar = torch.from_numpy(rng.standard_normal(w.f.shape)).to(dev)
    u = torch.empty_like(f)
    fbar = torch.empty_like(f)
    for _ in range(args.warmup):
        plan.apply(f, out=u)
        plan.apply_adjoint(ubar, out=fbar)
    torch.cuda.synchronize()

    # timed region: K steps of forward + adjoint, nothing else recorded (with the overlap
    # option, event records between launches on the caller's stream delay the concurrent
    # far-field chain: about 15% of the step)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(f, out=u)
        plan.apply_adjoint(ubar, out=fbar)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_step = 1e3 * t_total / args.steps
    value = N * args.steps / t_total

    # roofline pass: the same K steps again, HIP events around the launches of the dominant
    # kernel only (the near-field stage and its transpose), on the stream they run on
    plan.set_timing(True, kinds=("near", "adj_near"))
    plan.stage_times()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(f, out=u)
        plan.apply_adjoint(ubar, out=fbar)
    torch.cuda.synchronize()
    t_events = time.perf_counter() - t0
    st = plan.stage_times()
    plan.set_timing(False)

    # forward-only and adjoint-only throughput (no timing events)
    def timed(fn, reps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / reps

    t_fwd = timed(lambda: plan.apply(f, out=u), args.steps)
    t_adj = timed(lambda: plan.apply_adjoint(ubar, out=fbar), args.steps)

    # roofline of the dominant kernel: the near-field stage (forward) and its transpose
    # (adjoint) -- the same kernel instantiation, one launch each per step
    # (with the overlap option the near field of each apply runs as two launches)
    leaf_ms = st["near"][0] + st["adj_near"][0]
    leaf_n = st["near"][1] + st["adj_near"][1]
    launches_per_step = leaf_n / args.steps
    flops_per_launch = (info["flops_kind"]["near"] + info["flops_kind"]["adj_near"]) / launches_per_step
    avg_ms = leaf_ms / max(leaf_n, 1)
    achieved = flops_per_launch / (avg_ms * 1e-3)
    traffic = traffic_from_profile(plan_shape)
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64_MFMA / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_MFMA, "traffic": traffic,
                "kernel": "grg_kernel, 256-row tiles: near-field stage (forward) and its transpose (adjoint)",
                "flops_per_launch": flops_per_launch, "avg_launch_ms": avg_ms, "launches": leaf_n,
                "launches_per_step": launches_per_step,
                "timed_in": "a second pass of the same steps, right after the timed region",
                "pass_ms_per_step": 1e3 * t_events / args.steps}
    # per-stage breakdown: a separate pass with every launch timed (events perturb the overlap)
    plan.set_timing(True)
    plan.stage_times()
    for _ in range(args.steps):
        plan.apply(f, out=u)
        plan.apply_adjoint(ubar, out=fbar)
    stb = plan.stage_times()
    plan.set_timing(False)
    stage_ms = {k: v[0] / args.steps for k, v in stb.items()}
    whole = (info["flops_total"] + info["flops_adjoint"]) / (t_total / args.steps)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name + " (adaptive 20-Gaussian source, size-matched quadtree, seed %d)" % args.seed,
                   "n_leaves": int(w.n_leaves), "unknowns": int(N), "max_level": int(info["max_level"]), "p": 16,
                   "expansion_order": int(info["order"]), "step": "forward + adjoint",
                   "launch_shape": plan_shape, "autotune_s": t_tune},
        "roofline": roofline,
        "fwd_unknowns_per_s": N / t_fwd,
        "adj_unknowns_per_s": N / t_adj,
        "whole_path_tflops": whole / 1e12,
        "stage_ms_per_step": stage_ms,
        "plan_s": t_plan,
    }

    if not args.no_cpu_baseline:
        from oracle import fmm, tree

        print("bench: cpu baseline (oracle box code on the same workload)", file=sys.stderr, flush=True)
        try:
            from threadpoolctl import threadpool_info

            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = len(os.sched_getaffinity(0))
        bc = fmm.BoxCode(tree.Tree(w.centres, w.levels))
        ub = ubar.cpu().numpy()
        t_runs = []
        for _ in range(3):
            a = time.perf_counter()
            u_o = bc.apply(w.f)
            fb_o = bc.apply_adjoint(ub)
            t_runs.append(time.perf_counter() - a)
        t_cpu = sorted(t_runs)[1]
        u_g = u.cpu().numpy()
        fb_g = fbar.cpu().numpy()
        out["cpu_baseline"] = {"value": N / t_cpu, "unit": "unknowns/s", "cores": int(cores), "kind": "oracle",
                               "sample": "the full workload, one forward + one adjoint apply of the oracle box "
                                         "code (NumPy, order 50), median of 3 runs: %.2f s each" % t_cpu}
        out["rel_err_vs_oracle"] = {
            "forward": float(np.max(np.abs(u_g - u_o)) / np.max(np.abs(u_o))),
            "adjoint": float(np.max(np.abs(fb_g - fb_o)) / np.max(np.abs(fb_o)))}

    if not args.no_batched:
        print("bench: batched forest of %d trees" % args.batched_trees, file=sys.stderr, flush=True)
        trees = gen.config4(0, n_trees=args.batched_trees)
        off = np.cumsum([0] + [t.n_leaves for t in trees])
        Nb = int(off[-1]) * 256
        C = np.vstack([t.centres for t in trees])
        Lv = np.concatenate([t.levels for t in trees])
        t0 = time.perf_counter()
        fshape, _ = autotune(C, Lv, tree_offsets=off)
        t_ftune = time.perf_counter() - t0
        print("bench: forest launch shape %s (autotuner %.1fs)" % (fshape, t_ftune), file=sys.stderr, flush=True)
        forest = Plan(C, Lv, tree_offsets=off, use_graph=True, **fshape)
        F = torch.from_numpy(np.vstack([t.f for t in trees])).to(dev)
        Ub = torch.empty_like(F)
        Fb = torch.empty_like(F)
        for _ in range(2):
            forest.apply(F, out=Ub)
            forest.apply_adjoint(F, out=Fb)
        reps = max(3, args.steps // 2)
        tb_f = timed(lambda: forest.apply(F, out=Ub), reps)
        tb_a = timed(lambda: forest.apply_adjoint(F, out=Fb), reps)
        # sequential applies: one plan per tree, each with the shape the autotuner picks for
        # the median-size tree (tuning all 256 separately would take minutes)
        med = trees[int(np.argsort([t.n_leaves for t in trees])[len(trees) // 2])]
        sshape, _ = autotune(med.centres, med.levels)
        singles = [Plan(t.centres, t.levels, **sshape) for t in trees]
        views = [F[off[i]:off[i + 1]] for i in range(len(trees))]
        outs = [Ub[off[i]:off[i + 1]].clone() for i in range(len(trees))]
        outa = [o.clone() for o in outs]

        def seq_fwd():
            for p_, x, o in zip(singles, views, outs):
                p_.apply(x, out=o)

        def seq_adj():
            for p_, x, o in zip(singles, views, outa):
                p_.apply_adjoint(x, out=o)

        seq_fwd(); seq_adj()
        ts_f = timed(seq_fwd, 2)
        ts_a = timed(seq_adj, 2)
        dev_max = max(float((outs[i] - Ub[off[i]:off[i + 1]]).abs().max() / Ub[off[i]:off[i + 1]].abs().max())
                      for i in range(len(trees)))
        out["batched"] = {"workload": "forest of %d adaptive trees, 1-40 Gaussians each, min level 3" % len(trees),
                          "n_leaves": int(off[-1]), "unknowns": Nb,
                          "leaves_min": int(min(t.n_leaves for t in trees)),
                          "leaves_max": int(max(t.n_leaves for t in trees)),
                          "batched_fwd_unknowns_per_s": Nb / tb_f, "batched_adj_unknowns_per_s": Nb / tb_a,
                          "batched_fwd_adj_unknowns_per_s": Nb / (tb_f + tb_a),
                          "sequential_fwd_adj_unknowns_per_s": Nb / (ts_f + ts_a),
                          "speedup_fwd_adj": (ts_f + ts_a) / (tb_f + tb_a),
                          "launch_shape": fshape, "autotune_s": t_ftune, "sequential_launch_shape": sshape,
                          "max_rel_diff_batched_vs_sequential": dev_max}
        for p_ in singles:
            p_.close()
        forest.close()

    if not args.no_layer:
        out["layer_potential"] = layer_leg(args, dev)
    if not args.no_points:
        out["points"] = points_leg(args, dev)
    if not args.no_tree:
        out["tree"] = tree_leg(args, dev)
    if not args.no_strip:
        out["strip"] = strip_leg(args, dev)

    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
