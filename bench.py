#!/usr/bin/env python3
"""Throughput of the per-frame non-rigid Gauss-Newton solve on one MI355X.

One step = one batched solve of B independent frames of the chosen workload
(per-frame preprocessing + the full Gauss-Newton/PCG schedule), inputs
already resident in device memory; the node states are reset to the start
state inside the step.  Prints one JSON line: throughput, the dominant
kernel's achieved bandwidth against the HBM peak, per-kernel times and the
FP64 oracle's rate on the host; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "non-rigid GN frames/s at equal final energy, learned warm-start vs plain"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, n_act, n_nodes, n_edges, n_pix, n_faces, n_verts):
    """Bytes one launch must move for one frame (the method's minimum, not what
    an implementation happens to move)."""
    if kernel == "apply":          # v 12 + idx 16 + w 16 + H 24 per active vertex; p, Ap, g, R per node; edges
        return 68 * n_act + 96 * n_nodes + 16 * n_edges
    if kernel == "linearize":      # 58 B streamed + 16 texels x 16 B + 36 B written per active vertex
        return 350 * n_act + 96 * n_nodes + 16 * n_edges
    if kernel == "node_pcg":       # PCG vectors and partials per node
        return 240 * n_nodes
    if kernel == "node_init":
        return 240 * n_nodes
    if kernel == "blur":           # one pass: 3 channels read + written
        return 24 * n_pix
    if kernel == "dt_rows":        # column distances in, distances out
        return 8 * n_pix
    if kernel == "dt_cols":        # contour byte in, column distance written and re-read
        return 13 * n_pix
    if kernel == "raster":
        return 12 * n_faces + 12 * n_verts + 8 * n_pix // 4
    if kernel in ("contour", "decide", "deform_start", "contour_edges"):
        return 5 * n_pix if kernel == "contour" else 64 * n_verts
    return 0


def cpu_baseline(frame_dict, n_nodes, gn, pcg, weights):
    """The FP64 oracle (exact Cholesky solves) on one frame of the same workload."""
    import numpy as np  # noqa: F401
    from threadpoolctl import threadpool_limits

    from oracle import graph as og
    from oracle import nonrigid as onr
    cores = len(os.sched_getaffinity(0))
    f = frame_dict
    g = og.build_graph(f["xyz"], n_nodes)          # per-template setup, not timed (as on the GPU)
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        P = onr.Problem(f["xyz"], f["tri"], f["rgb"], g, f["cam"], f["mask"], f["image"], weights)
        out = onr.solve(P, gn, "chol")
        dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="frames/s", cores=cores, kind="oracle",
                sample="1 frame of the same workload (per-frame preprocessing + %d GN steps with exact "
                       "sparse-Cholesky solves, float64), %.1f s; final energy %.4f"
                       % (gn, dt, out["energies"][-1]["total"]))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="frame20k", choices=["small", "frame20k", "stress200k"])
    ap.add_argument("--batch", type=int, default=1, help="independent frames solved together per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(independent captures would shard one per GPU with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1810_02648_amd as cap
    import synth

    wl = synth.CONFIGS[args.workload]
    log("building workload", args.workload)
    f = synth.make_nonrigid_frame(args.workload, 0)
    nn, gn, pcg = f["n_nodes"], f["gn"], f["pcg"]
    ctx = cap.Context(0)
    xyz = torch.from_numpy(f["xyz"]).cuda()
    graph = cap.graph_build(ctx, xyz, nn)                     # on the GPU, per template (not timed)
    tmpl = cap.Template(ctx, torch.from_numpy(f["tri"]).cuda(), graph)
    start = torch.zeros((12, nn), dtype=torch.float32, device="cuda")
    start[0] = start[4] = start[8] = 1.0
    rgb = torch.from_numpy(f["rgb"]).cuda()
    mask = torch.from_numpy(f["mask"]).cuda()
    image = torch.from_numpy(f["image"]).cuda()
    frames = [cap.FrameInputs(tmpl, xyz, rgb, f["cam"], mask, image, start.clone()) for _ in range(args.batch)]
    prm = cap.params(*f["weights"], gn_iters=gn, pcg_iters=pcg)

    def step():
        for fr in frames:
            fr.node_state.copy_(start)
        return cap.batch_solve(ctx, frames, prm)

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        reps = step()
    torch.cuda.synchronize()
    log("timing", args.steps, "steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reps = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log("timed %.3f s" % elapsed)

    # per-kernel times from events around every launch, in a second pass of the same steps
    cap.profile_enable(ctx, True)
    cap.profile_read(ctx)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = cap.profile_read(ctx)
    cap.profile_enable(ctx, False)
    kernel_us = {k: round(1000.0 * ms / n, 3) for k, (ms, n) in prof.items() if n}
    per_step_us = {k: 1000.0 * ms / args.steps for k, (ms, n) in prof.items() if n}
    dom = max(per_step_us, key=per_step_us.get)
    r0 = reps[0]
    n_act = r0["n_visible"]
    n_edges = int((graph["edge_dst"] >= 0).sum().item())
    W, H = f["cam"].width, f["cam"].height
    bytes_launch = args.batch * algorithmic_bytes(dom, n_act, nn, n_edges, W * H, f["tri"].shape[1],
                                                  f["xyz"].shape[1])
    avg_s = prof[dom][0] / 1000.0 / prof[dom][1]
    achieved = bytes_launch / avg_s / 1e9
    apply_s = prof["apply"][0] / 1000.0 / max(prof["apply"][1], 1)
    apply_bytes = args.batch * algorithmic_bytes("apply", n_act, nn, n_edges, W * H, 0, 0)

    result = {
        "metric": METRIC,
        "value": args.steps * args.batch / elapsed,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "%s: %d-vertex ellipsoid template, %d-node deformation graph, %dx%d silhouette/colour "
                        "targets, %d GN x %d PCG, plain start (rest state); learned warm start not in this line"
                        % (args.workload, f["xyz"].shape[1], nn, W, H, gn, pcg),
            "batch": args.batch,
            "visible_vertices": n_act,
            "final_energy": r0["energy"][-1],
            "start_energy": r0["energy"][0],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_us": avg_s * 1e6,
            "algorithmic_bytes_per_launch": bytes_launch,
            "apply_achieved": apply_bytes / apply_s / 1e9,
        },
        "kernel_avg_us": kernel_us,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(f, nn, gn, pcg, f["weights"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
