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
    if kernel == "cg":             # the product, plus the PCG vector update (about 240 B per node)
        return 68 * n_act + (96 + 240) * n_nodes + 16 * n_edges
    if kernel == "cg_node":        # vectors and partials in, vectors (or the node state) out
        return 240 * n_nodes
    if kernel == "linearize":      # 58 B streamed + 16 texels x 16 B + 36 B written per active vertex
        return 350 * n_act + 96 * n_nodes + 16 * n_edges
    if kernel == "node_init":
        return 240 * n_nodes
    if kernel == "blur":           # one pass: 3 channels read + written
        return 24 * n_pix
    if kernel == "dt_rows":        # column distances in, distances out (+ contour edges per vertex)
        return 8 * n_pix + 64 * n_verts
    if kernel == "dt_cols":        # contour byte in, column distance written and re-read
        return 13 * n_pix
    if kernel == "raster":
        return 12 * n_faces + 12 * n_verts + 8 * n_pix // 4
    if kernel == "prep_image":     # blur 24 B, contour 5 B, depth-buffer clear 4 B per pixel
        return 33 * n_pix
    if kernel == "prep_geom":      # deformed start per vertex; contour bytes read by the segment pass
        return 64 * n_verts + n_pix
    if kernel == "prep_raster":    # faces, and the segment rows (8 B per 16-row segment, read and written)
        return 12 * n_faces + 12 * n_verts + 8 * n_pix // 4 + n_pix
    if kernel == "prep_cols":      # column distances (large faces: a few queued faces)
        return 13 * n_pix
    if kernel in ("contour", "decide", "deform_start", "contour_edges"):
        return 5 * n_pix if kernel == "contour" else 64 * n_verts
    if kernel in ("v_apply", "v_update"):   # per-vertex PCG: float64 vectors in and out, data block, one-ring table
        return 192 * n_verts
    if kernel == "v_lin":          # per-vertex linearisation: point, inputs, texel gathers, one-ring, PCG start
        return 570 * n_verts
    if kernel == "v_blur":         # the three blur levels: two passes each, 3 channels read + written per pass
        return 3 * 48 * n_pix
    if kernel == "pose_step":      # the 69 x 70 float64 system in, the pose out
        return 8 * 69 * 70 + 8 * 69
    if kernel == "pose_jtj":       # the Jacobian (about 115 + 400 rows x 80 float64) in, the system out
        return 8 * 515 * 80 + 8 * 69 * 70
    if kernel == "pose_rows":      # rows out, per contour vertex 44 B of vertex data in
        return 8 * 515 * 80 + 44 * 400
    if kernel == "pose_lbs":       # 5,000 vertices: xyz + binding in, positions out
        return 5000 * (12 + 32 + 12)
    return 0


# HBM bytes per launch of the J^T J p kernel, measured with rocprofv3 counter
# runs (FETCH_SIZE, WRITE_SIZE, scaled by a plain copy of known size) and kept
# in profiles/ with the fingerprint of the kernel sources they were taken on;
# a changed kernel reports null until it is measured again.
TRAFFIC_TABLE = os.path.join(ROOT, "profiles", "k_cg_hbm_traffic.md")
# Sequence mode's vertices per tile: on the 20k-vertex sequence, same-box runs
# at 96 / 128 / 160 / 256 (the library default) gave 128 the most frames/s
# (2-3 % over 256: shorter product launches outweigh the longer node pass).
SEQUENCE_TILE = 128
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1810_02648_amd", "csrc", f)
                  for f in ("solve_kernels.hip", "common.hpp", "device.hpp")]


def kernel_fingerprint():
    import hashlib
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES:
        with open(fn, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, key):
    """HBM bytes per launch for `kernel` on workload `key`, or None."""
    if kernel != "cg" or not os.path.exists(TRAFFIC_TABLE):
        return None
    fp = kernel_fingerprint()
    for line in open(TRAFFIC_TABLE):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 5 and cells[0] == key and cells[1] == fp:
            try:
                return float(cells[4].replace(",", ""))
            except ValueError:
                return None
    return None


def cpu_baseline_sequence(seq, t=2, n=3):
    """The FP64 oracle on the GPU leg's problem: frames t..t+n-1 of the
    sequence, each started from the oracle's own result of the frame before
    (its tracking of frames 0..t-1 from the rest state is set-up, not timed),
    with the sequence's weights, temporal prior, case-2 exclusion, contour rule
    and the plain schedule (GN steps x Jacobi-PCG iterations)."""
    from threadpoolctl import threadpool_limits

    from oracle import graph as og
    from oracle import nonrigid as onr
    cores = len(os.sched_getaffinity(0))
    g = og.build_graph(seq["xyz"], seq["n_nodes"])      # the template's graph (per template, not timed)

    def problem(k, start):
        return onr.Problem(seq["posed"][k], seq["tri"], seq["rgb"], g, seq["cam"], seq["masks"][k], seq["images"][k],
                           seq["weights"], state0=start.astype("float32"), w_vel=seq["w_vel"], case2="exclude",
                           outline=seq.get("outline", False))

    with threadpool_limits(limits=cores):
        st = onr.identity_state(seq["n_nodes"])
        for k in range(t):
            st = onr.solve(problem(k, st), seq["gn"], "pcg", seq["pcg"])["state"]
        t0 = time.perf_counter()
        for k in range(t, t + n):
            out = onr.solve(problem(k, st), seq["gn"], "pcg", seq["pcg"])
            st = out["state"]
        dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="frames/s", cores=cores, kind="oracle",
                sample="%d frames of the same sequence (frames %d-%d, each started from the oracle's own result of "
                       "the frame before; per-frame preprocessing + %d GN x %d Jacobi-PCG in float64 with the "
                       "sequence's weights, temporal prior, case-2 exclusion and contour rule, i.e. the GPU plain "
                       "leg's problem), %.1f s; last final energy %.4f"
                       % (n, t, t + n - 1, seq["gn"], seq["pcg"], dt, out["energies"][-1]["total"]))


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


def roofline_for(prof, steps, batch, n_act, nn, n_edges, W, H, nf, nv, key):
    per_step_us = {k: 1000.0 * ms / steps for k, (ms, n) in prof.items() if n}
    dom = max(per_step_us, key=per_step_us.get)
    bytes_launch = batch * algorithmic_bytes(dom, n_act, nn, n_edges, W * H, nf, nv)
    avg_s = prof[dom][0] / 1000.0 / prof[dom][1]
    achieved = bytes_launch / avg_s / 1e9
    apply_s = prof["cg"][0] / 1000.0 / max(prof["cg"][1], 1)
    apply_bytes = batch * algorithmic_bytes("apply", n_act, nn, n_edges, W * H, 0, 0)
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, key), "traffic_key": key,
            "avg_us": avg_s * 1e6, "algorithmic_bytes_per_launch": bytes_launch,
            "product_achieved_GBs": apply_bytes / apply_s / 1e9, "cg_avg_us": apply_s * 1e6}


def bench_sequence(args, cap, torch):
    """Learned vs plain warm start on held-out frames of a 300-frame sequence."""
    import numpy as np

    import synth.sequence
    from paper_1810_02648_amd import sequence as sq

    log("generating sequence", args.workload)
    seq = synth.sequence.make_sequence(args.workload, 0)
    ctx = cap.Context(0)
    cap.set_graphs(ctx, not args.no_graphs)
    tile = SEQUENCE_TILE if args.tile is None else args.tile
    S = sq.DeviceSequence(ctx, seq, vertices_per_tile=tile)
    log("plain tracking over %d frames" % S.n)
    states, _ = sq.track_plain(S)
    ntr = seq["n_train"]
    X, Y = sq.training_set(S, states, range(1, ntr))
    net = cap.WarmStart(ctx, S.nn, sq.init_params(0))
    log("training the warm start on %d frames" % len(X))
    t0 = time.perf_counter()
    losses = sq.train(S, net, X, Y, epochs=args.epochs, lr=1e-3, log=log)
    t_train = time.perf_counter() - t0
    test = list(range(ntr, S.n))
    for _ in range(args.warmup):
        sq.evaluate(S, net, states, test)
    log("timing %d passes over %d held-out frames" % (args.steps, len(test)))
    tp = tl = 0.0
    ev = None
    for _ in range(args.steps):
        ev = sq.evaluate(S, net, states, test)
        tp += ev["t_plain"]
        tl += ev["t_learned"]
    n = len(test) * args.steps
    # per-kernel times of one learned pass
    cap.profile_enable(ctx, True)
    cap.profile_read(ctx)
    sq.evaluate(S, net, states, test)
    prof = cap.profile_read(ctx)
    cap.profile_enable(ctx, False)
    W, H = seq["cam"].width, seq["cam"].height
    n_act = cap.nonrigid_solve(ctx, S.frame(test[0], states[test[0] - 1].clone()), S.prm)["n_visible"]
    n_edges = int((S.graph["edge_dst"] >= 0).sum().item())
    calls = 2 * len(test)    # one evaluate pass = one plain and one learned solve per frame
    roof = roofline_for(prof, calls, 1, n_act, S.nn, n_edges, W, H, seq["tri"].shape[1], seq["xyz"].shape[1],
                        "%s/tile%d" % (args.workload, tile))
    return {
        "metric": METRIC,
        "value": n / tl,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * tl / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "launch": "eager" if args.no_graphs else "HIP graph replay",
            "workload": "%s: %d-frame sequence, %d-vertex %s template, %d-node graph, %dx%d targets, %d GN x %d PCG; "
                        "train frames 1-%d, held-out frames %d-%d; one step = all held-out frames solved from "
                        "the learned start until the plain schedule's final energy"
                        % (args.workload, S.n, seq["xyz"].shape[1],
                           "articulated 23-joint body (sinusoidal joint angles + GP cloth offsets)"
                           if args.workload.startswith("body") else "ellipsoid (RBF-blended rigid motions + GP "
                           "cloth offsets)", S.nn, W, H, seq["gn"], seq["pcg"], ntr - 1, ntr, S.n - 1),
            "plain_frames_per_s": n / tp,
            "speedup_vs_plain": tp / tl,
            "mean_gn_steps_plain": float(np.mean(ev["plain_steps"])),
            "mean_gn_steps_learned": float(np.mean(ev["learned_steps"])),
            "target_reached_fraction": float(np.mean(ev["reached"])),
            "prediction_used_fraction": float(np.mean(ev["used_prediction"])),
            "vertices_per_tile": tile,
            "train_epochs": args.epochs,
            "train_seconds": t_train,
            "train_loss_first_last": [losses[0], losses[-1]],
        },
        "roofline": roof,
        "kernel_avg_us": {k: round(1000.0 * ms / c, 3) for k, (ms, c) in prof.items() if c},
    }, seq


def bench_frame(args, cap, torch):
    """Single frames (or a batch of independent frames) from the rest state."""
    import numpy as np
    import synth
    log("building workload", args.workload)
    f = synth.make_nonrigid_frame(args.workload, 0)
    nn, gn, pcg = f["n_nodes"], f["gn"], f["pcg"]
    ctx = cap.Context(0)
    cap.set_graphs(ctx, not args.no_graphs)
    xyz = torch.from_numpy(f["xyz"]).cuda()
    graph = cap.graph_build(ctx, xyz, nn)                     # on the GPU, per template (not timed)
    tri = torch.from_numpy(f["tri"]).cuda()
    start = torch.zeros((12, nn), dtype=torch.float32, device="cuda")
    start[0] = start[4] = start[8] = 1.0
    rgb = torch.from_numpy(f["rgb"]).cuda()
    mask = torch.from_numpy(f["mask"]).cuda()
    image = torch.from_numpy(f["image"]).cuda()
    prm = cap.params(*f["weights"], gn_iters=gn, pcg_iters=pcg)
    tile, tune = args.tile or 0, None
    if tile == 0:       # autotuned tile size (setup, not timed)
        probe = cap.Template(ctx, tri, graph)
        fr0 = [cap.FrameInputs(probe, xyz, rgb, f["cam"], mask, image, start.clone()) for _ in range(args.batch)]
        tile, tune = cap.autotune_tiles(ctx, [tri] * args.batch, [graph] * args.batch, fr0, prm)
        log("autotuned vertices_per_tile", tile, tune)
    tmpl = cap.Template(ctx, tri, graph, tile)
    frames = [cap.FrameInputs(tmpl, xyz, rgb, f["cam"], mask, image, start.clone()) for _ in range(args.batch)]
    pose = None
    if args.workload == "frame20k" and not args.no_pose:
        # the paper-shaped frame runs both stages: the pose stage on a 5,000-vertex skinned body
        from synth import body as sb
        pf = sb.make_pose_frame(n_vertices=5000, side=f["cam"].width, seed=0)
        b = pf["body"]
        body = cap.Body(ctx, torch.from_numpy(b["tri"]).cuda(), torch.from_numpy(b["xyz"]).cuda(),
                        torch.from_numpy(b["bind_idx"]).cuda(), torch.from_numpy(b["bind_w"]).cuda(), b["parents"],
                        b["joints"], [j not in sb.NO_DOF for j in range(len(sb.JOINTS))])
        rng = np.random.default_rng(11)
        nr = 3 * len(sb.dof_joints())
        pose0 = pf["gt_pose"].copy()
        pose0[:nr] += rng.normal(0.0, 0.05, nr)
        pose0[nr:nr + 3] += rng.normal(0.0, 0.02, 3)
        pose0 = torch.from_numpy(pose0).cuda()
        d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
        pin = cap.PoseInputs(body, pf["cam"], torch.from_numpy(pf["mask"]).cuda(), d64(pf["p2d"]), d64(pf["p3d"]),
                             d64(pf["lam"]), pose0.clone())
        pprm = cap.pose_params(1.0 / 9.0, 2500.0, 0.05, gn_iters=3)
        pose = dict(body=body, inputs=pin, prm=pprm, start=pose0, reports=[])

    def step():
        if pose is not None:
            pose["inputs"].pose.copy_(pose["start"])
            pose["reports"].append(cap.pose_solve(ctx, pose["inputs"], pose["prm"]))
        for fr in frames:
            fr.node_state.copy_(start)
        return cap.batch_solve(ctx, frames, prm)

    # warm-up: the given steps, and at least half a second so the clocks settle
    tw = time.perf_counter()
    k = 0
    while k < args.warmup or time.perf_counter() - tw < 0.5:
        reps = step()
        torch.cuda.synchronize()
        k += 1
    log("timing", args.steps, "steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reps = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cap.profile_enable(ctx, True)
    cap.profile_read(ctx)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = cap.profile_read(ctx)
    cap.profile_enable(ctx, False)
    r0 = reps[0]
    W, H = f["cam"].width, f["cam"].height
    n_edges = int((graph["edge_dst"] >= 0).sum().item())
    roof = roofline_for(prof, args.steps, args.batch, r0["n_visible"], nn, n_edges, W, H, f["tri"].shape[1],
                        f["xyz"].shape[1], "%sx%d/tile%d" % (args.workload, args.batch, tile))
    return {
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
            "launch": "eager" if args.no_graphs else "HIP graph replay",
            "workload": "%s: %s%d-vertex ellipsoid template, %d-node deformation graph, %dx%d silhouette/colour "
                        "targets, %d GN x %d PCG, plain start (rest state)"
                        % (args.workload, "pose stage + " if pose is not None else "", f["xyz"].shape[1], nn, W, H,
                           gn, pcg),
            "batch": args.batch,
            "vertices_per_tile": tile,
            "autotune_ms": None if tune is None else {str(k): round(v, 3) for k, v in tune.items()},
            "visible_vertices": r0["n_visible"],
            "final_energy": r0["energy"][-1],
            "start_energy": r0["energy"][0],
            "pose_stage": None if pose is None else {
                "workload": "23-joint skinned body, 5000 vertices, 69 unknowns, %dx%d, 3 GN with dense FP64 "
                            "Cholesky, start = ground truth + N(0, 0.05 rad)" % (W, H),
                "contour_vertices": pose["reports"][-1]["n_boundary"],
                "energy": [round(e, 3) for e in pose["reports"][-1]["energy"]],
            },
        },
        "roofline": roof,
        "kernel_avg_us": {k: round(1000.0 * ms / n, 3) for k, (ms, n) in prof.items() if n},
    }, f


def _distinct_frame(spec):
    import synth
    return synth.make_nonrigid_frame(spec["workload"], spec["seed"], n_vertices=spec["n_vertices"])


def make_distinct(workload, n, workers):
    """n captures of one configuration that share no data: capture i has seed i
    and a template of (configured vertex count - i) vertices, so templates,
    graphs, colours, deformations and targets all differ."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import synth
    nv0 = synth.CONFIGS[workload]["n_vertices"]
    specs = [dict(workload=workload, seed=i, n_vertices=nv0 - i) for i in range(n)]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_distinct_frame, specs))


def bench_vertex(args, cap, torch):
    """The per-vertex non-rigid stage (the paper's own Stage II) on frames of the
    articulated sequence: the paper's schedule (3 Gauss-Newton steps, one per
    photometric pyramid level 15/9/3, 4 PCG iterations each)."""
    import numpy as np

    import synth.sequence as ss
    n_frames = 2 + args.frames
    log("generating %d frames of %s" % (n_frames, args.workload))
    seq = ss.make_sequence(args.workload, 0, n_frames=n_frames, workers=min(16, len(os.sched_getaffinity(0))))
    ctx = cap.Context(0)
    cap.set_graphs(ctx, not args.no_graphs)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    tmpl = cap.VertexTemplate(ctx, d(seq["tri"]), d(seq["xyz"]), d(seq["classes"].astype(np.int32)))
    fs = [ss.vertex_frame(seq, t) for t in range(2, n_frames)]
    w = fs[0]["weights"]
    gn, pcg, blur = 3, 4, (15, 9, 3)
    prm = cap.vertex_params(w["w_photo"], w["w_sil"], w["w_smooth"], w["w_edge"], w["w_vel"], w["w_acc"],
                            gn_iters=gn, pcg_iters=pcg, exclude_case2=True, outline_only=True, blur_kernels=blur)
    rgb = d(seq["rgb"])
    frames, starts = [], []
    for f in fs:
        st = d(f["start"])
        starts.append(st)
        frames.append(cap.VertexInputs(tmpl, d(f["posed"]), rgb, f["cam"], d(f["mask"]), d(f["image"]), st.clone(),
                                       prev=d(f["prev"]), prev2=d(f["prev2"])))

    def step():
        reps = []
        for fr, st in zip(frames, starts):
            fr.V.copy_(st)
            reps.append(cap.vertex_solve(ctx, fr, prm))
        return reps

    tw = time.perf_counter()
    k = 0
    while k < args.warmup or time.perf_counter() - tw < 0.5:
        reps = step()
        torch.cuda.synchronize()
        k += 1
    log("timing", args.steps, "steps of", len(frames), "frames")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reps = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cap.profile_enable(ctx, True)
    cap.profile_read(ctx)
    step()
    torch.cuda.synchronize()
    prof = cap.profile_read(ctx)
    cap.profile_enable(ctx, False)
    nv = seq["xyz"].shape[1]
    W, H = seq["cam"].width, seq["cam"].height
    vk = {k: v for k, v in prof.items() if k.startswith("v_") and v[1]}
    dom = max(vk, key=lambda k: vk[k][0])
    avg_s = vk[dom][0] / 1000.0 / vk[dom][1]
    bytes_launch = algorithmic_bytes(dom, 0, 0, 0, W * H, 0, nv)
    achieved = bytes_launch / avg_s / 1e9
    errs = [float(np.sqrt(((fr.V.cpu().numpy() - f["gt"]) ** 2).sum(0)).mean()) for fr, f in zip(frames, fs)]
    errs0 = [float(np.sqrt(((f["start"] - f["gt"]) ** 2).sum(0)).mean()) for f in fs]
    n = args.steps * len(frames)
    return {
        "metric": "per-vertex non-rigid GN frames/s",
        "value": n / elapsed,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "launch": "eager" if args.no_graphs else "HIP graph replay",
            "workload": "%s per-vertex stage: %d frames (t = 2..%d) of the %d-vertex articulated body sequence, "
                        "%dx%d targets, %d GN x %d PCG, photometric pyramid %s, smooth/edge/velocity/acceleration "
                        "with Table 1 material weights; start = pose result + previous displacement"
                        % (args.workload, len(frames), n_frames - 1, nv, W, H, gn, pcg, "/".join(map(str, blur))),
            "mean_energy_start_final": [float(np.mean([r["energy"][0] for r in reps])),
                                        float(np.mean([r["energy"][-1] for r in reps]))],
            "mean_vertex_error_mm_start_final": [1000 * float(np.mean(errs0)), 1000 * float(np.mean(errs))],
        },
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "avg_us": avg_s * 1e6,
                     "algorithmic_bytes_per_launch": bytes_launch},
        "kernel_avg_us": {k: round(1000.0 * ms / c, 3) for k, (ms, c) in prof.items() if c},
    }, (seq, fs, w, gn, pcg, blur)


def bench_track(args, cap, torch):
    """Two-stage tracking (pose stage with Euler start, skinning, warped
    per-vertex stage) of the articulated sequence: stages of consecutive
    frames on two streams against both stages in order on one stream."""
    import numpy as np

    import synth.sequence as ss
    from paper_1810_02648_amd.pipeline import Tracker
    from synth import body as sb
    n = args.frames
    log("generating %d frames of %s" % (n, args.workload))
    seq = ss.make_sequence(args.workload, 0, n_frames=n, workers=min(16, len(os.sched_getaffinity(0))))
    ctx = cap.Context(0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    b = seq["body"]
    body = cap.Body(ctx, d(b["tri"]), d(b["xyz"]), d(b["bind_idx"]), d(b["bind_w"]), b["parents"], b["joints"],
                    [j not in sb.NO_DOF for j in range(len(sb.JOINTS))])
    vt = cap.VertexTemplate(ctx, d(b["tri"]), d(b["xyz"]), d(b["classes"]))
    frames = []
    for t in range(n):
        p2d, p3d, lam = ss.pose_detections(seq, t)
        frames.append(dict(mask=d(seq["masks"][t]), image=d(seq["images"][t]), p2d=d(p2d), p3d=d(p3d), lam=d(lam)))
    prm = cap.pose_params(gn_iters=3, **ss.tracking_pose_params(seq["cam"].width, 3 * len(sb.dof_joints())))
    T = Tracker(body, vt, d(seq["rgb"]), seq["cam"], frames, d(seq["poses"][0]), prm,
                ss.vertex_weights_for(seq["cam"].width))
    for c in (T.ctx_pose, T.ctx_nr):
        cap.set_graphs(c, not args.no_graphs)
    times = {}
    for mode, run in (("sequential", T.run_sequential), ("pipelined", T.run_pipelined)):
        for _ in range(max(args.warmup, 1)):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        times[mode] = time.perf_counter() - t0
        log(mode, "%.1f frames/s" % (args.steps * n / times[mode]))
    err = [1000 * float(np.sqrt(((T.V[t].cpu().numpy() - seq["gt"][t]) ** 2).sum(0)).mean()) for t in range(n)]
    err_s = [1000 * float(np.sqrt(((T.posed[t].cpu().numpy() - seq["gt"][t]) ** 2).sum(0)).mean())
             for t in range(n)]
    return {
        "metric": "two-stage tracking frames/s (pose + per-vertex non-rigid)",
        "value": args.steps * n / times["pipelined"],
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * times["pipelined"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "launch": "eager" if args.no_graphs else "HIP graph replay",
            "workload": "%s: %d frames, %d-vertex articulated body for both stages, %dx%d; pose stage 3 GN (69 "
                        "unknowns, Euler start), skinning, displacement-warped per-vertex stage 3 GN x 4 PCG with the "
                        "15/9/3 pyramid; one step = the whole sequence" % (args.workload, n, body.nv,
                                                                           seq["cam"].width, seq["cam"].height),
            "sequential_frames_per_s": args.steps * n / times["sequential"],
            "pipelined_speedup": times["sequential"] / times["pipelined"],
            "mean_vertex_error_mm_skinned_tracked": [float(np.mean(err_s)), float(np.mean(err))],
        },
    }, None


def cpu_baseline_vertex(data, n=3):
    """The FP64 oracle on the first n frames of the GPU leg's problem (same
    starts, inputs, weights, schedule and pyramid)."""
    from threadpoolctl import threadpool_limits

    from oracle import vertex as ov
    seq, fs, w, gn, pcg, blur = data
    cores = len(os.sched_getaffinity(0))
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        for f in fs[:n]:
            P = ov.VertexProblem(f["rest"], f["posed"], f["tri"], f["rgb"], f["classes"], f["cam"], f["mask"],
                                 f["image"], w, start=f["start"], prev=f["prev"], prev2=f["prev2"], case2="exclude",
                                 outline=True)
            out = ov.solve(P, gn, "pcg", pcg, blur_schedule=blur)
        dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="frames/s", cores=cores, kind="oracle",
                sample="%d frames of the same workload (decisions, pyramid blur and %d GN x %d Jacobi-PCG in float64 "
                       "each), %.1f s; last final energy %.4f" % (n, gn, pcg, dt, out["energies"][-1]["total"]))


def bench_batch(args, cap, torch):
    """Many independent frames solved together by one batched call per step:
    batch mode, frames of uneven size (log-uniform vertices, nodes and image
    sides); frame mode with --distinct, captures of one configuration that
    share no data (distinct templates and inputs)."""
    import synth
    workers = min(16, len(os.sched_getaffinity(0)))
    if args.mode == "batch":
        n = args.batch if args.batch > 1 else 64
        log("generating %d frames" % n)
        frames_h = synth.make_batch(n, 0, workers=min(8, workers))
        gn, pcg, weights = 5, 10, (1.0, 0.1, 10.0)      # the small configuration's schedule and weights
    else:
        n = args.batch
        log("generating %d distinct %s captures" % (n, args.workload))
        frames_h = make_distinct(args.workload, n, workers)
        gn, pcg, weights = frames_h[0]["gn"], frames_h[0]["pcg"], frames_h[0]["weights"]
    ctx = cap.Context(0)
    cap.set_graphs(ctx, not args.no_graphs)
    prm = cap.params(*weights, gn_iters=gn, pcg_iters=pcg)
    dev_in = []
    for f in frames_h:
        xyz = torch.from_numpy(f["xyz"]).cuda()
        g = cap.graph_build(ctx, xyz, f["n_nodes"])
        st = torch.zeros((12, f["n_nodes"]), dtype=torch.float32, device="cuda")
        st[0] = st[4] = st[8] = 1.0
        dev_in.append((xyz, torch.from_numpy(f["tri"]).cuda(), g, torch.from_numpy(f["rgb"]).cuda(),
                       torch.from_numpy(f["mask"]).cuda(), torch.from_numpy(f["image"]).cuda(), st))

    def make_frames(tile):
        return [cap.FrameInputs(cap.Template(ctx, tri, g, tile), xyz, rgb, f["cam"], mask, image, st.clone())
                for f, (xyz, tri, g, rgb, mask, image, st) in zip(frames_h, dev_in)]

    tile, tune = args.tile or 0, None
    if tile == 0:       # autotuned tile size for the whole batch (setup, not timed)
        tile, tune = cap.autotune_tiles(ctx, [d[1] for d in dev_in], [d[2] for d in dev_in], make_frames(0), prm)
        log("autotuned vertices_per_tile", tile, tune)
    frames = make_frames(tile)
    starts = [d[6] for d in dev_in]
    graphs = [d[2] for d in dev_in]

    def step():
        for fr, st in zip(frames, starts):
            fr.node_state.copy_(st)
        return cap.batch_solve(ctx, frames, prm)

    # warm-up: the given steps, and at least half a second so the clocks settle
    tw = time.perf_counter()
    k = 0
    while k < args.warmup or time.perf_counter() - tw < 0.5:
        reps = step()
        torch.cuda.synchronize()
        k += 1
    log("timing", args.steps, "steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reps = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    cap.profile_enable(ctx, True)
    cap.profile_read(ctx)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    prof = cap.profile_read(ctx)
    cap.profile_enable(ctx, False)
    per_step_us = {k: 1000.0 * ms / args.steps for k, (ms, c) in prof.items() if c}
    dom = max(per_step_us, key=per_step_us.get)

    def total_bytes(kernel):
        s = 0
        for f, g, r in zip(frames_h, graphs, reps):
            ne = int((g["edge_dst"] >= 0).sum().item())
            s += algorithmic_bytes(kernel, r["n_visible"], f["n_nodes"], ne, f["cam"].width * f["cam"].height,
                                   f["tri"].shape[1], f["xyz"].shape[1])
        return s

    avg_s = prof[dom][0] / 1000.0 / prof[dom][1]
    achieved = total_bytes(dom) / avg_s / 1e9
    apply_s = prof["cg"][0] / 1000.0 / max(prof["cg"][1], 1)
    key = ("batch%d/tile%d" % (n, tile)) if args.mode == "batch" else ("%sx%d-distinct/tile%d" % (args.workload, n, tile))
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, key), "traffic_key": key,
            "avg_us": avg_s * 1e6,
            "algorithmic_bytes_per_launch": total_bytes(dom),
            "product_achieved_GBs": total_bytes("apply") / apply_s / 1e9, "cg_avg_us": apply_s * 1e6}
    nv = [f["xyz"].shape[1] for f in frames_h]
    return {
        "metric": METRIC,
        "value": args.steps * n / elapsed,
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
            "launch": "eager" if args.no_graphs else "HIP graph replay",
            "workload": ("batch of %d independent frames, log-uniform 4k-40k vertices, 128-1000 nodes, 512-1080 px "
                         "square images" % n if args.mode == "batch" else
                         "%d distinct %s captures (seeds 0-%d, templates of %d..%d vertices, %d nodes, %d px images)"
                         % (n, args.workload, n - 1, max(nv), min(nv), frames_h[0]["n_nodes"],
                            frames_h[0]["cam"].width))
                        + " (%d vertices, %.1f Mpx in total), %d GN x %d PCG, plain start, one batched call per step"
                        % (sum(nv), sum(f["cam"].width ** 2 for f in frames_h) / 1e6, gn, pcg),
            "batch": n,
            "vertices_per_tile": tile,
            "autotune_ms": None if tune is None else {str(k): round(v, 3) for k, v in tune.items()},
            "final_energy_sum": float(sum(r["energy"][-1] for r in reps)),
            "start_energy_sum": float(sum(r["energy"][0] for r in reps)),
        },
        "roofline": roof,
        "kernel_avg_us": {k: round(1000.0 * ms / c, 3) for k, (ms, c) in prof.items() if c},
    }, frames_h


def main():
    import numpy as np
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="sequence", choices=["sequence", "frame", "batch", "vertex", "track", "copy"],
                    help="copy: a plain device copy of known size (calibrates the profiler's byte counters)")
    ap.add_argument("--workload", default=None,
                    help="sequence: body20k (default: articulated body), seq20k (ellipsoid), body_small, seq_small; "
                         "frame: frame20k (default), small, stress200k")
    ap.add_argument("--batch", type=int, default=1,
                    help="frame mode: copies of the frame solved together per step; batch mode: frames (default 64)")
    ap.add_argument("--epochs", type=int, default=40, help="sequence mode: training epochs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-pose", action="store_true", help="frame mode: leave out the pose stage")
    ap.add_argument("--no-graphs", action="store_true",
                    help="launch every kernel eagerly instead of replaying captured HIP graphs")
    ap.add_argument("--tile", type=int, default=None,
                    help="vertices per tile (0 = library default); default: %d in sequence mode, autotuned in frame "
                         "and batch modes" % SEQUENCE_TILE)
    ap.add_argument("--frames", type=int, default=40, help="vertex / track modes: frames per step")
    ap.add_argument("--distinct", action="store_true",
                    help="frame mode: the --batch captures share no data (capture i: seed i, template of N - i "
                         "vertices) instead of repeating one capture")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver has no multi-GPU path "
              "(independent captures would shard one per GPU with no communication)", file=sys.stderr)
        sys.exit(2)
    if args.workload is None:
        args.workload = "body20k" if args.mode in ("sequence", "vertex", "track") else "frame20k"

    import torch

    import paper_1810_02648_amd as cap

    if args.mode == "copy":
        n = 1 << 27                                   # 512 MiB of float32 each way
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                          "launches": args.warmup + args.steps}), flush=True)
        return
    if args.mode == "sequence":
        result, data = bench_sequence(args, cap, torch)
    elif args.mode == "vertex":
        result, data = bench_vertex(args, cap, torch)
    elif args.mode == "track":
        result, data = bench_track(args, cap, torch)
        args.no_cpu_baseline = True
    elif args.mode == "batch" or args.distinct:
        result, data = bench_batch(args, cap, torch)
    else:
        result, data = bench_frame(args, cap, torch)
    if args.distinct and not args.no_cpu_baseline:
        log("no cpu baseline for distinct captures (pass --no-cpu-baseline)")
    elif not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        if args.mode == "batch":
            # frames at the 25th, 50th and 75th percentile of vertex count; rate = 1 / mean time
            order = sorted(range(len(data)), key=lambda i: data[i]["xyz"].shape[1])
            pick = [order[len(order) * q // 4] for q in (1, 2, 3)]
            rates = [cpu_baseline(data[i], data[i]["n_nodes"], 5, 10, (1.0, 0.1, 10.0)) for i in pick]
            cb = dict(rates[0])
            cb["value"] = 1.0 / float(np.mean([1.0 / r["value"] for r in rates]))
            cb["sample"] = ("3 frames of the batch (%s vertices: its 25th/50th/75th percentile), each per-frame "
                            "preprocessing + 5 GN steps with exact sparse-Cholesky solves in float64; rate = 1 / mean "
                            "time" % "/".join(str(data[i]["xyz"].shape[1]) for i in pick))
            result["cpu_baseline"] = cb
        elif args.mode == "sequence":
            result["cpu_baseline"] = cpu_baseline_sequence(data)
        elif args.mode == "vertex":
            result["cpu_baseline"] = cpu_baseline_vertex(data)
        else:
            result["cpu_baseline"] = cpu_baseline(data, data["n_nodes"], data["gn"], data["pcg"], data["weights"])
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
