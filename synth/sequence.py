"""Seeded capture sequences: a template under smooth, cloth-like motion.

Recipe (30 fps):

* Template and camera as in ``synth.workloads`` (ellipsoid, square camera,
  f = 2S).  Colours are a smooth texture-like field rather than independent
  per-vertex noise: per channel 0.5 + 0.5 sin(k . x + phi) summed over three
  random wave vectors with |k| = 2 pi / U(0.1, 0.3) m and normalised to
  [0, 1] (patterns of about 10-30 cm, like clothing prints).
* Articulated part (what the pose stage explains): ``n_ctrl`` control
  vertices chosen at random; control point m rotates by the axis-angle vector
  a_m * sin(2 pi f_m t + phi_m) (per component a ~ U(0.05, 0.25) rad,
  f ~ U(0.2, 1.0) Hz, phi ~ U(0, 2 pi)) and every vertex moves by the
  normalised Gaussian-RBF blend of those rigid motions (kernel width: mean
  distance between a control point and its nearest neighbour).  This posed
  mesh is each frame's input mesh of the non-rigid stage (the paper's
  skinned mesh after Stage I, Sec. 3.4).
* Cloth-like part (what the non-rigid stage must recover): offsets
  o_m(t) = sum_{q=1..4} [A_q,m cos(w_q t) + B_q,m sin(w_q t)] / 2 at the control
  points, A_q and B_q draws of a Gaussian process over the rest control
  positions (squared-exponential kernel, length scale 0.2 m, amplitude
  0.03 m), w_q / 2 pi ~ U(0.5, 2) Hz, blended to the vertices with the same
  weights and added to the posed mesh.
* Each frame's mask and colour image are rendered from posed + offsets.

Articulated sequences (``body*``, the default benchmark workload):

* Template: the procedural 23-joint body of ``synth.body`` (one closed
  ellipsoid per bone, overlapping at the joints) meshed to exactly the
  requested vertex count, root 4.5 m in front of the camera (the 1.87 m body
  spans ~0.83 of the image height at f = 2S), smooth colours as above.
* Pose (what the pose stage explains): every rotational degree of freedom
  follows theta(t) = a sin(2 pi f t + phi), a ~ U(0.1, 0.5) rad,
  f ~ U(0.2, 1.0) Hz, phi ~ U(0, 2 pi); the skinned mesh at that pose is the
  frame's input mesh of the non-rigid stage.
* Cloth-like part: the same Gaussian-process offsets as above (length scale
  0.2 m, amplitude 0.03 m, 4 harmonics of 0.5-2 Hz) at 64 control vertices,
  blended to the vertices by rest-pose RBF weights and added to the posed
  mesh in the camera frame.
* Tracking uses the outline-only contour set: the body's parts are seen in
  front of one another, and contours inside the silhouette have no
  counterpart in the image's distance transform.

The paper's evaluation sequences (11 sequences, 7 actors, 540x960 video)
are not available; this motion stands in for their smooth body and cloth
motion.
"""
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
from scipy.spatial.transform import Rotation

from .render import render_targets
from .workloads import Camera, template_mesh

def _tracking_weights(side):
    """(w_sil, w_photo, w_arap), w_vel for tracking at image side `side`.

    The silhouette residual is in pixels and the regulariser residuals in
    metres, so their balance scales with (pixels per metre)^2, i.e. with
    side^2 at a fixed field of view.  At 1080^2 a weight sweep over 60 frames
    of the 20k sequence (w_arap 1e3..1e7, w_vel 1e2..1e4, w_photo 0.1..10)
    gives the lowest mean vertex error (31.7 mm against 42 mm for the posed
    input) at w_arap = 1e6, w_vel = 1e3; with the single-frame weights
    (w_arap = 10) the silhouette term folds the mesh within a few frames."""
    s = (side / 1080.0) ** 2
    return (1.0, 0.1, 1.0e6 * s), 1.0e3 * s


SEQUENCES = {
    # paper-shaped: 20,000 vertices, 500 nodes, 1080^2, 300 frames (200 train, 100 test)
    # Tracking uses the paper's temporal prior (w_vel per vertex, m^-2) and drops case-2
    # silhouette residuals: without an absolute anchor the monocular depth drifts
    # from frame to frame.
    "seq20k": dict(mesh="fib", n_vertices=20000, n_nodes=500, side=1080, n_frames=300, n_train=200,
                   gn=3, pcg=8, weights=_tracking_weights(1080)[0], w_vel=_tracking_weights(1080)[1]),
    # small, for tests
    "seq_small": dict(mesh="ico4", n_vertices=2562, n_nodes=64, side=256, n_frames=40, n_train=24,
                      gn=3, pcg=8, weights=_tracking_weights(256)[0], w_vel=_tracking_weights(256)[1]),
    # articulated body: 20,000 vertices, 500 nodes, 1080^2, 300 frames (200 train, 100 test)
    "body20k": dict(mesh="body", n_vertices=20000, n_nodes=500, side=1080, n_frames=300, n_train=200,
                    gn=3, pcg=8, weights=_tracking_weights(1080)[0], w_vel=_tracking_weights(1080)[1],
                    outline=True),
    # articulated body, small, for tests
    "body_small": dict(mesh="body", n_vertices=3000, n_nodes=64, side=256, n_frames=40, n_train=24,
                       gn=3, pcg=8, weights=_tracking_weights(256)[0], w_vel=_tracking_weights(256)[1],
                       outline=True),
}


def smooth_colours(xyz, rng):
    p = xyz.T.astype(np.float64)
    out = np.zeros((3, p.shape[0]))
    for c in range(3):
        for _ in range(3):
            d = rng.normal(size=3)
            k = d / np.linalg.norm(d) * (2.0 * np.pi / rng.uniform(0.1, 0.3))
            out[c] += np.sin(p @ k + rng.uniform(0.0, 2.0 * np.pi))
        out[c] = (out[c] - out[c].min()) / max(out[c].max() - out[c].min(), 1e-12)
    return out.astype(np.float32)


def _motion(xyz, rng, n_ctrl):
    p = xyz.T.astype(np.float64)
    ctrl = rng.choice(p.shape[0], size=n_ctrl, replace=False)
    c = p[ctrl]
    amp = rng.uniform(0.05, 0.25, size=(n_ctrl, 3))
    freq = rng.uniform(0.2, 1.0, size=(n_ctrl, 3))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(n_ctrl, 3))
    d2 = ((c[:, None, :] - c[None, :, :]) ** 2).sum(-1)
    K = 0.03 ** 2 * np.exp(-d2 / (2.0 * 0.2 ** 2)) + 1e-10 * np.eye(n_ctrl)
    L = np.linalg.cholesky(K)
    A = np.einsum("ij,qjd->qid", L, rng.normal(size=(4, n_ctrl, 3)))
    B = np.einsum("ij,qjd->qid", L, rng.normal(size=(4, n_ctrl, 3)))
    w = 2.0 * np.pi * rng.uniform(0.5, 2.0, size=4)
    dcc = np.sqrt(d2) + np.diag(np.full(n_ctrl, np.inf))
    sigma = dcc.min(axis=1).mean()
    wts = np.exp(-((p[:, None, :] - c[None, :, :]) ** 2).sum(-1) / (2.0 * sigma * sigma))
    wts /= wts.sum(axis=1, keepdims=True)
    return dict(c=c, amp=amp, freq=freq, phase=phase, A=A, B=B, w=w, wts=wts)


def _pose_at(xyz, m, t):
    """(posed mesh, posed mesh + cloth offsets) at time t, float32 [3][N]."""
    p = xyz.T.astype(np.float64)
    rv = m["amp"] * np.sin(2.0 * np.pi * m["freq"] * t + m["phase"])
    R = Rotation.from_rotvec(rv).as_matrix()
    off = (m["A"] * np.cos(m["w"] * t)[:, None, None] + m["B"] * np.sin(m["w"] * t)[:, None, None]).sum(0) / 2.0
    posed = np.zeros_like(p)
    for k in range(m["c"].shape[0]):
        posed += m["wts"][:, k:k + 1] * ((p - m["c"][k]) @ R[k].T + m["c"][k])
    gt = posed + m["wts"] @ off
    return (np.ascontiguousarray(posed.T.astype(np.float32)), np.ascontiguousarray(gt.T.astype(np.float32)))


def _render_frame(args):
    xyz, tri, rgb, cam, m, t = args
    posed, gt = _pose_at(xyz, m, t)
    mask, image = render_targets(gt, tri, rgb, cam)
    return posed, gt, mask, image


def _body_motion(body, rng, n_ctrl):
    """Sinusoidal joint angles and Gaussian-process cloth offsets of a body sequence."""
    from .body import dof_joints
    nd = 3 * len(dof_joints())
    amp = rng.uniform(0.1, 0.5, nd)
    freq = rng.uniform(0.2, 1.0, nd)
    phase = rng.uniform(0.0, 2.0 * np.pi, nd)
    cloth = _motion(body["xyz"], rng, n_ctrl)
    return dict(body=body, amp=amp, freq=freq, phase=phase, cloth=cloth)


def _body_pose_at(m, t):
    """(posed mesh, posed mesh + cloth offsets) of a body sequence at time t."""
    from .body import pose_mesh
    pose = np.zeros(69)
    pose[:m["amp"].size] = m["amp"] * np.sin(2.0 * np.pi * m["freq"] * t + m["phase"])
    posed, P = pose_mesh(m["body"], pose)
    pose[66:69] = P[0]                    # t' maps root-relative 3D joints to the camera frame
    c = m["cloth"]
    off = (c["A"] * np.cos(c["w"] * t)[:, None, None] + c["B"] * np.sin(c["w"] * t)[:, None, None]).sum(0) / 2.0
    gt = posed.T.astype(np.float64) + c["wts"] @ off
    return posed, np.ascontiguousarray(gt.T.astype(np.float32)), pose, P


def _render_body_frame(args):
    tri, rgb, cam, m, t = args
    posed, gt, pose, P = _body_pose_at(m, t)
    mask, image = render_targets(gt, tri, rgb, cam)
    return posed, gt, mask, image, pose, P


def make_sequence(name="seq20k", seed=0, n_frames=None, workers=None):
    """Template, camera, per-frame ground truth and rendered targets of a sequence."""
    cfg = dict(SEQUENCES[name])
    if n_frames is not None:
        cfg["n_frames"] = n_frames
        cfg["n_train"] = min(cfg["n_train"], n_frames)
    rng = np.random.Generator(np.random.PCG64(seed))
    cam = Camera.square(cfg["side"])
    if cfg["mesh"] == "body":
        from .body import make_body
        body = make_body(cfg["n_vertices"], root=(0.0, 0.0, 4.5))
        xyz, tri = body["xyz"], body["tri"]
        classes = body["classes"]
        parts = body["parts"]
        rgb = smooth_colours(xyz, rng)
        m = _body_motion(body, rng, 64)
        jobs = [(tri, rgb, cam, m, f / 30.0) for f in range(cfg["n_frames"])]
        render = _render_body_frame
    else:
        xyz, tri = template_mesh(cfg["mesh"], cfg["n_vertices"])
        classes = np.full(xyz.shape[1], 2, np.int32)      # one material: upper clothes
        parts = np.zeros(xyz.shape[1], np.int32)          # one body part
        rgb = smooth_colours(xyz, rng)
        m = _motion(xyz, rng, 24)
        jobs = [(xyz, tri, rgb, cam, m, f / 30.0) for f in range(cfg["n_frames"])]
        render = _render_frame
    if workers is None:
        workers = min(8, len(os.sched_getaffinity(0)))
    if workers > 1 and len(jobs) > 4:
        import multiprocessing as mp
        with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            frames = list(ex.map(render, jobs, chunksize=4))
    else:
        frames = [render(j) for j in jobs]
    extra = {}
    if cfg["mesh"] == "body":
        extra = dict(body=body, poses=[f[4] for f in frames], joints=[f[5] for f in frames])
    return dict(name=name, seed=seed, xyz=xyz, tri=tri, rgb=rgb, cam=cam, classes=classes, parts=parts,
                posed=[f[0] for f in frames], gt=[f[1] for f in frames], masks=[f[2] for f in frames],
                images=[f[3] for f in frames], **extra,
                n_nodes=cfg["n_nodes"], n_train=cfg["n_train"], gn=cfg["gn"], pcg=cfg["pcg"],
                weights=cfg["weights"], w_vel=cfg["w_vel"], outline=cfg.get("outline", False))


def vertex_weights_for(side):
    """Term weights of the per-vertex non-rigid stage for a square image of
    `side` pixels (positions in metres, colours in [0, 1], the silhouette
    residual in pixels).  The paper's values (Sec. 5: photo 10000,
    silhouette 600, smooth 10, edge 30, velocity 0.25, acceleration 0.1)
    keep their ratios within the data terms (photo / silhouette) and within
    the regularisers; the regularisers are scaled by k = 1e4 (side / 1080)^2
    against w_sil = 1 (a pixel residual's weight grows with the image side
    squared at a fixed field of view), the value of a sweep over k on the
    small body sequence."""
    k = 1.0e4 * (side / 1080.0) ** 2
    return dict(w_photo=10000.0 / 600.0, w_sil=1.0, w_smooth=10.0 * k, w_edge=30.0 * k, w_vel=0.25 * k,
                w_acc=0.1 * k)


def vertex_frame(seq, t, weights=None):
    """Inputs of the per-vertex non-rigid stage at frame t >= 2 of a sequence:
    rest template, posed mesh V^S_t (the pose stage's result), targets, the
    previous two frames' ground truth as V^{t-1}, V^{t-2}, and the start
    V^S_t + (V^{t-1} - V^S_{t-1}) (the previous displacement carried over)."""
    if t < 2:
        raise ValueError("t >= 2")
    side = seq["cam"].width
    prev, prev2 = seq["gt"][t - 1], seq["gt"][t - 2]
    start = (seq["posed"][t] + (prev - seq["posed"][t - 1])).astype(np.float32)
    return dict(rest=seq["xyz"], posed=seq["posed"][t], tri=seq["tri"], rgb=seq["rgb"], classes=seq["classes"],
                parts=seq["parts"],
                cam=seq["cam"], mask=seq["masks"][t], image=seq["images"][t], prev=prev, prev2=prev2,
                start=np.ascontiguousarray(start), gt=seq["gt"][t],
                weights=vertex_weights_for(side) if weights is None else weights,
                outline=seq.get("outline", False))


def pose_detections(seq, t, px_sigma=None, m_sigma=0.02):
    """Noisy 2D and 3D joint detections of frame t of a body sequence (the
    stand-in for the CNN detections of Sec. 3.3): 2D = projected ground-truth
    joints + N(0, px_sigma^2) px (default 3 px at 1080 px, scaled with the
    image side), 3D = root-relative ground truth + N(0, m_sigma^2) m,
    confidences 1; seeded by the frame index."""
    rng = np.random.Generator(np.random.PCG64(1000 + t))
    cam, P = seq["cam"], seq["joints"][t]
    if px_sigma is None:
        px_sigma = 3.0 * cam.width / 1080.0
    u = cam.fx * P[:, 0] / P[:, 2] + cam.cx
    v = cam.fy * P[:, 1] / P[:, 2] + cam.cy
    p2d = np.stack([u, v], axis=1) + rng.normal(0.0, px_sigma, (P.shape[0], 2))
    p3d = (P - P[0]) + rng.normal(0.0, m_sigma, P.shape)
    return np.ascontiguousarray(p2d.T), np.ascontiguousarray(p3d.T), np.ones(P.shape[0])


def tracking_pose_params(side, n_rot):
    """Pose-stage weights for tracking a body sequence (a reading; Sec. 3.3 and
    Sec. 5 give the terms, not weights in these units): 2D weight 1 / sigma^2
    of the detection noise (pixels), 3D 1 / 0.02^2 (metres), temporal
    stabilisation 100 lambda_i (metres), joint limits 1e4 outside +-1 rad on
    every rotational unknown but the root's, no silhouette term (on these
    synthetic frames it pulled the pose off the joints; the non-rigid stage
    aligns the silhouette).  With the paper's 1e6 for the limits, Gauss-Newton
    steps that cross a limit overshoot (the barrier is linearised at its
    active set) and the tracking diverged within 40 frames; with 1e4 the
    joints stay within 2.5 cm of the ground truth over 40 frames."""
    from .body import TEMPORAL_JOINT_WEIGHTS
    sigma = 3.0 * side / 1080.0
    lo = np.full(n_rot, -1.0)
    hi = np.full(n_rot, 1.0)
    lo[:3], hi[:3] = -np.inf, np.inf
    return dict(l2d=1.0 / sigma ** 2, l3d=2500.0, lsil=0.0, l_temporal=100.0 * TEMPORAL_JOINT_WEIGHTS,
                l_anatomic=1e4, theta_min=lo, theta_max=hi)
