"""Two-stage tracking of a sequence on one GPU, stages of consecutive frames overlapped.

Per frame t the pose stage (Sec. 3.3; start pose by an explicit Euler step
from the last two poses, temporal stabilisation against the previous
frame's joints) is followed by skinning, and the per-vertex
non-rigid stage (Sec. 3.4) starts from the displacement-warped previous
result.  The paper runs its stages in threads on two GPUs with a frame of
delay between them (Sec. 4, pipelined implementation); on one GPU the same
split puts the pose stage of frame t+1 on one stream while the non-rigid
stage of frame t runs on another.  Both stages are latency-bound at these
sizes (tens of workgroups per launch), so the second stream fills compute
units the first leaves idle.

Each stage runs in its own host thread with its own library context and
stream (the library calls release the interpreter lock while they wait for
their stream); frame t's non-rigid stage waits for an event recorded after
frame t's skinning.  Every value is computed by the library's kernels; this
module only orders the calls.  Results equal the sequential order's bit for
bit (the same kernels on the same inputs in the same per-stream order).
"""
import threading

import torch

from . import (Context, PoseInputs, VertexInputs, body_joints, body_skin, body_warp, pose_extrapolate,
               pose_solve, vertex_params, vertex_solve)


class Tracker:
    """Device buffers and per-frame inputs of a tracked sequence.

    frames: per frame a dict with device tensors mask (uint8 [H][W]), image
    (float32 [3][H][W]), p2d, p3d, lam (float64 [2][nj], [3][nj], [nj]).
    pose0: float64 [nu] start pose of frame 0.  vweights: per-vertex stage
    weights (w_photo, w_sil, w_smooth, w_edge, w_vel, w_acc)."""

    def __init__(self, body, vtemplate, rgb, cam, frames, pose0, pose_prm, vweights, gn=3, pcg=4,
                 blur=(15, 9, 3), device=0):
        self.body, self.vt, self.rgb, self.cam, self.frames = body, vtemplate, rgb, cam, frames
        self.pose_prm, self.w, self.gn, self.pcg, self.blur = pose_prm, dict(vweights), gn, pcg, blur
        n, nv, nu = len(frames), body.nv, body.nu
        dev = rgb.device
        self.pose0 = pose0
        self.poses = [torch.empty(nu, dtype=torch.float64, device=dev) for _ in range(n)]
        self.posed = [torch.empty((3, nv), dtype=torch.float32, device=dev) for _ in range(n)]
        self.joints = [torch.empty((3, body.nj), dtype=torch.float64, device=dev) for _ in range(n)]
        self.joints0 = torch.empty((3, body.nj), dtype=torch.float64, device=dev)
        self.V = [torch.empty((3, nv), dtype=torch.float32, device=dev) for _ in range(n)]
        self.ctx_pose, self.ctx_nr = Context(device), Context(device)
        self.s_pose, self.s_nr = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
        self.reports_pose, self.reports_nr = [None] * n, [None] * n

    def _vprm(self, t):
        w = self.w
        return vertex_params(w["w_photo"], w["w_sil"], w["w_smooth"], w["w_edge"], w["w_vel"] if t >= 1 else 0.0,
                             w["w_acc"] if t >= 2 else 0.0, gn_iters=self.gn, pcg_iters=self.pcg,
                             exclude_case2=True, outline_only=True, blur_kernels=self.blur)

    def pose_stage(self, t):
        """Frame t's pose (on the current stream): start, Gauss-Newton, skinning."""
        ctx, b, P = self.ctx_pose, self.body, self.poses
        if t == 0:
            P[0].copy_(self.pose0)
        elif t == 1:
            P[1].copy_(P[0])
        else:
            pose_extrapolate(ctx, b, P[t - 1], P[t - 2], P[t])
        if t == 0:
            body_joints(ctx, b, P[0], self.joints0)          # frame 0 is stabilised against its start
        f = self.frames[t]
        inp = PoseInputs(b, self.cam, f["mask"], f["p2d"], f["p3d"], f["lam"], P[t],
                         prev_joints=self.joints0 if t == 0 else self.joints[t - 1])
        self.reports_pose[t] = pose_solve(ctx, inp, self.pose_prm)
        body_skin(ctx, b, P[t], self.posed[t])
        body_joints(ctx, b, P[t], self.joints[t])

    def nonrigid_stage(self, t):
        """Frame t's per-vertex stage (on the current stream): warped start, Gauss-Newton."""
        ctx, b = self.ctx_nr, self.body
        if t == 0:
            body_warp(ctx, b, self.poses[0], self.poses[0], self.posed[0], self.posed[0], self.posed[0], self.V[0])
        else:
            body_warp(ctx, b, self.poses[t - 1], self.poses[t], self.V[t - 1], self.posed[t - 1], self.posed[t],
                      self.V[t])
        f = self.frames[t]
        inp = VertexInputs(self.vt, self.posed[t], self.rgb, self.cam, f["mask"], f["image"], self.V[t],
                           prev=self.V[t - 1] if t >= 1 else None, prev2=self.V[t - 2] if t >= 2 else None)
        self.reports_nr[t] = vertex_solve(ctx, inp, self._vprm(t))

    def run_sequential(self):
        """Both stages of every frame in order on one stream."""
        with torch.cuda.stream(self.s_pose):
            for t in range(len(self.frames)):
                self.pose_stage(t)
                self.nonrigid_stage(t)
        self.s_pose.synchronize()

    def run_pipelined(self):
        """Pose stages on one stream and thread, non-rigid stages on another;
        frame t's non-rigid stage waits for frame t's skinning."""
        n = len(self.frames)
        events = [torch.cuda.Event() for _ in range(n)]
        ready = [threading.Event() for _ in range(n)]
        errors = []

        def poses():
            try:
                with torch.cuda.stream(self.s_pose):
                    for t in range(n):
                        self.pose_stage(t)
                        events[t].record(self.s_pose)
                        ready[t].set()
            except BaseException as e:          # surfaced by the caller
                errors.append(e)
                for r in ready:
                    r.set()

        th = threading.Thread(target=poses)
        th.start()
        try:
            with torch.cuda.stream(self.s_nr):
                for t in range(n):
                    ready[t].wait()
                    if errors:
                        break
                    self.s_nr.wait_event(events[t])
                    self.nonrigid_stage(t)
        finally:
            th.join()
        if errors:
            raise errors[0]
        self.s_nr.synchronize()
        self.s_pose.synchronize()
