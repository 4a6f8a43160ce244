"""MI355X-native per-frame Gauss-Newton solvers (LiveCap pose and non-rigid stages).

Thin Python binding over the C ABI in ``libcapture.so`` (include/capture.h).
PyTorch only provides device memory and the stream: every step of the solve
runs in the library's HIP kernels.  Nothing here computes on the CPU; if the
library is missing, calls fail loudly.
"""
import ctypes as C
import math

import torch

from . import capi
from .capi import CaptureError  # noqa: F401

__all__ = ["Context", "Template", "FrameInputs", "graph_build", "CaptureError", "Body", "PoseInputs",
           "pose_params", "pose_solve", "pose_linearize", "autotune_tiles", "VertexTemplate", "VertexInputs",
           "vertex_params", "vertex_solve", "vertex_linearize", "body_skin", "body_warp", "pose_extrapolate",
           "body_joints"]


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(None)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, shape, name):
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError("%s must be a contiguous CUDA %s tensor of shape %s (got %s %s %s)"
                         % (name, dtype, tuple(shape), t.device, t.dtype, tuple(t.shape)))


class Context:
    """A library context on one device (owns nothing but the device id)."""

    def __init__(self, device=0):
        self.lib = capi.load()
        self.device = device
        h = C.c_void_p()
        capi.check(self.lib.capture_create(C.byref(h), device))
        self.h = h
        self._ws = None

    def close(self):
        if self.h:
            self.lib.capture_destroy(self.h)
            self.h = None

    def workspace(self, nbytes):
        """A device byte buffer of at least nbytes (kept and reused)."""
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda:%d" % self.device)
        return self._ws

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def graph_build(ctx, xyz, n_nodes):
    """Farthest-point nodes, 4-nearest binding and 8-nearest node edges."""
    nv = xyz.shape[1]
    _need(xyz, torch.float32, (3, nv), "xyz")
    dev = xyz.device
    g = dict(node_vertex=torch.empty(n_nodes, dtype=torch.int32, device=dev),
             bind_idx=torch.empty((4, nv), dtype=torch.int32, device=dev),
             bind_w=torch.empty((4, nv), dtype=torch.float32, device=dev),
             edge_dst=torch.empty((8, n_nodes), dtype=torch.int32, device=dev))
    capi.check(ctx.lib.capture_graph_build(ctx.h, _ptr(xyz), nv, n_nodes, _ptr(g["node_vertex"]),
                                           _ptr(g["bind_idx"]), _ptr(g["bind_w"]), _ptr(g["edge_dst"]),
                                           _stream()))
    return g


class Template:
    """Mesh topology plus deformation graph, planned for the device."""

    def __init__(self, ctx, tri, graph, vertices_per_tile=0):
        nf = tri.shape[1]
        nv = graph["bind_idx"].shape[1]
        nn = graph["node_vertex"].shape[0]
        _need(tri, torch.int32, (3, nf), "tri")
        _need(graph["node_vertex"], torch.int32, (nn,), "node_vertex")
        _need(graph["bind_idx"], torch.int32, (4, nv), "bind_idx")
        _need(graph["bind_w"], torch.float32, (4, nv), "bind_w")
        _need(graph["edge_dst"], torch.int32, (8, nn), "edge_dst")
        self.ctx = ctx
        self.nv, self.nf, self.nn = nv, nf, nn
        d = capi.TemplateDesc(nv, nf, nn, _ptr(tri), _ptr(graph["node_vertex"]), _ptr(graph["bind_idx"]),
                              _ptr(graph["bind_w"]), _ptr(graph["edge_dst"]), vertices_per_tile)
        h = C.c_void_p()
        capi.check(ctx.lib.capture_template_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h
        info = capi.TemplateInfo()
        capi.check(ctx.lib.capture_template_info_get(h, C.byref(info)))
        self.info = {name: getattr(info, name) for name, _ in capi.TemplateInfo._fields_}
        self.n_tiles = info.n_tiles

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.capture_template_destroy(self.h)
                self.h = None
        except Exception:
            pass


class FrameInputs:
    """Device tensors of one frame (see capture_frame)."""

    def __init__(self, template, xyz, rgb, camera, mask, image, node_state):
        nv, nn = template.nv, template.nn
        W, H = int(camera.width), int(camera.height)
        _need(xyz, torch.float32, (3, nv), "xyz")
        _need(rgb, torch.float32, (3, nv), "rgb")
        _need(mask, torch.uint8, (H, W), "mask")
        _need(image, torch.float32, (3, H, W), "image")
        _need(node_state, torch.float32, (12, nn), "node_state")
        self.template, self.xyz, self.rgb, self.mask, self.image, self.node_state = (
            template, xyz, rgb, mask, image, node_state)
        self.camera = capi.Camera(W, H, float(camera.fx), float(camera.fy), float(camera.cx), float(camera.cy))

    def struct(self):
        return capi.Frame(self.template.h, _ptr(self.xyz), _ptr(self.rgb), self.camera, _ptr(self.mask),
                          _ptr(self.image), _ptr(self.node_state))


def params(w_sil=1.0, w_photo=0.1, w_arap=10.0, gn_iters=5, pcg_iters=10, tau_color=math.inf, w_vel=0.0,
           exclude_case2=False, outline_only=False, pcg_tol=0.0, pcg_standard=False):
    flags = ((capi.FLAG_EXCLUDE_CASE2 if exclude_case2 else 0) | (capi.FLAG_OUTLINE_ONLY if outline_only else 0) |
             (capi.FLAG_PCG_STANDARD if pcg_standard else 0))
    return capi.NonrigidParams(w_sil, w_photo, w_arap, tau_color, w_vel, gn_iters, pcg_iters, flags, pcg_tol)


def _frames(frames):
    arr = (capi.Frame * len(frames))()
    for i, f in enumerate(frames):
        arr[i] = f.struct()
    return arr


def workspace_bytes(ctx, frames):
    arr = _frames(frames)
    n = C.c_size_t()
    capi.check(ctx.lib.capture_workspace_size(ctx.h, len(frames), arr, C.byref(n)))
    return n.value


def _report_dict(r, gn):
    return dict(energy=[r.energy[k] for k in range(r.gn_done + 1)], e_photo=r.e_photo, e_sil=r.e_sil,
                e_sil_abs=r.e_sil_abs, e_arap=r.e_arap, e_vel=r.e_vel, n_visible=r.n_visible,
                n_boundary=r.n_boundary, gn_done=r.gn_done, status=r.status, warm_start=r.warm_start,
                energy_prev=r.energy_prev, energy_pred=r.energy_pred)


def batch_solve(ctx, frames, prm):
    """Solve every frame in place (node_state); returns one report dict per frame."""
    arr = _frames(frames)
    nbytes = workspace_bytes(ctx, frames)
    ws = ctx.workspace(nbytes)
    reps = (capi.Report * len(frames))()
    capi.check(ctx.lib.capture_batch_solve(ctx.h, len(frames), arr, C.byref(prm), reps, _ptr(ws),
                                           ws.numel(), _stream()))
    return [_report_dict(reps[i], prm.gn_iters) for i in range(len(frames))]


def nonrigid_solve(ctx, frame, prm):
    arr = _frames([frame])
    ws = ctx.workspace(workspace_bytes(ctx, [frame]))
    rep = capi.Report()
    capi.check(ctx.lib.capture_nonrigid_solve(ctx.h, arr, C.byref(prm), C.byref(rep), _ptr(ws), ws.numel(),
                                              _stream()))
    return _report_dict(rep, prm.gn_iters)


def nonrigid_solve_noalloc(ctx, frame, prm):
    """capture_nonrigid_solve_noalloc: the solve with the library's fixed device scratch."""
    arr = _frames([frame])
    rep = capi.Report()
    capi.check(ctx.lib.capture_nonrigid_solve_noalloc(ctx.h, arr, C.byref(prm), C.byref(rep), _stream()))
    return _report_dict(rep, prm.gn_iters)


def autotune_tiles(ctx, tris, graphs, frames, prm, candidates=(64, 128, 192, 256)):
    """Pick vertices_per_tile by timing batched solves of `frames` with templates
    rebuilt from (tri, graph) at each candidate; frames' node states are kept.
    Returns (best, {candidate: best ms})."""
    n = len(frames)
    keep = []
    descs = (capi.TemplateDesc * n)()
    for i, (tri, g) in enumerate(zip(tris, graphs)):
        nv = g["bind_idx"].shape[1]
        descs[i] = capi.TemplateDesc(nv, tri.shape[1], g["node_vertex"].shape[0], _ptr(tri), _ptr(g["node_vertex"]),
                                     _ptr(g["bind_idx"]), _ptr(g["bind_w"]), _ptr(g["edge_dst"]), 0)
        keep.append((tri, g))
    cand = (C.c_int32 * len(candidates))(*candidates)
    times = (C.c_double * len(candidates))()
    best = C.c_int32()
    capi.check(ctx.lib.capture_autotune_tiles(ctx.h, n, descs, _frames(frames), C.byref(prm), cand, len(candidates),
                                              C.byref(best), times, _stream()))
    return best.value, {c: times[k] for k, c in enumerate(candidates)}


def frame_decisions(ctx, frame):
    """Per-frame preprocessing outputs: dt, blurred, zbuf, vflags (device tensors)."""
    arr = _frames([frame])
    ws = ctx.workspace(workspace_bytes(ctx, [frame]))
    H, W = frame.camera.height, frame.camera.width
    dev = frame.xyz.device
    out = dict(dt=torch.empty((H, W), dtype=torch.float32, device=dev),
               blurred=torch.empty((3, H, W), dtype=torch.float32, device=dev),
               zbuf=torch.empty((H, W), dtype=torch.int32, device=dev),
               vflags=torch.empty(frame.template.nv, dtype=torch.uint8, device=dev))
    capi.check(ctx.lib.capture_frame_decisions(ctx.h, arr, _ptr(out["dt"]), _ptr(out["blurred"]),
                                               _ptr(out["zbuf"]), _ptr(out["vflags"]), _ptr(ws), ws.numel(),
                                               _stream()))
    return out


def linearize(ctx, frame, prm, p=None):
    """rhs, diag (and A p) at the frame's node_state, plus the 5 energy terms."""
    arr = _frames([frame])
    ws = ctx.workspace(workspace_bytes(ctx, [frame]))
    nn = frame.template.nn
    dev = frame.xyz.device
    rhs = torch.empty((6, nn), dtype=torch.float32, device=dev)
    diag = torch.empty((6, nn), dtype=torch.float32, device=dev)
    Ap = torch.empty((6, nn), dtype=torch.float32, device=dev) if p is not None else None
    if p is not None:
        _need(p, torch.float32, (6, nn), "p")
    e = (C.c_double * 5)()
    capi.check(ctx.lib.capture_linearize(ctx.h, arr, C.byref(prm), _ptr(rhs), _ptr(diag), _ptr(p), _ptr(Ap), e,
                                         _ptr(ws), ws.numel(), _stream()))
    return dict(rhs=rhs, diag=diag, Ap=Ap, energy=list(e))


def set_graphs(ctx, on=True):
    """Replay solves from captured HIP graphs (see capture_set_graphs)."""
    capi.check(ctx.lib.capture_set_graphs(ctx.h, 1 if on else 0))


def profile_enable(ctx, on=True):
    """Bracket every solver-kernel launch with HIP events (see capture_profile_enable)."""
    capi.check(ctx.lib.capture_profile_enable(ctx.h, 1 if on else 0))


def profile_read(ctx):
    """{kernel: (total_ms, launches)} since the last read; resets the counters."""
    out = {}
    for name in capi.KERNELS:
        ms = C.c_double()
        n = C.c_int64()
        capi.check(ctx.lib.capture_profile_read(ctx.h, name.encode(), C.byref(ms), C.byref(n)))
        out[name] = (ms.value, n.value)
    return out


class WarmStart:
    """The learned warm-start network (library-owned weights and Adam state)."""

    def __init__(self, ctx, max_nodes, params):
        import numpy as np
        self.ctx = ctx
        w = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if w.size != capi.WS_PARAMS:
            raise ValueError("need %d parameters" % capi.WS_PARAMS)
        h = C.c_void_p()
        capi.check(ctx.lib.capture_warmstart_create(ctx.h, max_nodes, w.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.capture_warmstart_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def set_scaling(self, mean, std):
        import numpy as np
        m = np.ascontiguousarray(np.asarray(mean, np.float32)[:27])
        s = np.ascontiguousarray(np.asarray(std, np.float32)[:27])
        capi.check(self.ctx.lib.capture_warmstart_set_scaling(self.h, m.ctypes.data_as(C.c_void_p),
                                                              s.ctypes.data_as(C.c_void_p)))

    def fit_scaling(self, features):
        _need(features, torch.float32, (features.shape[0], 32), "features")
        capi.check(self.ctx.lib.capture_warmstart_fit_scaling(self.ctx.h, self.h, _ptr(features),
                                                              features.shape[0], _stream()))

    def params(self):
        import numpy as np
        out = np.zeros(capi.WS_PARAMS, np.float32)
        steps = C.c_int64()
        capi.check(self.ctx.lib.capture_warmstart_get_params(self.h, out.ctypes.data_as(C.c_void_p),
                                                             C.byref(steps)))
        return out, steps.value

    def forward(self, template, features):
        _need(features, torch.float32, (template.nn, 32), "features")
        y = torch.empty((template.nn, 6), dtype=torch.float32, device=features.device)
        capi.check(self.ctx.lib.capture_warmstart_forward(self.ctx.h, self.h, template.h, _ptr(features), _ptr(y),
                                                          _stream()))
        return y

    def train_step(self, template, features, target, lr=1e-3, update=True, grads=None):
        _need(features, torch.float32, (template.nn, 32), "features")
        _need(target, torch.float32, (template.nn, 6), "target")
        if grads is not None:
            _need(grads, torch.float32, (capi.WS_PARAMS,), "grads")
        loss = C.c_double()
        capi.check(self.ctx.lib.capture_warmstart_train_step(self.ctx.h, self.h, template.h, _ptr(features),
                                                             _ptr(target), lr, 1 if update else 0, _ptr(grads),
                                                             C.byref(loss), _stream()))
        return loss.value


def warmstart_features(ctx, frame, prm, state_prev2=None):
    """Raw features [n_nodes][32] at the frame's node_state."""
    arr = _frames([frame])
    ws = ctx.workspace(workspace_bytes(ctx, [frame]))
    X = torch.empty((frame.template.nn, 32), dtype=torch.float32, device=frame.xyz.device)
    capi.check(ctx.lib.capture_warmstart_features(ctx.h, arr, _ptr(state_prev2), C.byref(prm), _ptr(X), _ptr(ws),
                                                  ws.numel(), _stream()))
    return X


def warmstart_target(ctx, state_prev, state_next):
    nn = state_prev.shape[1]
    _need(state_prev, torch.float32, (12, nn), "state_prev")
    _need(state_next, torch.float32, (12, nn), "state_next")
    t = torch.empty((nn, 6), dtype=torch.float32, device=state_prev.device)
    capi.check(ctx.lib.capture_warmstart_target(ctx.h, nn, _ptr(state_prev), _ptr(state_next), _ptr(t), _stream()))
    return t


def nonrigid_solve_warm(ctx, frame, prm, net, state_prev2=None, target_energy=-math.inf):
    """Solve from the network's predicted start (or the frame's state when that is better)."""
    arr = _frames([frame])
    ws = ctx.workspace(workspace_bytes(ctx, [frame]))
    rep = capi.Report()
    capi.check(ctx.lib.capture_nonrigid_solve_warm(ctx.h, arr, C.byref(prm), net.h, _ptr(state_prev2),
                                                   float(target_energy), C.byref(rep), _ptr(ws), ws.numel(),
                                                   _stream()))
    return _report_dict(rep, prm.gn_iters)


# ---------------------------------------------------------------- pose stage
class Body:
    """Skeleton, skinned mesh and mesh tables of the pose stage (capture_body)."""

    def __init__(self, ctx, tri, xyz, bind_joint, bind_w, parents, rest_joints, has_rotation):
        nf = tri.shape[1]
        nv = xyz.shape[1]
        nj = len(parents)
        _need(tri, torch.int32, (3, nf), "tri")
        _need(xyz, torch.float32, (3, nv), "xyz")
        _need(bind_joint, torch.int32, (4, nv), "bind_joint")
        _need(bind_w, torch.float32, (4, nv), "bind_w")
        par = (C.c_int32 * nj)(*[int(p) for p in parents])
        rest = (C.c_double * (3 * nj))(*[float(x) for x in rest_joints.reshape(-1)])
        rot = (C.c_int32 * nj)(*[int(bool(r)) for r in has_rotation])
        d = capi.BodyDesc(nv, nf, nj, _ptr(tri), _ptr(xyz), _ptr(bind_joint), _ptr(bind_w),
                          C.cast(par, C.c_void_p), C.cast(rest, C.c_void_p), C.cast(rot, C.c_void_p))
        h = C.c_void_p()
        capi.check(ctx.lib.capture_body_create(ctx.h, C.byref(d), C.byref(h)))
        self.ctx, self.h, self.nv, self.nf, self.nj = ctx, h, nv, nf, nj
        n = C.c_int32()
        capi.check(ctx.lib.capture_body_unknowns(h, C.byref(n)))
        self.nu = n.value

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.capture_body_destroy(self.h)
                self.h = None
        except Exception:
            pass


class PoseInputs:
    """Device tensors of one pose frame (see capture_pose_frame)."""

    def __init__(self, body, camera, mask, p2d, p3d, lam, pose, prev_joints=None):
        W, H = int(camera.width), int(camera.height)
        nj = body.nj
        _need(mask, torch.uint8, (H, W), "mask")
        _need(p2d, torch.float64, (2, nj), "p2d")
        _need(p3d, torch.float64, (3, nj), "p3d")
        _need(lam, torch.float64, (nj,), "lambda")
        _need(pose, torch.float64, (body.nu,), "pose")
        if prev_joints is not None:
            _need(prev_joints, torch.float64, (3, nj), "prev_joints")
        self.body, self.mask, self.p2d, self.p3d, self.lam, self.pose = body, mask, p2d, p3d, lam, pose
        self.prev_joints = prev_joints
        self.camera = capi.Camera(W, H, float(camera.fx), float(camera.fy), float(camera.cx), float(camera.cy))

    def struct(self):
        return capi.PoseFrame(self.body.h, self.camera, _ptr(self.mask), _ptr(self.p2d), _ptr(self.p3d),
                              _ptr(self.lam), _ptr(self.pose), _ptr(self.prev_joints))


def pose_params(l2d=1.0 / 9.0, l3d=2500.0, lsil=0.05, gn_iters=3, exclude_case2=True, outline_only=True,
                l_temporal=None, l_anatomic=0.0, theta_min=None, theta_max=None):
    """l_temporal: per-joint temporal weights (lambda_temporal * lambda_j);
    theta_min / theta_max: limits of the rotational unknowns (default unlimited)."""
    flags = (capi.FLAG_EXCLUDE_CASE2 if exclude_case2 else 0) | (capi.FLAG_OUTLINE_ONLY if outline_only else 0)
    lt = (C.c_double * capi.MAX_JOINTS)(*([float(x) for x in l_temporal] if l_temporal is not None else []))
    lo = (C.c_double * capi.MAX_POSE_UNKNOWNS)(*([-math.inf] * capi.MAX_POSE_UNKNOWNS))
    hi = (C.c_double * capi.MAX_POSE_UNKNOWNS)(*([math.inf] * capi.MAX_POSE_UNKNOWNS))
    for q, x in enumerate(theta_min if theta_min is not None else []):
        lo[q] = float(x)
    for q, x in enumerate(theta_max if theta_max is not None else []):
        hi[q] = float(x)
    return capi.PoseParams(l2d, l3d, lsil, gn_iters, flags, lt, l_anatomic, lo, hi)


def _pose_ws(ctx, fr):
    n = C.c_size_t()
    capi.check(ctx.lib.capture_pose_workspace_size(ctx.h, C.byref(fr), C.byref(n)))
    return ctx.workspace(n.value)


def pose_solve(ctx, frame, prm):
    """Gauss-Newton pose solve in place (frame.pose); returns the report as a dict."""
    fr = frame.struct()
    ws = _pose_ws(ctx, fr)
    rep = capi.PoseReport()
    capi.check(ctx.lib.capture_pose_solve(ctx.h, C.byref(fr), C.byref(prm), C.byref(rep), _ptr(ws), ws.numel(),
                                          _stream()))
    return dict(energy=[rep.energy[k] for k in range(rep.gn_done + 1)], e2d=rep.e2d, e3d=rep.e3d,
                e_sil=rep.e_sil, e_sil_abs=rep.e_sil_abs, e_temporal=rep.e_temporal, e_anatomic=rep.e_anatomic,
                n_visible=rep.n_visible, n_boundary=rep.n_boundary,
                gn_done=rep.gn_done, status=rep.status)


def pose_linearize(ctx, frame, prm):
    """Decisions and normal equations at frame.pose: system [nu][nu+1] (J^T J | -J^T B F),
    the 6 energy terms (2D, 3D, silhouette, silhouette with |b|, temporal, limits) and the vertex flags."""
    fr = frame.struct()
    ws = _pose_ws(ctx, fr)
    nu = frame.body.nu
    dev = frame.pose.device
    system = torch.empty((nu, nu + 1), dtype=torch.float64, device=dev)
    vflags = torch.empty(frame.body.nv, dtype=torch.uint8, device=dev)
    e = (C.c_double * 6)()
    capi.check(ctx.lib.capture_pose_linearize(ctx.h, C.byref(fr), C.byref(prm), _ptr(system), e, _ptr(vflags),
                                              _ptr(ws), ws.numel(), _stream()))
    return dict(system=system, energy=list(e), vflags=vflags)


# ---------------------------------------------------------------- per-vertex non-rigid stage
class VertexTemplate:
    """Mesh, rest pose and material classes (Table 1) of the per-vertex stage."""

    def __init__(self, ctx, tri, rest, classes, parts=None):
        nf, nv = tri.shape[1], rest.shape[1]
        _need(tri, torch.int32, (3, nf), "tri")
        _need(rest, torch.float32, (3, nv), "rest")
        _need(classes, torch.int32, (nv,), "classes")
        if parts is not None:
            _need(parts, torch.int32, (nv,), "parts")
        self.ctx, self.nv, self.nf = ctx, nv, nf
        d = capi.VertexTemplateDesc(nv, nf, _ptr(tri), _ptr(rest), _ptr(classes), _ptr(parts))
        h = C.c_void_p()
        capi.check(ctx.lib.capture_vertex_template_create(ctx.h, C.byref(d), C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if self.h:
                self.ctx.lib.capture_vertex_template_destroy(self.h)
                self.h = None
        except Exception:
            pass


class VertexInputs:
    """Device tensors of one per-vertex frame (see capture_vertex_frame); V is updated in place."""

    def __init__(self, template, posed, rgb, camera, mask, image, V, prev=None, prev2=None):
        nv = template.nv
        W, H = int(camera.width), int(camera.height)
        for t, name in ((posed, "posed"), (rgb, "rgb"), (V, "V")):
            _need(t, torch.float32, (3, nv), name)
        for t, name in ((prev, "prev"), (prev2, "prev2")):
            if t is not None:
                _need(t, torch.float32, (3, nv), name)
        _need(mask, torch.uint8, (H, W), "mask")
        _need(image, torch.float32, (3, H, W), "image")
        self.template, self.posed, self.rgb, self.mask, self.image, self.V = template, posed, rgb, mask, image, V
        self.prev, self.prev2 = prev, prev2
        self.camera = capi.Camera(W, H, float(camera.fx), float(camera.fy), float(camera.cx), float(camera.cy))

    def struct(self):
        return capi.VertexFrame(self.template.h, _ptr(self.posed), _ptr(self.prev), _ptr(self.prev2), _ptr(self.rgb),
                                self.camera, _ptr(self.mask), _ptr(self.image), _ptr(self.V))


def vertex_params(w_photo, w_sil, w_smooth, w_edge, w_vel=0.0, w_acc=0.0, gn_iters=3, pcg_iters=4,
                  tau_color=math.inf, exclude_case2=False, outline_only=False, blur_kernels=None, snap_max_px=0.0,
                  snap_steps=4, snap_rings=2, snap_iters=8, part_mask=False, part_dilation=10):
    flags = ((capi.FLAG_EXCLUDE_CASE2 if exclude_case2 else 0) | (capi.FLAG_OUTLINE_ONLY if outline_only else 0) |
             (capi.FLAG_PART_MASK if part_mask else 0))
    bk = (C.c_int32 * capi.MAX_GN)()
    for g, k in enumerate(blur_kernels or ()):
        bk[g] = int(k)
    return capi.VertexParams(w_photo, w_sil, w_smooth, w_edge, w_vel, w_acc, tau_color, gn_iters, pcg_iters, flags,
                             bk, snap_max_px, snap_steps, snap_rings, snap_iters, part_dilation)


def _vertex_ws(ctx, fr, prm):
    n = C.c_size_t()
    capi.check(ctx.lib.capture_vertex_workspace_size(ctx.h, C.byref(fr), C.byref(prm), C.byref(n)))
    return ctx.workspace(n.value)


def vertex_solve(ctx, frame, prm):
    """Gauss-Newton solve of one per-vertex frame; frame.V holds the result."""
    fr = frame.struct()
    ws = _vertex_ws(ctx, fr, prm)
    rep = capi.VertexReport()
    capi.check(ctx.lib.capture_vertex_solve(ctx.h, C.byref(fr), C.byref(prm), C.byref(rep), _ptr(ws), ws.numel(),
                                            _stream()))
    g = rep.gn_done
    out = {name: getattr(rep, name) for name, _ in capi.VertexReport._fields_ if name != "energy"}
    out["energy"] = [rep.energy[k] for k in range(g + 1)]
    return out


def vertex_linearize(ctx, frame, prm, p=None):
    """Decisions and one linearisation at frame.V: rhs, diag (float64 [3][nv]),
    J^T |B| J p if p is given, the 7 energy terms and the vertex flags."""
    nv = frame.template.nv
    fr = frame.struct()
    ws = _vertex_ws(ctx, fr, prm)
    dev = frame.V.device
    rhs = torch.empty((3, nv), dtype=torch.float64, device=dev)
    diag = torch.empty_like(rhs)
    Ap = torch.empty_like(rhs) if p is not None else None
    if p is not None:
        _need(p, torch.float64, (3, nv), "p")
    flags = torch.empty(nv, dtype=torch.uint8, device=dev)
    en = (C.c_double * 7)()
    capi.check(ctx.lib.capture_vertex_linearize(ctx.h, C.byref(fr), C.byref(prm), _ptr(rhs), _ptr(diag), _ptr(p),
                                                _ptr(Ap), en, _ptr(flags), _ptr(ws), ws.numel(), _stream()))
    return dict(rhs=rhs, diag=diag, Ap=Ap, energy=list(en), vflags=flags)


# ---------------------------------------------------------------- between stages and frames (enqueue only)
def body_skin(ctx, body, pose, out):
    """out [3][nv] float32 <- skinned mesh of `body` at `pose` (float64 [nu])."""
    _need(pose, torch.float64, (body.nu,), "pose")
    _need(out, torch.float32, (3, body.nv), "out")
    capi.check(ctx.lib.capture_body_skin(ctx.h, body.h, _ptr(pose), _ptr(out), _stream()))
    return out


def body_warp(ctx, body, pose_prev, pose_cur, V_prev, posed_prev, posed_cur, out):
    """out <- posed_cur + M_cur M_prev^T (V_prev - posed_prev) (displacement warping)."""
    for t, name in ((pose_prev, "pose_prev"), (pose_cur, "pose_cur")):
        _need(t, torch.float64, (body.nu,), name)
    for t, name in ((V_prev, "V_prev"), (posed_prev, "posed_prev"), (posed_cur, "posed_cur"), (out, "out")):
        _need(t, torch.float32, (3, body.nv), name)
    capi.check(ctx.lib.capture_body_warp(ctx.h, body.h, _ptr(pose_prev), _ptr(pose_cur), _ptr(V_prev),
                                         _ptr(posed_prev), _ptr(posed_cur), _ptr(out), _stream()))
    return out


def pose_extrapolate(ctx, body, pose_prev, pose_prev2, out):
    """out <- pose_prev + (pose_prev - pose_prev2) (explicit Euler step)."""
    for t, name in ((pose_prev, "pose_prev"), (pose_prev2, "pose_prev2"), (out, "out")):
        _need(t, torch.float64, (body.nu,), name)
    capi.check(ctx.lib.capture_pose_extrapolate(ctx.h, body.h, _ptr(pose_prev), _ptr(pose_prev2), _ptr(out),
                                                _stream()))
    return out


def body_joints(ctx, body, pose, out):
    """out [3][nj] float64 <- joint positions at `pose`."""
    _need(pose, torch.float64, (body.nu,), "pose")
    _need(out, torch.float64, (3, body.nj), "out")
    capi.check(ctx.lib.capture_body_joints(ctx.h, body.h, _ptr(pose), _ptr(out), _stream()))
    return out
