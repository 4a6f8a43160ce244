"""Seeded non-rigid workloads (template, camera, ground truth, targets).

Recipe:

* Template: an ellipsoid with semi-axes (0.15, 0.5, 0.15) m (long axis along
  the image's +y), centred 2.5 m in front of the camera.  The small case uses
  an icosphere of subdivision level 4 (2,562 vertices, 5,120 faces); other
  sizes use a Fibonacci-spiral hull with exactly the requested vertex count.
* Vertex colours: i.i.d. uniform in [0, 1]^3 per vertex.
* Camera: pinhole, square image of side S, focal length 2S, principal point
  ((S-1)/2, (S-1)/2); world = camera frame (the paper's static camera).
* Ground truth: a smooth deformation field owned by this generator.  It picks
  ``n_ctrl`` control vertices at random, draws for each an axis-angle rotation
  with i.i.d. N(0, 0.05^2) rad components and a translation with i.i.d.
  N(0, 0.01^2) m components, and moves every vertex by the normalised
  Gaussian-RBF blend (over all control points) of those rigid motions.  The
  field is *not* expressed in the solver's deformation graph, so, as with real
  footage, the targets are not exactly reachable by the solver.
* Targets: mask and colour image rendered from the ground-truth mesh
  (``synth.render``), background colour 0.
"""
from dataclasses import dataclass

import numpy as np
from scipy.spatial.transform import Rotation

from .meshes import ellipsoid_icosphere, fibonacci_ellipsoid
from .render import render_targets

SEMI_AXES = (0.15, 0.5, 0.15)
CENTRE = (0.0, 0.0, 2.5)


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    @staticmethod
    def square(side):
        f = float(2 * side)
        c = (side - 1) / 2.0
        return Camera(int(side), int(side), f, f, c, c)

    def as_array(self):
        return np.array([self.fx, self.fy, self.cx, self.cy], dtype=np.float32)


# name -> recipe.  Weights are (w_sil, w_photo, w_arap); schedule is (GN, PCG).
CONFIGS = {
    # 2,562-vertex icosphere ellipsoid, 64 nodes, 256^2, 5 GN x 10 PCG.
    "small": dict(mesh="ico4", n_vertices=2562, n_nodes=64, side=256, gn=5, pcg=10,
                  weights=(1.0, 0.1, 10.0)),
    # paper-shaped non-rigid frame: 20,000 vertices, 500 nodes, 1080^2, 3 GN x 8 PCG.
    "frame20k": dict(mesh="fib", n_vertices=20000, n_nodes=500, side=1080, gn=3, pcg=8,
                     weights=(1.0, 0.1, 10.0)),
    # stress capture: 200,000 vertices, 4,000 nodes, 2048^2, 3 GN x 10 PCG.
    "stress200k": dict(mesh="fib", n_vertices=200000, n_nodes=4000, side=2048, gn=3, pcg=10,
                       weights=(1.0, 0.1, 10.0)),
}


def template_mesh(mesh, n_vertices):
    if mesh == "ico4":
        return ellipsoid_icosphere(4, SEMI_AXES, CENTRE)
    return fibonacci_ellipsoid(n_vertices, SEMI_AXES, CENTRE)


def smooth_field(xyz, n_ctrl, rng, rot_sigma=0.05, trans_sigma=0.01):
    """Ground-truth deformation: normalised Gaussian-RBF blend of random rigid motions."""
    p = xyz.T.astype(np.float64)
    ctrl = rng.choice(p.shape[0], size=n_ctrl, replace=False)
    c = p[ctrl]
    rot = Rotation.from_rotvec(rng.normal(0.0, rot_sigma, size=(n_ctrl, 3)))
    trans = rng.normal(0.0, trans_sigma, size=(n_ctrl, 3))
    # kernel width: mean distance from a control point to its nearest other one
    dcc = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=2)
    np.fill_diagonal(dcc, np.inf)
    sigma = dcc.min(axis=1).mean()
    out = np.zeros_like(p)
    wsum = np.zeros(p.shape[0])
    mats = rot.as_matrix()
    if n_ctrl * p.shape[0] <= 5e7:
        for m in range(n_ctrl):
            d2 = ((p - c[m]) ** 2).sum(axis=1)
            w = np.exp(-d2 / (2.0 * sigma * sigma))
            moved = (p - c[m]) @ mats[m].T + c[m] + trans[m]
            out += w[:, None] * moved
            wsum += w
    else:
        # large meshes: each control point only touches vertices within 6 sigma
        # (the kernel is below exp(-18) beyond), found with a k-d tree
        from scipy.spatial import cKDTree
        tree = cKDTree(p)
        for m in range(n_ctrl):
            idx = np.asarray(tree.query_ball_point(c[m], 6.0 * sigma), dtype=np.int64)
            if idx.size == 0:
                continue
            q = p[idx] - c[m]
            w = np.exp(-(q * q).sum(axis=1) / (2.0 * sigma * sigma))
            out[idx] += w[:, None] * (q @ mats[m].T + c[m] + trans[m])
            wsum[idx] += w
        far = wsum == 0.0          # beyond every control point's support: left in place
        out[far] = p[far]
        wsum[far] = 1.0
    out /= wsum[:, None]
    return np.ascontiguousarray(out.T.astype(np.float32))


def make_nonrigid_frame(name="small", seed=0, n_vertices=None, n_nodes=None, side=None):
    """One non-rigid frame: template, camera, ground truth and rendered targets."""
    cfg = dict(CONFIGS[name])
    if n_vertices is not None:
        cfg["n_vertices"] = n_vertices
        cfg["mesh"] = "fib"
    if n_nodes is not None:
        cfg["n_nodes"] = n_nodes
    if side is not None:
        cfg["side"] = side
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz, tri = template_mesh(cfg["mesh"], cfg["n_vertices"])
    rgb = rng.uniform(0.0, 1.0, size=(3, xyz.shape[1])).astype(np.float32)
    cam = Camera.square(cfg["side"])
    gt = smooth_field(xyz, cfg["n_nodes"], rng)
    mask, image = render_targets(gt, tri, rgb, cam)
    return dict(name=name, seed=seed, xyz=xyz, tri=tri, rgb=rgb, cam=cam, gt_xyz=gt,
                mask=mask, image=image, n_nodes=cfg["n_nodes"], gn=cfg["gn"], pcg=cfg["pcg"],
                weights=cfg["weights"])


def batch_specs(n=64, seed=0):
    """Sizes of a batch of independent frames: vertex count, node count and
    image side each drawn log-uniform (4,000-40,000 vertices, 128-1,000 nodes,
    512-1,080 px square images), plus a seed per frame."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def lu(lo, hi):
        return int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))

    specs = []
    for i in range(n):
        nv, nn, side = lu(4000, 40000), lu(128, 1000), lu(512, 1080)
        specs.append(dict(n_vertices=nv, n_nodes=min(nn, nv), side=side, seed=1000 * seed + i))
    return specs


def _batch_frame(spec):
    return make_nonrigid_frame("frame20k", spec["seed"], n_vertices=spec["n_vertices"], n_nodes=spec["n_nodes"],
                               side=spec["side"])


def make_batch(n=64, seed=0, workers=8):
    """The frames of ``batch_specs`` (generated in worker processes)."""
    specs = batch_specs(n, seed)
    if workers <= 1:
        return [_batch_frame(s) for s in specs]
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_batch_frame, specs))
