"""Seeded procedural body: skeleton, skinned mesh, poses, detections and targets.

Stand-in for the paper's scanned actor (Sec. 3.1: template of about 5000
vertices, manually placed skeleton, skinning weights from an auto-rigger)
and for the CNN joint detections (Sec. 3.3, 2D and 3D joints).

Skeleton: 23 joints (pelvis root; spine1, spine2, neck, head; per side
clavicle, shoulder, elbow, wrist, hand end; per side hip, knee, ankle, toe),
body height 1.7 m, camera frame (+y points down the image).
Mesh: one closed ellipsoid per bone (Fibonacci hulls), vertex counts by
surface area summing exactly to the requested count; parts may overlap.
Skinning: each vertex binds to the 4 bones nearest to it (segment distance),
weights exp(-d^2 / (2 * 0.04^2)) normalised; a bone moves with its parent
joint.
"""
import numpy as np

from .meshes import fibonacci_ellipsoid
from .render import render_targets
from .workloads import Camera

JOINTS = ["pelvis", "spine1", "spine2", "neck", "head",
          "l_clavicle", "l_shoulder", "l_elbow", "l_wrist", "l_hand",
          "r_clavicle", "r_shoulder", "r_elbow", "r_wrist", "r_hand",
          "l_hip", "l_knee", "l_ankle", "l_toe",
          "r_hip", "r_knee", "r_ankle", "r_toe"]
PARENTS = np.array([-1, 0, 1, 2, 3, 2, 5, 6, 7, 8, 2, 10, 11, 12, 13, 0, 15, 16, 17, 0, 19, 20, 21], np.int32)
# joints without their own rotation (hand ends)
NO_DOF = (9, 14)

# rest joint positions relative to the pelvis (metres, +y down, +z away from the camera)
_REST = np.array([
    [0.00, 0.00, 0.00], [0.00, -0.12, 0.00], [0.00, -0.30, 0.00], [0.00, -0.50, 0.00], [0.00, -0.72, 0.00],
    [0.06, -0.46, 0.00], [0.19, -0.45, 0.00], [0.45, -0.45, 0.00], [0.70, -0.45, 0.00], [0.80, -0.45, 0.00],
    [-0.06, -0.46, 0.00], [-0.19, -0.45, 0.00], [-0.45, -0.45, 0.00], [-0.70, -0.45, 0.00], [-0.80, -0.45, 0.00],
    [0.10, 0.05, 0.00], [0.10, 0.48, 0.00], [0.10, 0.88, 0.02], [0.10, 0.92, -0.12],
    [-0.10, 0.05, 0.00], [-0.10, 0.48, 0.00], [-0.10, 0.88, 0.02], [-0.10, 0.92, -0.12]])

# end points of the bones that hang off the head and toe joints (so that their
# rotations move vertices): head top and toe tips
_ENDS = {4: np.array([0.00, -0.94, 0.00]), 18: np.array([0.10, 0.93, -0.20]), 22: np.array([-0.10, 0.93, -0.20])}

# (start point, end point, radius) per body part; an int is a joint, a key into _ENDS
# prefixed with "e" is a bone end
_PARTS = [(0, 2, 0.16), (2, 3, 0.10), (4, "e4", 0.11), (6, 7, 0.055), (7, 8, 0.045), (8, 9, 0.04),
          (11, 12, 0.055), (12, 13, 0.045), (13, 14, 0.04), (15, 16, 0.08), (16, 17, 0.06),
          (17, 18, 0.045), (18, "e18", 0.04), (19, 20, 0.08), (20, 21, 0.06), (21, 22, 0.045),
          (22, "e22", 0.04), (5, 6, 0.05), (10, 11, 0.05)]


# material class (Table 1 class id) of each part: a synthetic stand-in for the
# per-vertex semantic labels of the paper's template (Sec. 3.1): pelvis part
# loose (1, dress/skirt), chest, neck and clavicles upper clothes (2), head
# face/hair (7), arms (5), hands gloves (6), legs pants (3), feet shoes (6)
PART_CLASS = np.array([1, 2, 7, 5, 5, 6, 5, 5, 6, 3, 3, 6, 6, 3, 3, 6, 6, 2, 2], np.int32)


# body-part label of each part for the silhouette term's part mask: 0 torso
# (pelvis, chest, neck, clavicles), 1 head, 2 / 3 left / right arm (upper arm,
# forearm, hand), 4 / 5 left / right leg (thigh, shin, foot, toe)
PART_GROUP = np.array([0, 0, 1, 2, 2, 2, 3, 3, 3, 4, 4, 4, 4, 5, 5, 5, 5, 0, 0], np.int32)

# Per-joint temporal smoothness weights lambda_i of the pose stage (Sec. 3.3:
# 2.5 torso and head, 2.0 shoulders, 1.5 knees and elbows, 1.0 hands and
# feet), mapped onto this skeleton: clavicles count as shoulders, hips as
# torso, wrists and hand ends as hands, ankles and toes as feet.
TEMPORAL_JOINT_WEIGHTS = np.array([2.5, 2.5, 2.5, 2.5, 2.5,
                                   2.0, 2.0, 1.5, 1.0, 1.0,
                                   2.0, 2.0, 1.5, 1.0, 1.0,
                                   2.5, 1.5, 1.0, 1.0,
                                   2.5, 1.5, 1.0, 1.0])


def dof_joints():
    """Joints that carry 3 axis-angle unknowns, in unknown order (pelvis first)."""
    return [j for j in range(len(JOINTS)) if j not in NO_DOF]


def _frame(d):
    d = d / np.linalg.norm(d)
    a = np.array([1.0, 0.0, 0.0]) if abs(d[0]) < 0.9 else np.array([0.0, 0.0, 1.0])
    u = np.cross(d, a)
    u /= np.linalg.norm(u)
    return np.stack([u, d, np.cross(u, d)], axis=1)     # columns: across, along, across


def make_body(n_vertices, root=(0.0, 0.0, 4.0)):
    """Rest mesh (posed at the root), rest joints, topology and LBS binding."""
    J = _REST + np.asarray(root)

    def pt(x):
        return J[x] if not isinstance(x, str) else _ENDS[int(x[1:])] + np.asarray(root)

    lens = []
    for a, b, r in _PARTS:
        L = np.linalg.norm(pt(b) - pt(a))
        h = 0.5 * L + 0.6 * r
        lens.append((h, r))
    area = np.array([4 * np.pi * ((h * r) ** 1.6 * 2 + (r * r) ** 1.6) ** (1 / 1.6) / 3 ** (1 / 1.6)
                     for h, r in lens])
    counts = np.maximum(32, np.floor(area / area.sum() * n_vertices).astype(int))
    counts[0] += n_vertices - counts.sum()
    xyz, tri, off = [], [], 0
    for (a, b, r), (h, rr), n in zip(_PARTS, lens, counts):
        c = 0.5 * (pt(a) + pt(b))
        F = _frame(pt(b) - pt(a))
        p, t = fibonacci_ellipsoid(int(n), (1.0, 1.0, 1.0), (0.0, 0.0, 0.0))
        p = p.T.astype(np.float64) * np.array([rr, h, rr])
        p = p @ F.T + c
        xyz.append(p)
        tri.append(t.T.astype(np.int64) + off)
        off += int(n)
    xyz = np.concatenate(xyz)
    tri = np.concatenate(tri)
    part = np.repeat(np.arange(len(_PARTS)), counts)
    # binding: 4 nearest bones (segment distance), a bone moves with its start joint
    bones = [(PARENTS[j], J[PARENTS[j]], J[j]) for j in range(1, len(JOINTS))]
    bones += [(j, J[j], _ENDS[j] + np.asarray(root)) for j in sorted(_ENDS)]
    d = np.zeros((xyz.shape[0], len(bones)))
    for k, (_, A, B) in enumerate(bones):
        ab = B - A
        s = np.clip(((xyz - A) @ ab) / (ab @ ab), 0.0, 1.0)
        d[:, k] = np.linalg.norm(xyz - (A + s[:, None] * ab), axis=1)
    order = np.argsort(d, axis=1, kind="stable")[:, :4]
    dk = np.take_along_axis(d, order, axis=1)
    w = np.exp(-dk * dk / (2 * 0.04 ** 2))
    w = np.where(w.sum(axis=1, keepdims=True) > 0, w, np.eye(4)[0])
    w /= w.sum(axis=1, keepdims=True)
    bind_joint = np.array([bones[k][0] for k in range(len(bones))])[order]
    return dict(xyz=np.ascontiguousarray(xyz.T.astype(np.float32)),
                tri=np.ascontiguousarray(tri.T.astype(np.int32)),
                joints=np.ascontiguousarray(J.T.astype(np.float64)),
                parents=PARENTS.copy(),
                bind_idx=np.ascontiguousarray(bind_joint.T.astype(np.int32)),
                bind_w=np.ascontiguousarray(w.T.astype(np.float32)),
                part=part.astype(np.int32),
                classes=PART_CLASS[part].astype(np.int32),
                parts=PART_GROUP[part].astype(np.int32))


def _rodrigues(w):
    th = np.linalg.norm(w)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K


def pose_mesh(body, pose):
    """Ground-truth posing used to render targets (input generation only):
    joint rotations compose down the tree, vertices follow by linear blending."""
    J = body["joints"].T
    par = body["parents"]
    dof = dof_joints()
    Rl = [np.eye(3) for _ in JOINTS]
    for i, j in enumerate(dof):
        Rl[j] = _rodrigues(pose[3 * i:3 * i + 3])
    RG = [None] * len(JOINTS)
    P = np.zeros_like(J)
    for j in range(len(JOINTS)):
        if par[j] < 0:
            RG[j] = Rl[j]
            P[j] = J[j] + pose[63:66]
        else:
            RG[j] = RG[par[j]] @ Rl[j]
            P[j] = P[par[j]] + RG[par[j]] @ (J[j] - J[par[j]])
    v = body["xyz"].T.astype(np.float64)
    out = np.zeros_like(v)
    for s in range(4):
        j = body["bind_idx"][s]
        w = body["bind_w"][s].astype(np.float64)[:, None]
        loc = v - J[j]
        rot = np.einsum("nab,nb->na", np.stack([RG[x] for x in j]), loc)
        out += w * (rot + P[j])
    return np.ascontiguousarray(out.T.astype(np.float32)), P


def make_pose_frame(n_vertices=5000, side=1080, seed=0, angle_sigma=0.15, px_sigma=3.0, m_sigma=0.02):
    """Body, camera, ground-truth pose, noisy 2D/3D detections and target silhouette."""
    rng = np.random.Generator(np.random.PCG64(seed))
    body = make_body(n_vertices)
    cam = Camera.square(side)
    gt = np.zeros(69)
    gt[:63] = rng.normal(0.0, angle_sigma, 63)
    gt[63:66] = rng.normal(0.0, 0.05, 3)
    posed, P = pose_mesh(body, gt)
    gt[66:69] = P[0]                      # t' maps root-relative detections to the camera frame
    u = cam.fx * P[:, 0] / P[:, 2] + cam.cx
    v = cam.fy * P[:, 1] / P[:, 2] + cam.cy
    p2d = np.stack([u, v], axis=1) + rng.normal(0.0, px_sigma, (len(JOINTS), 2))
    p3d = (P - P[0]) + rng.normal(0.0, m_sigma, (len(JOINTS), 3))
    rgb = np.full((3, body["xyz"].shape[1]), 0.5, np.float32)
    mask, _ = render_targets(posed, body["tri"], rgb, cam)
    return dict(body=body, cam=cam, gt_pose=gt, gt_joints=P, posed=posed, mask=mask,
                p2d=np.ascontiguousarray(p2d.T), p3d=np.ascontiguousarray(p3d.T),
                lam=np.ones(len(JOINTS)))
