"""Deformation-graph construction (oracle).

The paper optimises vertex positions directly and names the embedded
deformation graph only as the alternative it chose not to use (Sec. 6); the
graph here follows the standard embedded-deformation construction, with every
choice the text leaves open fixed as follows:

* nodes: Euclidean farthest-point sampling over the vertices, seeded at
  vertex 0; ties in the argmax go to the lowest vertex index;
* binding: each vertex binds to its 4 nearest nodes (ties -> lower node
  index), weights w_ik proportional to exp(-d_ik^2 / (2 sigma_i^2)) with
  sigma_i the distance to the 4th-nearest node, normalised to sum to one
  (uniform weights if sigma_i is 0);
* edges: each node links to its 8 nearest other nodes (ties -> lower index),
  directed, padded with -1 when fewer than 8 other nodes exist.

Squared distances that decide indices use one float32 recipe,
``((dx*dx) + (dy*dy)) + (dz*dz)`` with ``d = a - b`` rounded per step, so that
the selected indices can be compared bit for bit.
"""
import numpy as np

F32 = np.float32


def _d2_f32(ax, ay, az, bx, by, bz):
    dx = (ax - bx).astype(F32)
    dy = (ay - by).astype(F32)
    dz = (az - bz).astype(F32)
    return ((dx * dx) + (dy * dy)) + (dz * dz)


def farthest_point_sampling(xyz, n_nodes):
    """Indices of ``n_nodes`` vertices chosen by farthest-point sampling."""
    x, y, z = (xyz[0].astype(F32), xyz[1].astype(F32), xyz[2].astype(F32))
    nv = x.size
    if not 1 <= n_nodes <= nv:
        raise ValueError("n_nodes must be in [1, n_vertices]")
    sel = np.zeros(n_nodes, dtype=np.int32)
    mind = _d2_f32(x, y, z, x[0], y[0], z[0])
    for n in range(1, n_nodes):
        s = int(np.argmax(mind))          # first maximum = lowest index
        sel[n] = s
        mind = np.minimum(mind, _d2_f32(x, y, z, x[s], y[s], z[s]))
    return sel


def bind_vertices(xyz, node_vertex, k=4, chunk=4096):
    """4-nearest-node binding: (bind_idx int32 [k][nv], bind_w float64 [k][nv])."""
    x, y, z = (xyz[0].astype(F32), xyz[1].astype(F32), xyz[2].astype(F32))
    gx, gy, gz = x[node_vertex], y[node_vertex], z[node_vertex]
    nv, nn = x.size, node_vertex.size
    if nn < k:
        raise ValueError("need at least k nodes")
    idx = np.zeros((k, nv), dtype=np.int32)
    w = np.zeros((k, nv), dtype=np.float64)
    for s in range(0, nv, chunk):
        e = min(nv, s + chunk)
        d2 = _d2_f32(x[s:e, None], y[s:e, None], z[s:e, None], gx[None, :], gy[None, :], gz[None, :])
        order = np.argsort(d2, axis=1, kind="stable")[:, :k]   # stable: ties keep lower index first
        dk = np.take_along_axis(d2, order, axis=1).astype(np.float64)
        sig2 = dk[:, k - 1:k]
        with np.errstate(divide="ignore", invalid="ignore"):
            ww = np.where(sig2 > 0, np.exp(-dk / (2.0 * sig2)), 1.0)
        ww /= ww.sum(axis=1, keepdims=True)
        idx[:, s:e] = order.T
        w[:, s:e] = ww.T
    return idx, w


def node_edges(xyz, node_vertex, k=8):
    """Directed node graph: edge_dst int32 [k][nn], -1 where absent."""
    x, y, z = (xyz[0].astype(F32), xyz[1].astype(F32), xyz[2].astype(F32))
    gx, gy, gz = x[node_vertex], y[node_vertex], z[node_vertex]
    nn = node_vertex.size
    d2 = _d2_f32(gx[:, None], gy[:, None], gz[:, None], gx[None, :], gy[None, :], gz[None, :])
    d2[np.arange(nn), np.arange(nn)] = np.inf          # exclude self
    order = np.argsort(d2, axis=1, kind="stable")
    out = np.full((k, nn), -1, dtype=np.int32)
    m = min(k, nn - 1)
    out[:m, :] = order[:, :m].T
    return out


def build_graph(xyz, n_nodes):
    """Full graph: node_vertex, bind_idx, bind_w (float32), edge_dst."""
    nodes = farthest_point_sampling(xyz, n_nodes)
    bidx, bw = bind_vertices(xyz, nodes)
    edges = node_edges(xyz, nodes)
    return dict(node_vertex=nodes, bind_idx=bidx, bind_w=bw.astype(F32), bind_w64=bw,
                edge_dst=edges)
