"""Helpers for the GPU tests: move seeded inputs to the device and call the library."""
import numpy as np
import torch

import paper_1810_02648_amd as cap


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def device_graph(g):
    return dict(node_vertex=dev(g["node_vertex"].astype(np.int32)), bind_idx=dev(g["bind_idx"].astype(np.int32)),
                bind_w=dev(g["bind_w"].astype(np.float32)), edge_dst=dev(g["edge_dst"].astype(np.int32)))


def identity_state(nn):
    s = np.zeros((12, nn), np.float32)
    s[0] = s[4] = s[8] = 1.0
    return s


def make_frame(ctx, f, graph, state=None, tmpl=None, vertices_per_tile=0):
    """FrameInputs for a synthetic frame dict and a host graph dict."""
    if tmpl is None:
        tmpl = cap.Template(ctx, dev(f["tri"]), device_graph(graph), vertices_per_tile)
    nn = graph["node_vertex"].size
    st = identity_state(nn) if state is None else state.astype(np.float32)
    return cap.FrameInputs(tmpl, dev(f["xyz"]), dev(f["rgb"]), f["cam"], dev(f["mask"]), dev(f["image"]),
                           dev(st))
