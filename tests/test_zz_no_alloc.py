"""The allocation-free solve (capture_nonrigid_solve_noalloc) against the
workspace solve (capture_nonrigid_solve) through the C ABI: two calls in a row
on one device, the second with a smaller frame, each bitwise equal to the
workspace solve of the same frame; a frame beyond the scratch is refused
before any launch."""
import numpy as np
import pytest

import synth
from oracle import graph as og

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _solve_both(ctx, f, nn, prm):
    import paper_1810_02648_amd as cap
    from gpu_util import make_frame
    g = og.build_graph(f["xyz"], nn)
    a = make_frame(ctx, f, g)
    b = make_frame(ctx, f, g, tmpl=a.template)
    ref = cap.nonrigid_solve(ctx, a, prm)
    got = cap.nonrigid_solve_noalloc(ctx, b, prm)
    torch.cuda.synchronize()
    return a, b, ref, got


def test_noalloc_solve_equals_workspace_solve():
    import paper_1810_02648_amd as cap
    ctx = cap.Context(0)
    cases = [("mid", synth.make_nonrigid_frame("small", 2, n_vertices=9001, n_nodes=203, side=517), 203),
             ("small0", synth.make_nonrigid_frame("small", 0), 64)]
    for name, f, nn in cases:          # the second call has the smaller frame
        print("noalloc case", name, flush=True)
        prm = cap.params(*f["weights"], gn_iters=3, pcg_iters=8)
        a, b, ref, got = _solve_both(ctx, f, nn, prm)
        assert got["status"] == 0 and ref["status"] == 0
        assert np.array_equal(a.node_state.cpu().numpy().view(np.uint32), b.node_state.cpu().numpy().view(np.uint32))
        assert got["energy"] == ref["energy"]
        assert (got["n_visible"], got["n_boundary"], got["gn_done"]) == (ref["n_visible"], ref["n_boundary"],
                                                                         ref["gn_done"])


def test_noalloc_refuses_a_frame_beyond_its_scratch():
    import paper_1810_02648_amd as cap
    from gpu_util import dev, make_frame
    ctx = cap.Context(0)
    f = synth.make_nonrigid_frame("small", 0)
    g = og.build_graph(f["xyz"], 64)
    fr = make_frame(ctx, f, g)
    big = synth.Camera.square(2048)          # 2048^2 image: ~100 MiB of workspace
    fr_big = cap.FrameInputs(fr.template, fr.xyz, fr.rgb, big, dev(np.zeros((2048, 2048), np.uint8)),
                             dev(np.zeros((3, 2048, 2048), np.float32)), fr.node_state)
    before = fr.node_state.cpu().numpy().copy()
    with pytest.raises(cap.CaptureError) as e:
        cap.nonrigid_solve_noalloc(ctx, fr_big, cap.params(gn_iters=1, pcg_iters=1))
    assert e.value.code == -6
    assert np.array_equal(fr.node_state.cpu().numpy(), before)
