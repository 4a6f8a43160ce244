"""CPU checks of the C ABI: the library loads and exports every declared entry point."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            names |= set(re.findall(r"CAPTURE_API\s+[\w\s\*]*?\b(capture_\w+)\s*\(", text))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("capture_nonrigid_solve", "capture_batch_solve", "capture_graph_build",
                     "capture_workspace_size", "capture_template_create", "capture_last_error",
                     "capture_pose_solve", "capture_body_create", "capture_vertex_solve",
                     "capture_vertex_template_create", "capture_body_warp", "capture_body_skin"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1810_02648_amd import capi
    if not os.path.exists(capi.LIB_PATH):
        pytest.skip("library not built")
    lib = capi.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(capi.SIGNATURES) == declared_functions()


def test_struct_layouts_match_header():
    """ctypes mirrors of the header structs have the C sizes (checked with the host compiler)."""
    import ctypes
    import subprocess
    import tempfile
    from paper_1810_02648_amd import capi
    src = r"""
#include <stdio.h>
#include "capture.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(capture_camera),
         sizeof(capture_template_desc), sizeof(capture_frame), sizeof(capture_nonrigid_params), sizeof(capture_report),
         sizeof(capture_body_desc), sizeof(capture_pose_frame), sizeof(capture_pose_params),
         sizeof(capture_pose_report), sizeof(capture_template_info), sizeof(capture_vertex_template_desc),
         sizeof(capture_vertex_frame), sizeof(capture_vertex_params), sizeof(capture_vertex_report));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        sizes = [int(x) for x in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert sizes == [ctypes.sizeof(capi.Camera), ctypes.sizeof(capi.TemplateDesc), ctypes.sizeof(capi.Frame),
                     ctypes.sizeof(capi.NonrigidParams), ctypes.sizeof(capi.Report), ctypes.sizeof(capi.BodyDesc),
                     ctypes.sizeof(capi.PoseFrame), ctypes.sizeof(capi.PoseParams), ctypes.sizeof(capi.PoseReport),
                     ctypes.sizeof(capi.TemplateInfo), ctypes.sizeof(capi.VertexTemplateDesc),
                     ctypes.sizeof(capi.VertexFrame), ctypes.sizeof(capi.VertexParams),
                     ctypes.sizeof(capi.VertexReport)]
