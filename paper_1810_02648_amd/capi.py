"""ctypes declarations of libcapture.so (mirrors include/capture.h)."""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcapture.so")

MAX_GN = 32
STATUS = {0: "CAPTURE_OK", -1: "CAPTURE_EINVAL", -2: "CAPTURE_ENOTSPD", -3: "CAPTURE_ENONFINITE",
          -4: "CAPTURE_EHIP", -5: "CAPTURE_ENOMEM", -6: "CAPTURE_EUNSUPPORTED"}


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class TemplateDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_triangles", C.c_int32), ("n_nodes", C.c_int32),
                ("tri", C.c_void_p), ("node_vertex", C.c_void_p), ("bind_idx", C.c_void_p),
                ("bind_w", C.c_void_p), ("edge_dst", C.c_void_p), ("vertices_per_tile", C.c_int32)]


class TemplateInfo(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_triangles", C.c_int32), ("n_nodes", C.c_int32),
                ("n_tiles", C.c_int32), ("n_slots", C.c_int32), ("max_slots", C.c_int32),
                ("max_contrib", C.c_int32), ("vertices_per_tile", C.c_int32)]


class Frame(C.Structure):
    _fields_ = [("tmpl", C.c_void_p), ("xyz", C.c_void_p), ("rgb", C.c_void_p), ("camera", Camera),
                ("mask", C.c_void_p), ("image", C.c_void_p), ("node_state", C.c_void_p)]


class NonrigidParams(C.Structure):
    _fields_ = [("w_sil", C.c_float), ("w_photo", C.c_float), ("w_arap", C.c_float),
                ("tau_color", C.c_float), ("w_vel", C.c_float), ("gn_iters", C.c_int32),
                ("pcg_iters", C.c_int32), ("flags", C.c_uint32), ("pcg_tol", C.c_float)]


FLAG_EXCLUDE_CASE2 = 1
FLAG_OUTLINE_ONLY = 2
FLAG_PCG_STANDARD = 4
FLAG_PART_MASK = 8
MAX_JOINTS = 32
MAX_POSE_UNKNOWNS = 81


class Report(C.Structure):
    _fields_ = [("energy", C.c_double * (MAX_GN + 1)), ("e_photo", C.c_double), ("e_sil", C.c_double),
                ("e_sil_abs", C.c_double), ("e_arap", C.c_double), ("e_vel", C.c_double),
                ("energy_prev", C.c_double),
                ("energy_pred", C.c_double), ("n_visible", C.c_int32), ("n_boundary", C.c_int32),
                ("gn_done", C.c_int32), ("warm_start", C.c_int32), ("status", C.c_int32)]


class BodyDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_triangles", C.c_int32), ("n_joints", C.c_int32),
                ("tri", C.c_void_p), ("xyz", C.c_void_p), ("bind_joint", C.c_void_p), ("bind_w", C.c_void_p),
                ("parents", C.c_void_p), ("rest_joints", C.c_void_p), ("has_rotation", C.c_void_p)]


class PoseFrame(C.Structure):
    _fields_ = [("body", C.c_void_p), ("camera", Camera), ("mask", C.c_void_p), ("p2d", C.c_void_p),
                ("p3d", C.c_void_p), ("lambda_", C.c_void_p), ("pose", C.c_void_p), ("prev_joints", C.c_void_p)]


class PoseParams(C.Structure):
    _fields_ = [("l2d", C.c_double), ("l3d", C.c_double), ("lsil", C.c_double), ("gn_iters", C.c_int32),
                ("flags", C.c_uint32), ("l_temporal", C.c_double * MAX_JOINTS), ("l_anatomic", C.c_double),
                ("theta_min", C.c_double * MAX_POSE_UNKNOWNS), ("theta_max", C.c_double * MAX_POSE_UNKNOWNS)]


class PoseReport(C.Structure):
    _fields_ = [("energy", C.c_double * (MAX_GN + 1)), ("e2d", C.c_double), ("e3d", C.c_double),
                ("e_sil", C.c_double), ("e_sil_abs", C.c_double), ("e_temporal", C.c_double),
                ("e_anatomic", C.c_double), ("n_visible", C.c_int32),
                ("n_boundary", C.c_int32), ("gn_done", C.c_int32), ("status", C.c_int32)]


VERTEX_MAX_RING = 32


class VertexTemplateDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_triangles", C.c_int32), ("tri", C.c_void_p), ("rest", C.c_void_p),
                ("classes", C.c_void_p), ("parts", C.c_void_p)]


class VertexFrame(C.Structure):
    _fields_ = [("tmpl", C.c_void_p), ("posed", C.c_void_p), ("prev", C.c_void_p), ("prev2", C.c_void_p),
                ("rgb", C.c_void_p), ("camera", Camera), ("mask", C.c_void_p), ("image", C.c_void_p),
                ("V", C.c_void_p)]


class VertexParams(C.Structure):
    _fields_ = [("w_photo", C.c_float), ("w_sil", C.c_float), ("w_smooth", C.c_float), ("w_edge", C.c_float),
                ("w_vel", C.c_float), ("w_acc", C.c_float), ("tau_color", C.c_float), ("gn_iters", C.c_int32),
                ("pcg_iters", C.c_int32), ("flags", C.c_uint32), ("blur_kernel", C.c_int32 * MAX_GN),
                ("snap_max_px", C.c_float), ("snap_steps", C.c_int32), ("snap_rings", C.c_int32),
                ("snap_iters", C.c_int32), ("part_dilation", C.c_int32)]


class VertexReport(C.Structure):
    _fields_ = [("energy", C.c_double * (MAX_GN + 1)), ("e_photo", C.c_double), ("e_sil", C.c_double),
                ("e_sil_abs", C.c_double), ("e_smooth", C.c_double), ("e_edge", C.c_double), ("e_vel", C.c_double),
                ("e_acc", C.c_double), ("n_visible", C.c_int32), ("n_boundary", C.c_int32), ("gn_done", C.c_int32),
                ("n_snapped", C.c_int32), ("status", C.c_int32)]


_P = C.c_void_p
SIGNATURES = {
    "capture_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "capture_destroy": (None, [_P]),
    "capture_last_error": (C.c_char_p, []),
    "capture_graph_build": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P]),
    "capture_template_create": (C.c_int, [_P, C.POINTER(TemplateDesc), C.POINTER(C.c_void_p)]),
    "capture_template_destroy": (None, [_P]),
    "capture_template_info_get": (C.c_int, [_P, C.POINTER(TemplateInfo)]),
    "capture_workspace_size": (C.c_int, [_P, C.c_int32, C.POINTER(Frame), C.POINTER(C.c_size_t)]),
    "capture_nonrigid_solve": (C.c_int, [_P, C.POINTER(Frame), C.POINTER(NonrigidParams), C.POINTER(Report),
                                         _P, C.c_size_t, _P]),
    "capture_nonrigid_solve_noalloc": (C.c_int, [_P, C.POINTER(Frame), C.POINTER(NonrigidParams),
                                                 C.POINTER(Report), _P]),
    "capture_batch_solve": (C.c_int, [_P, C.c_int32, C.POINTER(Frame), C.POINTER(NonrigidParams),
                                      C.POINTER(Report), _P, C.c_size_t, _P]),
    "capture_frame_decisions": (C.c_int, [_P, C.POINTER(Frame), _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "capture_linearize": (C.c_int, [_P, C.POINTER(Frame), C.POINTER(NonrigidParams), _P, _P, _P, _P,
                                    C.POINTER(C.c_double), _P, C.c_size_t, _P]),
    "capture_warmstart_create": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_void_p)]),
    "capture_warmstart_destroy": (None, [_P]),
    "capture_warmstart_set_scaling": (C.c_int, [_P, _P, _P]),
    "capture_warmstart_get_params": (C.c_int, [_P, _P, C.POINTER(C.c_int64)]),
    "capture_warmstart_fit_scaling": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "capture_warmstart_target": (C.c_int, [_P, C.c_int32, _P, _P, _P, _P]),
    "capture_warmstart_features": (C.c_int, [_P, C.POINTER(Frame), _P, C.POINTER(NonrigidParams), _P, _P,
                                             C.c_size_t, _P]),
    "capture_warmstart_forward": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "capture_warmstart_train_step": (C.c_int, [_P, _P, _P, _P, _P, C.c_float, C.c_int, _P,
                                               C.POINTER(C.c_double), _P]),
    "capture_nonrigid_solve_warm": (C.c_int, [_P, C.POINTER(Frame), C.POINTER(NonrigidParams), _P, _P,
                                              C.c_double, C.POINTER(Report), _P, C.c_size_t, _P]),
    "capture_body_create": (C.c_int, [_P, C.POINTER(BodyDesc), C.POINTER(C.c_void_p)]),
    "capture_body_destroy": (None, [_P]),
    "capture_body_unknowns": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "capture_pose_workspace_size": (C.c_int, [_P, C.POINTER(PoseFrame), C.POINTER(C.c_size_t)]),
    "capture_pose_solve": (C.c_int, [_P, C.POINTER(PoseFrame), C.POINTER(PoseParams), C.POINTER(PoseReport),
                                     _P, C.c_size_t, _P]),
    "capture_pose_linearize": (C.c_int, [_P, C.POINTER(PoseFrame), C.POINTER(PoseParams), _P,
                                         C.POINTER(C.c_double), _P, _P, C.c_size_t, _P]),
    "capture_autotune_tiles": (C.c_int, [_P, C.c_int32, C.POINTER(TemplateDesc), C.POINTER(Frame),
                                         C.POINTER(NonrigidParams), C.POINTER(C.c_int32), C.c_int32,
                                         C.POINTER(C.c_int32), C.POINTER(C.c_double), _P]),
    "capture_vertex_template_create": (C.c_int, [_P, C.POINTER(VertexTemplateDesc), C.POINTER(C.c_void_p)]),
    "capture_vertex_template_destroy": (None, [_P]),
    "capture_vertex_workspace_size": (C.c_int, [_P, C.POINTER(VertexFrame), C.POINTER(VertexParams),
                                                C.POINTER(C.c_size_t)]),
    "capture_vertex_solve": (C.c_int, [_P, C.POINTER(VertexFrame), C.POINTER(VertexParams),
                                       C.POINTER(VertexReport), _P, C.c_size_t, _P]),
    "capture_vertex_linearize": (C.c_int, [_P, C.POINTER(VertexFrame), C.POINTER(VertexParams), _P, _P, _P, _P,
                                           C.POINTER(C.c_double), _P, _P, C.c_size_t, _P]),
    "capture_body_skin": (C.c_int, [_P, _P, _P, _P, _P]),
    "capture_body_warp": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "capture_pose_extrapolate": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "capture_body_joints": (C.c_int, [_P, _P, _P, _P, _P]),
    "capture_set_graphs": (C.c_int, [_P, C.c_int]),
    "capture_profile_enable": (C.c_int, [_P, C.c_int]),
    "capture_profile_read": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
}

KERNELS = ("blur", "contour", "dt_cols", "dt_rows", "deform_start", "raster", "contour_edges", "decide",
           "linearize", "node_init", "cg", "cg_node", "ws_features", "ws_mlp", "pose_lbs", "pose_rows",
           "pose_jtj", "pose_step", "prep_image", "prep_geom", "prep_raster", "prep_cols", "v_blur", "v_lin",
           "v_apply", "v_update", "v_snap")
WS_PARAMS = 38662

_lib = None


def load():
    """Load libcapture.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcapture.so is not built (run __graft_entry__.build() or "
                              "python paper_1810_02648_amd/build.py): %s" % LIB_PATH)
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class CaptureError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


def check(code):
    if code != 0:
        msg = load().capture_last_error()
        raise CaptureError(code, msg.decode() if msg else "")
    return code
