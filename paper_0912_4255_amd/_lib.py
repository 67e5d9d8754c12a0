"""ctypes mirror of include/rsfstat.h and the loader of librsfstat.so.

Argument marshalling only: no arithmetic of the method happens here.  The
loader raises if the shared library is missing; there is no fallback path.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsfstat.so")

RSF_MAX_DET = 4
RSF_OK, RSF_EINVAL, RSF_EUNSUPPORTED, RSF_EWORKSPACE, RSF_EHIP = 0, -1, -2, -3, -4
RSF_MODE_PLAIN, RSF_MODE_BATCHED = 0, 1
RSF_ENTRY_RESAMPLE, RSF_ENTRY_FSTAT, RSF_ENTRY_POINT, RSF_ENTRY_BACKWARD, RSF_ENTRY_TOPK = 0, 1, 2, 3, 4
RSF_ENTRY_SEMICOHERENT = 5
RSF_FLAG_DEGENERATE, RSF_FLAG_WINDOW, RSF_FLAG_ORBIT = 1, 2, 4
RSF_ROWS_GENERAL, RSF_ROWS_GENERAL_WIDE, RSF_ROWS_FIXED, RSF_ROWS_RUNTIME = 0, 1, 2, 3

EXPORTS = [
    "rsf_plan_create", "rsf_plan_destroy", "rsf_plan_query", "rsf_plan_first_pass", "rsf_plan_set_batching", "rsf_plan_batching", "rsf_fft_factor",
    "rsf_plan_set_spin_order", "rsf_plan_set_binary",
    "rsf_workspace_size",
    "rsf_resample", "rsf_fstat", "rsf_fstat_topk", "rsf_fstat_semicoherent", "rsf_fstat_point",
    "rsf_fstat_backward", "rsf_fstat_backward_static",
    "rsf_get_flags", "rsf_last_error", "rsf_version", "rsf_profile_enable", "rsf_profile_read",
    "rsf_graph_create_fstat", "rsf_graph_create_topk", "rsf_graph_launch", "rsf_graph_destroy",
    "rsf_segments_workspace_size", "rsf_fstat_topk_segments", "rsf_graph_create_topk_segments",
    "rsf_sft_plan_create", "rsf_sft_plan_destroy", "rsf_sft_plan_query", "rsf_sft_workspace_size",
    "rsf_sft_heterodyne", "rsf_sft_profile_enable", "rsf_sft_profile_read",
    "rsf_hetdec_plan_create", "rsf_hetdec_plan_destroy", "rsf_hetdec", "rsf_hetdec_profile_enable",
    "rsf_hetdec_profile_read",
]


class Detector(C.Structure):
    _fields_ = [("lat", C.c_double), ("lon", C.c_double), ("gamma", C.c_double), ("sigma2", C.c_double)]


class Ephemeris(C.Structure):
    _fields_ = [("au_c", C.c_double), ("re_c", C.c_double), ("p_orb", C.c_double), ("p_sid", C.c_double),
                ("eps", C.c_double), ("lambda0", C.c_double), ("theta0", C.c_double)]


class PlanDesc(C.Structure):
    _fields_ = [("n_det", C.c_int32), ("nfft_policy", C.c_int32), ("kernel", C.c_int32),
                ("taps", C.c_int32), ("storage", C.c_int32), ("fft_l1", C.c_int32),
                ("n", C.c_int64), ("dt", C.c_double), ("t_start", C.c_double), ("f_het", C.c_double),
                ("f_lo", C.c_double), ("f_hi", C.c_double), ("eph", Ephemeris),
                ("det", Detector * RSF_MAX_DET)]


class Segment(C.Structure):
    _fields_ = [("x", C.c_void_p * RSF_MAX_DET), ("gaps", C.c_void_p * RSF_MAX_DET),
                ("n_gaps", C.c_int32 * RSF_MAX_DET)]


class Resampled(C.Structure):
    _fields_ = [("z", C.c_void_p), ("a", C.c_void_p), ("b", C.c_void_p), ("tm", C.c_void_p),
                ("mask", C.c_void_p), ("abc", C.c_void_p), ("u", C.c_void_p)]


class TopkEntry(C.Structure):
    _fields_ = [("twoF", C.c_float), ("sky", C.c_int32), ("fdot", C.c_int32), ("bin", C.c_int32)]


class SftDesc(C.Structure):
    _fields_ = [("n_sft", C.c_int64), ("sft_len", C.c_int64), ("dt_raw", C.c_double), ("k_lo", C.c_int64),
                ("n_bins", C.c_int64), ("t_start", C.c_double), ("f_het", C.c_double), ("band", C.c_double),
                ("n_out", C.c_int64), ("dk", C.c_int32), ("median_window", C.c_int32),
                ("band_taper", C.c_double), ("edge_taper_s", C.c_double)]


class HetdecDesc(C.Structure):
    _fields_ = [("n_raw", C.c_int64), ("dt_raw", C.c_double), ("f_het", C.c_double), ("D", C.c_int32),
                ("K", C.c_int32), ("beta", C.c_double), ("n_out", C.c_int64)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


_lib = None


def load(path=None):
    """Load librsfstat.so (built in-tree by paper_0912_4255_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("RSF_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"librsfstat.so not found at {path}: build it with "
                           "`python -m paper_0912_4255_amd.build` (no fallback path exists)")
    lib = C.CDLL(path)
    vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int, C.c_size_t
    lib.rsf_plan_create.argtypes = [C.POINTER(vp), C.POINTER(PlanDesc)]
    lib.rsf_plan_destroy.argtypes = [vp]
    lib.rsf_plan_query.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64),
                                   C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    lib.rsf_plan_first_pass.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.rsf_plan_set_batching.argtypes = [vp, i32, i32]
    lib.rsf_plan_set_spin_order.argtypes = [vp, i32]
    lib.rsf_plan_set_binary.argtypes = [vp, i32]
    lib.rsf_fft_factor.argtypes = [i64, i32, i32, C.POINTER(i32), C.POINTER(i32)]
    lib.rsf_plan_batching.argtypes = [vp, i64, i64, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.rsf_workspace_size.argtypes = [vp, i32, i64, i64, i32, C.POINTER(sz)]
    lib.rsf_resample.argtypes = [vp, C.POINTER(Segment), vp, i64, C.POINTER(Resampled), vp, sz, vp]
    lib.rsf_fstat.argtypes = [vp, C.POINTER(Segment), vp, i64, vp, i64, i32, vp, vp, sz, vp]
    lib.rsf_fstat_topk.argtypes = [vp, C.POINTER(Segment), vp, i64, vp, i64, i32, vp, vp, sz, vp]
    lib.rsf_fstat_semicoherent.argtypes = [vp, C.POINTER(Segment), vp, i64, vp, i64, C.c_double, C.c_double,
                                           C.c_double, i64, vp, vp, sz, vp]
    lib.rsf_fstat_point.argtypes = [vp, C.POINTER(Segment), vp, i64, vp, vp, sz, vp]
    lib.rsf_fstat_backward.argtypes = [vp, C.POINTER(Segment), vp, i64, vp, vp, vp, vp, sz, vp]
    lib.rsf_fstat_backward_static.argtypes = [vp, C.POINTER(Segment), vp, i64, vp, vp, vp, vp]
    lib.rsf_get_flags.argtypes = [vp, vp, C.POINTER(C.c_uint32), vp]
    lib.rsf_graph_create_fstat.argtypes = [C.POINTER(vp), vp, C.POINTER(Segment), vp, i64, vp, i64, vp, vp, sz]
    lib.rsf_graph_create_topk.argtypes = [C.POINTER(vp), vp, C.POINTER(Segment), vp, i64, vp, i64, i32, vp, vp,
                                          sz]
    lib.rsf_segments_workspace_size.argtypes = [C.POINTER(vp), i64, i64, i64, C.POINTER(sz)]
    lib.rsf_fstat_topk_segments.argtypes = [C.POINTER(vp), C.POINTER(Segment), i64, vp, i64, vp, i64, i32, vp, vp,
                                            sz, vp]
    lib.rsf_graph_create_topk_segments.argtypes = [C.POINTER(vp), C.POINTER(vp), C.POINTER(Segment), i64, vp, i64,
                                                   vp, i64, i32, vp, vp, sz]
    lib.rsf_graph_launch.argtypes = [vp, vp]
    lib.rsf_graph_destroy.argtypes = [vp]
    lib.rsf_profile_enable.argtypes = [vp, i32]
    lib.rsf_profile_read.argtypes = [vp, C.POINTER(KernelTime), i32, C.POINTER(C.c_int)]
    dp = C.POINTER(C.c_double)
    lib.rsf_sft_plan_create.argtypes = [C.POINTER(vp), C.POINTER(SftDesc), dp]
    lib.rsf_sft_plan_destroy.argtypes = [vp]
    lib.rsf_sft_plan_query.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), i64, C.POINTER(i64)]
    lib.rsf_sft_workspace_size.argtypes = [vp, C.POINTER(sz)]
    lib.rsf_sft_heterodyne.argtypes = [vp, vp, vp, vp, sz, vp]
    lib.rsf_sft_profile_enable.argtypes = [vp, i32]
    lib.rsf_sft_profile_read.argtypes = [vp, C.POINTER(KernelTime), i32, C.POINTER(C.c_int)]
    lib.rsf_hetdec_plan_create.argtypes = [C.POINTER(vp), C.POINTER(HetdecDesc)]
    lib.rsf_hetdec_plan_destroy.argtypes = [vp]
    lib.rsf_hetdec.argtypes = [vp, vp, vp, vp]
    lib.rsf_hetdec_profile_enable.argtypes = [vp, i32]
    lib.rsf_hetdec_profile_read.argtypes = [vp, C.POINTER(KernelTime), i32, C.POINTER(C.c_int)]
    lib.rsf_last_error.restype = C.c_char_p
    lib.rsf_last_error.argtypes = []
    lib.rsf_version.argtypes = []
    for name in EXPORTS:
        getattr(lib, name).restype = C.c_int if name != "rsf_last_error" else C.c_char_p
    _lib = lib
    return lib


class RsfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rsf error {code}: {msg}")
        self.code = code


def check(rc):
    if rc != RSF_OK:
        raise RsfError(rc, load().rsf_last_error().decode())
    return rc
