"""ctypes binding of libprism (include/prism.h): argument marshalling only.

Loading fails loudly when the library has not been built; there is no
Python or CPU fallback for any compute entry point.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# PRISM_LIBRARY names another build of the same library (the host-sanitizer
# build used by the CPU tests); the default is the in-tree libprism.so.
LIB_PATH = os.environ.get("PRISM_LIBRARY") or os.path.join(_HERE, "libprism.so")

PRISM_OK = 0
PRISM_EINVAL = -1
PRISM_ENOSPACE = -2
PRISM_EHIP = -3
PRISM_ENOTREADY = -4
PRISM_MAX_DET = 32
PRISM_PREC_FP32 = 0
PRISM_PREC_BF16 = 1
PRISM_PREC_FP16 = 2
PRISM_NOALLOC_SCRATCH_BYTES = 256 << 20

EXPORTS = (
    "prism_plan_create", "prism_plan_destroy", "prism_wavelength", "prism_alpha_max",
    "prism_beam_count", "prism_beams", "prism_active_beam_count", "prism_smatrix_bytes", "prism_build_workspace_bytes",
    "prism_multislice_workspace_bytes", "prism_probe_workspace_bytes", "prism_probe_group",
    "prism_probe_order",
    "prism_set_probe_precision", "prism_set_potential_slices", "prism_build_smatrix",
    "prism_probe_outputs", "prism_probe_outputs_noalloc", "prism_probe_cbed",
    "prism_multislice_outputs",
    "prism_probe_outputs_accumulate", "prism_probe_cbed_accumulate",
    "prism_probe_batch_workspace_bytes", "prism_probe_batch", "prism_probe_class",
    "prism_multislice_outputs_accumulate", "prism_build_batch_workspace_bytes",
    "prism_build_smatrix_batch", "prism_server_workspace_bytes", "prism_server_create",
    "prism_server_destroy", "prism_server_admit", "prism_server_submit_build",
    "prism_server_set_lru_eviction", "prism_server_set_dispatch_limit", "prism_server_evictions", "prism_server_evict",
    "prism_server_submit",
    "prism_server_flush", "prism_server_poll", "prism_server_wait", "prism_server_stats",
    "prism_server_call_stats",
    "prism_set_tuning", "prism_get_tuning", "prism_profile_enable", "prism_profile_report",
    "prism_last_error",
)


class PrismGeometry(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("cell_A", ctypes.c_double), ("energy_keV", ctypes.c_double),
                ("n_slices", ctypes.c_int), ("slice_thickness_A", ctypes.POINTER(ctypes.c_double))]


class PrismOptics(ctypes.Structure):
    _fields_ = [("alpha_mrad", ctypes.c_double), ("C1_A", ctypes.c_double),
                ("C3_A", ctypes.c_double), ("tilt_x_mrad", ctypes.c_double),
                ("tilt_y_mrad", ctypes.c_double)]


class PrismDetector(ctypes.Structure):
    _fields_ = [("n_det", ctypes.c_int), ("edges_mrad", ctypes.POINTER(ctypes.c_double))]


class PrismBuildItem(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("f", ctypes.c_int),
                ("alpha_max_mrad", ctypes.c_double), ("smatrix_dev", ctypes.c_void_p),
                ("smatrix_bytes", ctypes.c_size_t)]


class PrismProbeRequest(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("f", ctypes.c_int),
                ("alpha_max_mrad", ctypes.c_double), ("smatrix_dev", ctypes.c_void_p),
                ("smatrix_bytes", ctypes.c_size_t), ("probe_xy_dev", ctypes.c_void_p),
                ("n_probes", ctypes.c_int), ("optics", ctypes.POINTER(PrismOptics)),
                ("detector", ctypes.POINTER(PrismDetector)), ("out_dev", ctypes.c_void_p),
                ("cbed_dev", ctypes.c_void_p), ("accumulate", ctypes.c_int),
                ("weight", ctypes.c_double)]


class PrismTuning(ctypes.Structure):
    _fields_ = [("row_iters", ctypes.c_int), ("row_min_groups", ctypes.c_int),
                ("col_iters", ctypes.c_int), ("col_min_groups", ctypes.c_int),
                ("wave_chunk_mib", ctypes.c_int), ("probe_group", ctypes.c_int),
                ("window_tile_div", ctypes.c_int)]


class PrismError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libprism status {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libprism.so once; raises ImportError if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run `python -m paper_1702_01904_amd.build`")
    # torch ships its own HIP runtime with the same soname (libamdhip64.so.7).
    # Importing torch first makes libprism bind to that already-loaded copy,
    # so the process holds one HIP/HSA runtime and shares torch's device
    # memory and streams.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    SZ = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "prism_plan_create": (I, [ctypes.POINTER(P), ctypes.POINTER(PrismGeometry)]),
        "prism_plan_destroy": (None, [P]),
        "prism_wavelength": (I, [P, ctypes.POINTER(D)]),
        "prism_alpha_max": (I, [P, I, D, ctypes.POINTER(D)]),
        "prism_beam_count": (I, [P, I, D, ctypes.POINTER(I)]),
        "prism_active_beam_count": (I, [P, I, D, ctypes.POINTER(PrismOptics), ctypes.POINTER(I)]),
        "prism_beams": (I, [P, I, D, ctypes.POINTER(ctypes.c_int32), I]),
        "prism_smatrix_bytes": (I, [P, I, D, SZ]),
        "prism_build_workspace_bytes": (I, [P, I, D, SZ, SZ]),
        "prism_multislice_workspace_bytes": (I, [P, I, SZ, SZ]),
        "prism_probe_workspace_bytes": (I, [P, I, D, ctypes.POINTER(PrismOptics), SZ, SZ]),
        "prism_probe_group": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "prism_probe_order": (I, [P, I, P, I, P]),
        "prism_set_probe_precision": (I, [P, I]),
        "prism_set_potential_slices": (I, [P, P]),
        "prism_build_smatrix": (I, [P, I, D, P, ctypes.c_size_t, P, ctypes.c_size_t, P]),
        "prism_probe_outputs": (I, [P, I, D, P, ctypes.c_size_t, P, I,
                                    ctypes.POINTER(PrismOptics), ctypes.POINTER(PrismDetector), P,
                                    P, ctypes.c_size_t, P]),
        "prism_probe_outputs_noalloc": (I, [P, I, D, P, ctypes.c_size_t, P, I,
                                            ctypes.POINTER(PrismOptics),
                                            ctypes.POINTER(PrismDetector), P, P]),
        "prism_probe_cbed": (I, [P, I, D, P, ctypes.c_size_t, P, I, ctypes.POINTER(PrismOptics),
                                 P, P, ctypes.c_size_t, P]),
        "prism_multislice_outputs": (I, [P, P, I, ctypes.POINTER(PrismOptics),
                                         ctypes.POINTER(PrismDetector), P, P, ctypes.c_size_t, P]),
        "prism_probe_outputs_accumulate": (I, [P, I, D, P, ctypes.c_size_t, P, I,
                                               ctypes.POINTER(PrismOptics),
                                               ctypes.POINTER(PrismDetector), D, P, P,
                                               ctypes.c_size_t, P]),
        "prism_probe_cbed_accumulate": (I, [P, I, D, P, ctypes.c_size_t, P, I,
                                            ctypes.POINTER(PrismOptics), D, P, P,
                                            ctypes.c_size_t, P]),
        "prism_multislice_outputs_accumulate": (I, [P, P, I, ctypes.POINTER(PrismOptics),
                                                    ctypes.POINTER(PrismDetector), D, P, P,
                                                    ctypes.c_size_t, P]),
        "prism_probe_batch_workspace_bytes": (I, [ctypes.POINTER(PrismProbeRequest), I, SZ, SZ]),
        "prism_probe_batch": (I, [ctypes.POINTER(PrismProbeRequest), I, P, ctypes.c_size_t, P]),
        "prism_probe_class": (I, [P, I, ctypes.POINTER(ctypes.c_ulonglong)]),
        "prism_build_batch_workspace_bytes": (I, [ctypes.POINTER(PrismBuildItem), I, SZ, SZ]),
        "prism_build_smatrix_batch": (I, [ctypes.POINTER(PrismBuildItem), I, P, ctypes.c_size_t,
                                          P]),
        "prism_server_workspace_bytes": (I, [I, I, I, ctypes.c_size_t, SZ]),
        "prism_server_create": (I, [ctypes.POINTER(P), ctypes.c_size_t, I, I, I, P,
                                    ctypes.c_size_t]),
        "prism_server_destroy": (None, [P]),
        "prism_server_admit": (I, [P, P, I, D, P, ctypes.c_size_t, P, ctypes.c_size_t,
                                   ctypes.POINTER(I)]),
        "prism_server_submit_build": (I, [P, P, I, D, P, ctypes.c_size_t, P, ctypes.c_size_t,
                                          ctypes.POINTER(I), ctypes.POINTER(ctypes.c_longlong)]),
        "prism_server_set_lru_eviction": (I, [P, I]),
        "prism_server_set_dispatch_limit": (I, [P, I]),
        "prism_server_evictions": (I, [P, ctypes.POINTER(I), I, ctypes.POINTER(I)]),
        "prism_server_evict": (I, [P, I]),
        "prism_server_submit": (I, [P, I, P, I, ctypes.POINTER(PrismOptics),
                                    ctypes.POINTER(PrismDetector), P,
                                    ctypes.POINTER(ctypes.c_longlong)]),
        "prism_server_flush": (I, [P]),
        "prism_server_poll": (I, [P, ctypes.POINTER(ctypes.c_longlong), I, ctypes.POINTER(I)]),
        "prism_server_wait": (I, [P, ctypes.c_longlong]),
        "prism_server_stats": (I, [P, SZ, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "prism_server_call_stats": (I, [P, ctypes.POINTER(ctypes.c_longlong),
                                        ctypes.POINTER(ctypes.c_longlong)]),
        "prism_set_tuning": (I, [P, ctypes.POINTER(PrismTuning)]),
        "prism_get_tuning": (I, [P, ctypes.POINTER(PrismTuning)]),
        "prism_profile_enable": (I, [P, I]),
        "prism_profile_report": (I, [P, ctypes.c_char_p, ctypes.c_size_t]),
        "prism_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(code):
    if code != PRISM_OK:
        msg = lib().prism_last_error().decode(errors="replace")
        raise PrismError(code, msg)
    return code
