"""MI355X PRISM / multislice STEM simulation (Ophus, arXiv:1702.01904).

Thin Python layer over libprism (C ABI in include/prism.h). PyTorch is used
only to own device memory and streams; every step of the simulation runs
in the library's HIP kernels. Tensors passed in must already live on the
GPU with the stated dtype and shape; nothing is copied implicitly.
"""
import ctypes

import numpy as np

from . import _native
from ._native import PrismError, PrismOptics, PrismDetector, PrismGeometry  # noqa: F401

__all__ = ["Plan", "PrismError", "Server", "build_batch_workspace_bytes", "build_smatrix_batch",
           "probe_batch", "probe_batch_workspace_bytes", "tile_order", "untile"]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _nbytes(t):
    return ctypes.c_size_t(t.numel() * t.element_size())


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _optics(optics):
    """dict(alpha_mrad, C1_A=0, C3_A=0, tilt_x_mrad=0, tilt_y_mrad=0) -> prism_optics."""
    return PrismOptics(float(optics["alpha_mrad"]), float(optics.get("C1_A", 0.0)),
                       float(optics.get("C3_A", 0.0)), float(optics.get("tilt_x_mrad", 0.0)),
                       float(optics.get("tilt_y_mrad", 0.0)))


class _Det:
    """Keeps the edges array alive while the C struct points at it."""

    def __init__(self, edges_mrad):
        self.edges = np.ascontiguousarray(np.asarray(edges_mrad, dtype=np.float64).reshape(-1, 2))
        self.struct = PrismDetector(self.edges.shape[0],
                                    self.edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))


def _check_dev(t, dtype, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")


_TUNING_FIELDS = ("row_iters", "row_min_groups", "col_iters", "col_min_groups",
                  "wave_chunk_mib", "probe_group", "window_tile_div")
_TUNING = None


def _tuning_table():
    """Per-grid launch shapes from the committed sweep (tuning_gfx950.json), or {}."""
    global _TUNING
    if _TUNING is None:
        import json
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")
        _TUNING = {}
        if os.path.exists(path):
            with open(path) as fh:
                _TUNING = {k: v["tuning"] for k, v in json.load(fh).get("grids", {}).items()}
    return _TUNING


class Plan:
    """One grid / cell / energy / slicing (prism_plan). A plan for a grid in
    the committed tuning table gets that grid's launch shapes."""

    def __init__(self, n, cell_A, energy_keV, slice_thickness_A):
        self._L = _native.lib()
        th = np.ascontiguousarray(np.asarray(slice_thickness_A, dtype=np.float64))
        g = PrismGeometry(int(n), float(cell_A), float(energy_keV), int(th.size),
                          th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        h = ctypes.c_void_p()
        _native.check(self._L.prism_plan_create(ctypes.byref(h), ctypes.byref(g)))
        self._h = h
        self.n = int(n)
        self.cell = float(cell_A)
        self.energy_keV = float(energy_keV)
        self.n_slices = int(th.size)
        self._phase = None
        tuned = _tuning_table().get(str(self.n))
        if tuned:
            self.set_tuning(tuned)

    def close(self):
        if getattr(self, "_h", None):
            self._L.prism_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ host queries
    @property
    def wavelength(self):
        v = ctypes.c_double()
        _native.check(self._L.prism_wavelength(self._h, ctypes.byref(v)))
        return v.value

    def alpha_max_default(self, alpha_mrad, f):
        """The paper's beam-set limit for probe semi-angle alpha (prism_alpha_max), mrad."""
        v = ctypes.c_double()
        _native.check(self._L.prism_alpha_max(self._h, int(f), float(alpha_mrad), ctypes.byref(v)))
        return v.value

    def active_beam_count(self, f, alpha_max_mrad, optics):
        """B_A: beams of the set inside the probe aperture (prism_active_beam_count)."""
        v = ctypes.c_int()
        o = _optics(optics)
        _native.check(self._L.prism_active_beam_count(self._h, int(f), float(alpha_max_mrad),
                                                      ctypes.byref(o), ctypes.byref(v)))
        return v.value

    def beam_count(self, f, alpha_max_mrad):
        v = ctypes.c_int()
        _native.check(self._L.prism_beam_count(self._h, int(f), float(alpha_max_mrad),
                                               ctypes.byref(v)))
        return v.value

    def beams(self, f, alpha_max_mrad):
        B = self.beam_count(f, alpha_max_mrad)
        out = np.zeros((B, 2), dtype=np.int32)
        _native.check(self._L.prism_beams(self._h, int(f), float(alpha_max_mrad),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), B))
        return out

    def smatrix_bytes(self, f, alpha_max_mrad):
        v = ctypes.c_size_t()
        _native.check(self._L.prism_smatrix_bytes(self._h, int(f), float(alpha_max_mrad),
                                                  ctypes.byref(v)))
        return v.value

    def build_workspace_bytes(self, f, alpha_max_mrad):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _native.check(self._L.prism_build_workspace_bytes(self._h, int(f), float(alpha_max_mrad),
                                                          ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def multislice_workspace_bytes(self, n_det):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        _native.check(self._L.prism_multislice_workspace_bytes(self._h, int(n_det),
                                                               ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def probe_workspace_bytes(self, f, alpha_max_mrad, optics):
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        o = _optics(optics)
        _native.check(self._L.prism_probe_workspace_bytes(self._h, int(f), float(alpha_max_mrad),
                                                          ctypes.byref(o), ctypes.byref(a),
                                                          ctypes.byref(b)))
        return a.value, b.value

    def set_tuning(self, tuning):
        """Launch shapes (prism_set_tuning): dict of prism_tuning fields, absent or 0 = default."""
        t = _native.PrismTuning(*[int(tuning.get(k, 0)) for k in _TUNING_FIELDS])
        _native.check(self._L.prism_set_tuning(self._h, ctypes.byref(t)))

    def tuning(self):
        """The plan's effective launch shapes as a dict (prism_get_tuning)."""
        t = _native.PrismTuning()
        _native.check(self._L.prism_get_tuning(self._h, ctypes.byref(t)))
        return {k: getattr(t, k) for k in _TUNING_FIELDS}

    def probe_group(self, f):
        g, tx, ty = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _native.check(self._L.prism_probe_group(self._h, int(f), ctypes.byref(g), ctypes.byref(tx),
                                                ctypes.byref(ty)))
        return g.value, tx.value, ty.value

    def probe_class(self, f):
        """Launch-class key of the probe step (prism_probe_class)."""
        k = ctypes.c_ulonglong()
        _native.check(self._L.prism_probe_class(self._h, int(f), ctypes.byref(k)))
        return k.value

    # ------------------------------------------------------------ kernel timing
    def probe_order(self, f, probes):
        """Permutation (int64) visiting host probe positions [P][2] in compact runs."""
        xy = np.ascontiguousarray(np.asarray(probes, dtype=np.float64).reshape(-1, 2))
        perm = np.empty(xy.shape[0], dtype=np.int32)
        _native.check(self._L.prism_probe_order(
            self._h, int(f), xy.ctypes.data_as(ctypes.c_void_p), int(xy.shape[0]),
            perm.ctypes.data_as(ctypes.c_void_p)))
        return perm.astype(np.int64)

    def profile(self, enable=True):
        """Bracket every kernel launch of this plan with HIP events on its stream."""
        _native.check(self._L.prism_profile_enable(self._h, 1 if enable else 0))

    def profile_report(self):
        """{kernel: dict(launches, total_ms, min_ms, max_ms)}; waits for the events, clears them."""
        buf = ctypes.create_string_buffer(1 << 16)
        _native.check(self._L.prism_profile_report(self._h, buf, len(buf)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, cnt, tot, mn, mx = line.split()
            out[name] = dict(launches=int(cnt), total_ms=float(tot), min_ms=float(mn),
                             max_ms=float(mx))
        return out

    PRECISIONS = {"fp32": _native.PRISM_PREC_FP32, "bf16": _native.PRISM_PREC_BF16,
                  "fp16": _native.PRISM_PREC_FP16}

    def set_probe_precision(self, precision):
        """Operand precision of the probe-step window sum: "fp32", "bf16" or "fp16"."""
        if precision not in self.PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(self.PRECISIONS)}")
        _native.check(self._L.prism_set_probe_precision(self._h, self.PRECISIONS[precision]))

    # ------------------------------------------------------------ device calls
    def set_potential_slices(self, phase):
        """phase: float32 device tensor [H][n][n] (radians); borrowed, kept referenced."""
        import torch
        _check_dev(phase, torch.float32, self.n_slices * self.n * self.n, "phase")
        _native.check(self._L.prism_set_potential_slices(self._h, _ptr(phase)))
        self._phase = phase

    def build_smatrix(self, f, alpha_max_mrad, smatrix, workspace, stream=None):
        """smatrix: complex64 device tensor [B][n/2][n/2]; workspace: uint8 device tensor."""
        import torch
        B = self.beam_count(f, alpha_max_mrad)
        _check_dev(smatrix, torch.complex64, B * (self.n // 2) ** 2, "smatrix")
        _check_dev(workspace, torch.uint8, None, "workspace")
        _native.check(self._L.prism_build_smatrix(self._h, int(f), float(alpha_max_mrad),
                                                  _ptr(smatrix), _nbytes(smatrix), _ptr(workspace),
                                                  workspace.numel(), _stream_ptr(stream)))

    def probe_outputs(self, f, alpha_max_mrad, smatrix, probe_xy, optics, edges_mrad, out,
                      workspace, stream=None):
        """probe_xy: float64 device [P][2] (A); out: float64 device [P][n_det]."""
        self._probe_outputs(None, f, alpha_max_mrad, smatrix, probe_xy, optics, edges_mrad, out,
                            workspace, stream)

    def probe_outputs_noalloc(self, f, alpha_max_mrad, smatrix, probe_xy, optics, edges_mrad,
                              out, stream=None):
        """probe_outputs without a workspace: the library-held scratch of
        prism_probe_outputs_noalloc (calls overlapping on one GPU race)."""
        import torch
        det = _Det(edges_mrad)
        P = probe_xy.shape[0]
        _check_dev(probe_xy, torch.float64, 2 * P, "probe_xy")
        _check_dev(out, torch.float64, P * det.edges.shape[0], "out")
        _check_dev(smatrix, torch.complex64, None, "smatrix")
        o = _optics(optics)
        _native.check(self._L.prism_probe_outputs_noalloc(
            self._h, int(f), float(alpha_max_mrad), _ptr(smatrix), _nbytes(smatrix),
            _ptr(probe_xy), int(P), ctypes.byref(o), ctypes.byref(det.struct), _ptr(out),
            _stream_ptr(stream)))

    def probe_outputs_accumulate(self, f, alpha_max_mrad, smatrix, probe_xy, optics, edges_mrad,
                                 weight, out, workspace, stream=None):
        """As probe_outputs, but out += weight * result (frozen-phonon averaging)."""
        self._probe_outputs(float(weight), f, alpha_max_mrad, smatrix, probe_xy, optics,
                            edges_mrad, out, workspace, stream)

    def _probe_outputs(self, weight, f, alpha_max_mrad, smatrix, probe_xy, optics, edges_mrad,
                       out, workspace, stream):
        import torch
        det = _Det(edges_mrad)
        P = probe_xy.shape[0]
        _check_dev(probe_xy, torch.float64, 2 * P, "probe_xy")
        _check_dev(out, torch.float64, P * det.edges.shape[0], "out")
        _check_dev(smatrix, torch.complex64, None, "smatrix")
        _check_dev(workspace, torch.uint8, None, "workspace")
        o = _optics(optics)
        head = (self._h, int(f), float(alpha_max_mrad), _ptr(smatrix), _nbytes(smatrix),
                _ptr(probe_xy), int(P), ctypes.byref(o), ctypes.byref(det.struct))
        tail = (_ptr(out), _ptr(workspace), workspace.numel(), _stream_ptr(stream))
        if weight is None:
            _native.check(self._L.prism_probe_outputs(*head, *tail))
        else:
            _native.check(self._L.prism_probe_outputs_accumulate(*head, weight, *tail))

    def probe_cbed(self, f, alpha_max_mrad, smatrix, probe_xy, optics, out, workspace, stream=None):
        """Full diffraction patterns: out float32 device [P][W][W] (W = n / 2f, fftfreq order)."""
        self._probe_cbed(None, f, alpha_max_mrad, smatrix, probe_xy, optics, out, workspace, stream)

    def probe_cbed_accumulate(self, f, alpha_max_mrad, smatrix, probe_xy, optics, weight, out,
                              workspace, stream=None):
        """As probe_cbed, but out += weight * pattern (frozen-phonon averaging)."""
        self._probe_cbed(float(weight), f, alpha_max_mrad, smatrix, probe_xy, optics, out,
                         workspace, stream)

    def _probe_cbed(self, weight, f, alpha_max_mrad, smatrix, probe_xy, optics, out, workspace,
                    stream):
        import torch
        P = probe_xy.shape[0]
        w = self.n // (2 * int(f))
        _check_dev(probe_xy, torch.float64, 2 * P, "probe_xy")
        _check_dev(out, torch.float32, P * w * w, "out")
        _check_dev(smatrix, torch.complex64, None, "smatrix")
        _check_dev(workspace, torch.uint8, None, "workspace")
        o = _optics(optics)
        head = (self._h, int(f), float(alpha_max_mrad), _ptr(smatrix), _nbytes(smatrix),
                _ptr(probe_xy), int(P), ctypes.byref(o))
        tail = (_ptr(out), _ptr(workspace), workspace.numel(), _stream_ptr(stream))
        if weight is None:
            _native.check(self._L.prism_probe_cbed(*head, *tail))
        else:
            _native.check(self._L.prism_probe_cbed_accumulate(*head, weight, *tail))

    def multislice_outputs(self, probe_xy, optics, edges_mrad, out, workspace, stream=None):
        self._multislice_outputs(None, probe_xy, optics, edges_mrad, out, workspace, stream)

    def multislice_outputs_accumulate(self, probe_xy, optics, edges_mrad, weight, out, workspace,
                                      stream=None):
        """As multislice_outputs, but out += weight * result (frozen-phonon averaging)."""
        self._multislice_outputs(float(weight), probe_xy, optics, edges_mrad, out, workspace,
                                 stream)

    def _multislice_outputs(self, weight, probe_xy, optics, edges_mrad, out, workspace, stream):
        import torch
        det = _Det(edges_mrad)
        P = probe_xy.shape[0]
        _check_dev(probe_xy, torch.float64, 2 * P, "probe_xy")
        _check_dev(out, torch.float64, P * det.edges.shape[0], "out")
        _check_dev(workspace, torch.uint8, None, "workspace")
        o = _optics(optics)
        head = (self._h, _ptr(probe_xy), int(P), ctypes.byref(o), ctypes.byref(det.struct))
        tail = (_ptr(out), _ptr(workspace), workspace.numel(), _stream_ptr(stream))
        if weight is None:
            _native.check(self._L.prism_multislice_outputs(*head, *tail))
        else:
            _native.check(self._L.prism_multislice_outputs_accumulate(*head, weight, *tail))


def _batch_items(items, with_outputs):
    arr = (_native.PrismBuildItem * max(1, len(items)))()
    for k, it in enumerate(items):
        plan, f, amax = it[0], int(it[1]), float(it[2])
        S = it[3] if with_outputs else None
        if S is not None:
            import torch
            B = plan.beam_count(f, amax)
            _check_dev(S, torch.complex64, B * (plan.n // 2) ** 2, f"smatrix of item {k}")
        arr[k] = _native.PrismBuildItem(plan._h, f, amax, _ptr(S) if S is not None else None,
                                        _nbytes(S) if S is not None else 0)
    return arr


def build_batch_workspace_bytes(items):
    """(preferred, minimum) workspace bytes of build_smatrix_batch for items
    [(plan, f, alpha_max_mrad), ...] (or the 4-tuples of that call)."""
    arr = _batch_items(items, False)
    pref, mn = ctypes.c_size_t(), ctypes.c_size_t()
    _native.check(_native.lib().prism_build_batch_workspace_bytes(arr, len(items),
                                                                  ctypes.byref(pref),
                                                                  ctypes.byref(mn)))
    return pref.value, mn.value


def build_smatrix_batch(items, workspace, stream=None):
    """S-matrices of several specimens in shared launches.

    items: [(plan, f, alpha_max_mrad, smatrix), ...], smatrix a complex64
    device tensor [B][n/2][n/2] per item; workspace: uint8 device tensor.
    """
    import torch
    _check_dev(workspace, torch.uint8, None, "workspace")
    arr = _batch_items(items, True)
    _native.check(_native.lib().prism_build_smatrix_batch(arr, len(items), _ptr(workspace),
                                                          workspace.numel(), _stream_ptr(stream)))


class _Requests:
    """prism_probe_request array for probe_batch; keeps the optics and
    detector structs alive while the C array points at them."""

    def __init__(self, requests, with_buffers):
        import torch
        self.keep = []
        self.arr = (_native.PrismProbeRequest * max(1, len(requests)))()
        for k, r in enumerate(requests):
            plan, f, amax = r["plan"], int(r["f"]), float(r["alpha_max_mrad"])
            o = _optics(r["optics"])
            edges = r.get("edges_mrad")
            det = _Det(edges) if edges is not None else None
            self.keep += [o, det]
            S = xy = out = None
            P = int(r["probe_xy"].shape[0]) if r.get("probe_xy") is not None else int(r.get("n_probes", 0))
            if with_buffers:
                S, xy, out = r["smatrix"], r["probe_xy"], r["out"]
                _check_dev(S, torch.complex64, None, f"smatrix of request {k}")
                _check_dev(xy, torch.float64, 2 * P, f"probe_xy of request {k}")
                if det is not None:
                    _check_dev(out, torch.float64, P * det.edges.shape[0], f"out of request {k}")
                else:
                    w = plan.n // (2 * f)
                    _check_dev(out, torch.float32, P * w * w, f"cbed out of request {k}")
            weight = r.get("weight")
            self.arr[k] = _native.PrismProbeRequest(
                plan._h, f, amax, _ptr(S) if S is not None else None,
                _nbytes(S) if S is not None else 0, _ptr(xy) if xy is not None else None, P,
                ctypes.pointer(o), ctypes.pointer(det.struct) if det is not None else None,
                _ptr(out) if (out is not None and det is not None) else None,
                _ptr(out) if (out is not None and det is None) else None,
                0 if weight is None else 1, 0.0 if weight is None else float(weight))


def probe_batch_workspace_bytes(requests):
    """(preferred, minimum) workspace bytes of probe_batch for the same
    requests (device buffers not needed: give n_probes instead of probe_xy)."""
    rq = _Requests(requests, False)
    pref, mn = ctypes.c_size_t(), ctypes.c_size_t()
    _native.check(_native.lib().prism_probe_batch_workspace_bytes(
        rq.arr, len(requests), ctypes.byref(pref), ctypes.byref(mn)))
    return pref.value, mn.value


def probe_batch(requests, workspace, stream=None):
    """Probe steps of several requests in shared launches (prism_probe_batch).

    requests: dicts with plan, f, alpha_max_mrad, smatrix (complex64 device
    [B][n/2][n/2]), probe_xy (float64 device [P][2]), optics (dict as for
    probe_outputs), edges_mrad ([n_det][2]; None for the full CBED), out
    (float64 [P][n_det], or float32 [P][W][W] for the CBED) and optionally
    weight (out += weight * result). workspace: uint8 device tensor.
    """
    import torch
    _check_dev(workspace, torch.uint8, None, "workspace")
    rq = _Requests(requests, True)
    _native.check(_native.lib().prism_probe_batch(rq.arr, len(requests), _ptr(workspace),
                                                  workspace.numel(), _stream_ptr(stream)))


class Server:
    """Resident S-matrices and merged probe queries (prism_server_*).

    Device buffers handed to admit/submit are kept referenced here until
    their queries are reported done (poll / wait) or the specimen evicted.
    """

    @staticmethod
    def workspace_bytes(n_streams, max_probes, max_det, probe_ws_bytes):
        b = ctypes.c_size_t()
        _native.check(_native.lib().prism_server_workspace_bytes(
            int(n_streams), int(max_probes), int(max_det), int(probe_ws_bytes), ctypes.byref(b)))
        return b.value

    def __init__(self, budget_bytes, workspace, n_streams=4, max_probes=65536, max_det=16):
        import torch
        _check_dev(workspace, torch.uint8, None, "workspace")
        self._L = _native.lib()
        h = ctypes.c_void_p()
        _native.check(self._L.prism_server_create(ctypes.byref(h), int(budget_bytes),
                                                  int(n_streams), int(max_probes), int(max_det),
                                                  _ptr(workspace), workspace.numel()))
        self._h = h
        self._ws = workspace
        self._spec = {}
        self._live = {}

    def close(self):
        if getattr(self, "_h", None):
            self._L.prism_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, plan, f, alpha_max_mrad, smatrix, build_workspace=None):
        """Admit (and with build_workspace, build) one specimen's S-matrix; returns its id."""
        import torch
        B = plan.beam_count(f, alpha_max_mrad)
        _check_dev(smatrix, torch.complex64, B * (plan.n // 2) ** 2, "smatrix")
        i = ctypes.c_int()
        wp, wn = (None, 0)
        if build_workspace is not None:
            _check_dev(build_workspace, torch.uint8, None, "build_workspace")
            wp, wn = _ptr(build_workspace), build_workspace.numel()
        _native.check(self._L.prism_server_admit(self._h, plan._h, int(f), float(alpha_max_mrad),
                                                 _ptr(smatrix), _nbytes(smatrix), wp, wn,
                                                 ctypes.byref(i)))
        self._spec[i.value] = (plan, smatrix, build_workspace)
        return i.value

    def submit_build(self, plan, f, alpha_max_mrad, smatrix, build_workspace):
        """Queue one specimen's S-matrix build (dispatched by a flush once it
        fits the budget); returns (specimen id, ticket)."""
        import torch
        B = plan.beam_count(f, alpha_max_mrad)
        _check_dev(smatrix, torch.complex64, B * (plan.n // 2) ** 2, "smatrix")
        _check_dev(build_workspace, torch.uint8, None, "build_workspace")
        i, t = ctypes.c_int(), ctypes.c_longlong()
        _native.check(self._L.prism_server_submit_build(
            self._h, plan._h, int(f), float(alpha_max_mrad), _ptr(smatrix), _nbytes(smatrix),
            _ptr(build_workspace), build_workspace.numel(), ctypes.byref(i), ctypes.byref(t)))
        self._spec[i.value] = (plan, smatrix, build_workspace)
        return i.value, t.value

    def set_lru_eviction(self, enable=True):
        """Let admission release idle S-matrices, least recently used first."""
        _native.check(self._L.prism_server_set_lru_eviction(self._h, 1 if enable else 0))

    def set_dispatch_limit(self, calls_per_slot):
        """Queries wait queued while every slot holds this many calls (0: no limit)."""
        _native.check(self._L.prism_server_set_dispatch_limit(self._h, int(calls_per_slot)))

    def evictions(self, capacity=1024):
        """Ids released by LRU eviction since the last call (their buffers are dropped here)."""
        buf = (ctypes.c_int * int(capacity))()
        n = ctypes.c_int()
        _native.check(self._L.prism_server_evictions(self._h, buf, int(capacity),
                                                     ctypes.byref(n)))
        ids = [buf[k] for k in range(n.value)]
        for sid in ids:
            self._spec.pop(sid, None)
        return ids

    def evict(self, sid):
        _native.check(self._L.prism_server_evict(self._h, int(sid)))
        self._spec.pop(sid, None)

    def submit(self, sid, probe_xy, optics, edges_mrad, out):
        """Queue one query; returns its ticket (runs at the next flush)."""
        import torch
        det = _Det(edges_mrad)
        P = probe_xy.shape[0]
        _check_dev(probe_xy, torch.float64, 2 * P, "probe_xy")
        _check_dev(out, torch.float64, P * det.edges.shape[0], "out")
        o = _optics(optics)
        t = ctypes.c_longlong()
        _native.check(self._L.prism_server_submit(self._h, int(sid), _ptr(probe_xy), int(P),
                                                  ctypes.byref(o), ctypes.byref(det.struct),
                                                  _ptr(out), ctypes.byref(t)))
        self._live[t.value] = (probe_xy, out)
        return t.value

    def flush(self):
        _native.check(self._L.prism_server_flush(self._h))

    def poll(self, capacity=4096):
        """Tickets of queries that finished since the last poll / wait."""
        buf = (ctypes.c_longlong * int(capacity))()
        n = ctypes.c_int()
        _native.check(self._L.prism_server_poll(self._h, buf, int(capacity), ctypes.byref(n)))
        done = [buf[k] for k in range(n.value)]
        for t in done:
            self._live.pop(t, None)
        return done

    def wait(self, ticket):
        _native.check(self._L.prism_server_wait(self._h, int(ticket)))
        self._live.pop(ticket, None)

    def stats(self):
        b, q, f = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_int()
        _native.check(self._L.prism_server_stats(self._h, ctypes.byref(b), ctypes.byref(q),
                                                 ctypes.byref(f)))
        return b.value, q.value, f.value

    def call_stats(self):
        """(probe-step calls dispatched, calls that read several specimens)."""
        c, m = ctypes.c_longlong(), ctypes.c_longlong()
        _native.check(self._L.prism_server_call_stats(self._h, ctypes.byref(c), ctypes.byref(m)))
        return c.value, m.value


def tile_order(nx, ny, tx, ty):
    """Permutation putting a raster scan (x fastest) into tx x ty probe tiles.

    Probes of one tile share their PRISM windows; pass ``probes[perm]`` to
    the probe step and undo with ``untile``. Edge tiles may be partial.
    """
    idx = []
    for by in range(0, ny, ty):
        for bx in range(0, nx, tx):
            for j in range(by, min(by + ty, ny)):
                for i in range(bx, min(bx + tx, nx)):
                    idx.append(j * nx + i)
    return np.asarray(idx, dtype=np.int64)


def untile(values, perm):
    """Inverse of ``values = original[perm]`` along the first axis."""
    out = np.empty_like(values)
    out[perm] = values
    return out
