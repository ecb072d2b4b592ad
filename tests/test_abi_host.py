"""Host-side checks of libprism: no kernel is launched.

Every argument check in the library runs before anything is enqueued, so
these cases never touch device memory even though some pass dummy
pointers (they are rejected first).
"""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_1702_01904_amd import _native, Plan, PrismError, tile_order, untile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "prism.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(prism_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    decl = _declared()
    assert len(decl) >= 15
    assert set(decl) == set(_native.EXPORTS)
    L = _native.lib()
    for name in decl:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _native.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (prism_\w+)", out))
    assert set(decl) <= exported


def _plan(n=128, cell=12.8, E=80.0, H=4):
    return Plan(n, cell, E, np.full(H, 2.0))


def test_plan_accepts_the_supported_grids():
    for n in (128, 192, 256, 384, 512, 576, 768, 1024, 1152, 1536, 2048):
        p = Plan(n, 0.1 * n, 80.0, [2.0])
        assert p.beam_count(4, 30.0) > 0


@pytest.mark.parametrize("n", [100, 64, 4096, 0, -128, 96, 3072, 320, 640, 1728, 2304])
def test_plan_rejects_bad_grid(n):
    with pytest.raises(PrismError) as e:
        Plan(n, 12.8, 80.0, [2.0])
    assert e.value.code == _native.PRISM_EINVAL


@pytest.mark.parametrize("cell,E,th", [(0.0, 80.0, [2.0]), (12.8, -1.0, [2.0]),
                                       (12.8, 80.0, [2.0, 0.0]), (float("nan"), 80.0, [2.0])])
def test_plan_rejects_bad_geometry(cell, E, th):
    with pytest.raises(PrismError):
        Plan(128, cell, E, th)


def test_wavelength_matches_oracle():
    for E in (80.0, 200.0, 300.0):
        p = Plan(128, 12.8, E, [2.0])
        assert p.wavelength == O.wavelength(E)


@pytest.mark.parametrize("n,cell,E,alpha,f", [(128, 12.8, 80.0, 20.0, 1), (128, 12.8, 80.0, 20.0, 2),
                                              (1024, 40.0, 200.0, 25.0, 4),
                                              (1024, 40.0, 200.0, 25.0, 8),
                                              (1024, 40.0, 200.0, 25.0, 16),
                                              (256, 25.6, 80.0, 20.0, 4),
                                              (2048, 80.0, 80.0, 20.0, 8)])
def test_beam_set_identical_to_oracle(n, cell, E, alpha, f):
    p = Plan(n, cell, E, [2.0])
    lam = O.wavelength(E)
    amax = O.default_alpha_max(alpha * 1e-3, f, lam, 1 / cell) * 1e3
    assert abs(p.alpha_max_default(alpha, f) - amax) <= 1e-12 * amax
    got = p.beams(f, amax)
    ref = O.beam_set(n, cell, lam, f, amax * 1e-3)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref.astype(np.int32))
    assert p.smatrix_bytes(f, amax) == len(ref) * (n // 2) ** 2 * 8


def test_beam_set_edge_cases():
    p = _plan()
    with pytest.raises(PrismError):
        p.beams(3, 30.0)          # 128 % 6 != 0
    with pytest.raises(PrismError):
        p.beams(0, 30.0)
    with pytest.raises(PrismError):
        p.beams(2, -1.0)
    with pytest.raises(PrismError):
        p.beams(2, float("inf"))
    # tiny alpha_max keeps only the zero beam
    assert p.beams(2, 1e-6).tolist() == [[0, 0]]
    # huge alpha_max is capped by the half-band limit
    big = p.beams(1, 1e6)
    assert ((big.astype(np.int64) ** 2).sum(axis=1) * 16 < 128 * 128).all()
    assert len(big) == sum(1 for m in range(-40, 41) for k in range(-40, 41)
                           if 16 * (m * m + k * k) < 128 * 128)


def test_workspace_queries_are_consistent():
    p = _plan(256, 25.6, 80.0, 8)
    amax = p.alpha_max_default(20.0, 2)
    pref, mn = p.build_workspace_bytes(2, amax)
    assert 0 < mn <= pref
    pref_m, mn_m = p.multislice_workspace_bytes(4)
    assert 0 < mn_m <= pref_m
    optics = dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0)
    pref_p, mn_p = p.probe_workspace_bytes(2, amax, optics)
    assert 0 < mn_p <= pref_p
    with pytest.raises(PrismError):
        p.multislice_workspace_bytes(0)
    with pytest.raises(PrismError):
        p.multislice_workspace_bytes(33)


def test_probe_precision_setting_and_workspace():
    p = _plan(256, 25.6, 80.0, 8)
    amax = p.alpha_max_default(20.0, 2)
    optics = dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0)
    pref32, mn32 = p.probe_workspace_bytes(2, amax, optics)
    L, h = _raw(p)
    for bad in (-1, 3, 99):
        assert L.prism_set_probe_precision(h, bad) == _native.PRISM_EINVAL
    assert L.prism_set_probe_precision(None, 1) == _native.PRISM_EINVAL
    with pytest.raises(ValueError):
        p.set_probe_precision("fp8")
    n_act = int(np.sum(np.hypot(*p.beams(2, amax).T.astype(float)) * 2 * p.wavelength / 25.6
                       <= 20e-3))
    n_actp = -(-n_act // 64) * 64
    for prec in ("bf16", "fp16"):
        p.set_probe_precision(prec)
        pref, mn = p.probe_workspace_bytes(2, amax, optics)
        # the packed 16-bit S-matrix copy is part of every 16-bit workspace
        assert mn >= 128 * 128 * n_actp * 4
        assert 0 < mn <= pref
    p.set_probe_precision("fp32")
    assert p.probe_workspace_bytes(2, amax, optics) == (pref32, mn32)


def test_probe_group_shapes():
    p = Plan(1024, 40.0, 200.0, [2.0])
    p.set_tuning({})                      # the library's own choice, per window size
    assert p.probe_group(4) == (64, 8, 8)
    assert p.probe_group(8) == (32, 8, 4)
    assert p.probe_group(16) == (16, 4, 4)
    p.set_tuning({"probe_group": 16})     # a fixed group for every factor
    assert p.probe_group(4) == (16, 4, 4)
    assert p.probe_group(8) == (16, 4, 4)


def _raw(p):
    return p._L, p._h


SBIG = 1 << 40   # S-matrix byte size passed with a dummy pointer: large enough for any case


def test_errors_before_any_launch():
    p = _plan()
    L, h = _raw(p)
    amax = p.alpha_max_default(20.0, 2)
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails validation first
    # potential not set
    r = L.prism_build_smatrix(h, 2, amax, dummy, SBIG, dummy, 1 << 30, None)
    assert r == _native.PRISM_ENOTREADY
    assert b"potential" in L.prism_last_error()
    # null buffers
    assert L.prism_build_smatrix(h, 2, amax, None, SBIG, dummy, 1 << 30, None) == _native.PRISM_EINVAL
    L.prism_set_potential_slices(h, dummy)
    # workspace too small
    r = L.prism_build_smatrix(h, 2, amax, dummy, SBIG, dummy, 1024, None)
    assert r == _native.PRISM_ENOSPACE
    # bad f
    assert L.prism_build_smatrix(h, 3, amax, dummy, SBIG, dummy, 1 << 30, None) == _native.PRISM_EINVAL

    optics = _native.PrismOptics(20.0, 0.0, 0.0)
    edges = (ctypes.c_double * 2)(40.0, 150.0)
    det = _native.PrismDetector(1, edges)
    # multislice: too small workspace, bad detector, aperture past the band limit
    r = L.prism_multislice_outputs(h, dummy, 4, ctypes.byref(optics), ctypes.byref(det), dummy,
                                   dummy, 64, None)
    assert r == _native.PRISM_ENOSPACE
    bad_det = _native.PrismDetector(0, edges)
    assert L.prism_multislice_outputs(h, dummy, 4, ctypes.byref(optics), ctypes.byref(bad_det),
                                      dummy, dummy, 1 << 30, None) == _native.PRISM_EINVAL
    rev = (ctypes.c_double * 2)(150.0, 40.0)
    rev_det = _native.PrismDetector(1, rev)
    assert L.prism_multislice_outputs(h, dummy, 4, ctypes.byref(optics), ctypes.byref(rev_det),
                                      dummy, dummy, 1 << 30, None) == _native.PRISM_EINVAL
    wide = _native.PrismOptics(120.0, 0.0, 0.0)   # 120 mrad > 104 mrad half-band at 80 keV
    assert L.prism_multislice_outputs(h, dummy, 4, ctypes.byref(wide), ctypes.byref(det), dummy,
                                      dummy, 1 << 30, None) == _native.PRISM_EINVAL
    # zero probes is a no-op that needs no buffers
    assert L.prism_multislice_outputs(h, None, 0, ctypes.byref(optics), ctypes.byref(det), None,
                                      None, 0, None) == _native.PRISM_OK
    # probe step: window too large (f = 1 at n = 128 gives W = 64: fine; n=1024 f=1 W=512: not)
    big = Plan(1024, 102.4, 80.0, [2.0])
    Lb, hb = _raw(big)
    amax1 = big.alpha_max_default(20.0, 1)
    r = Lb.prism_probe_outputs(hb, 1, amax1, dummy, SBIG, dummy, 4, ctypes.byref(optics),
                               ctypes.byref(det), dummy, dummy, 1 << 30, None)
    assert r == _native.PRISM_EINVAL and b"window" in Lb.prism_last_error()
    # tilt: aperture pushed across the half-band limit (104 mrad at 80 keV)
    tilted = _native.PrismOptics(20.0, 0.0, 0.0, 90.0, 0.0)
    assert L.prism_multislice_outputs(h, dummy, 4, ctypes.byref(tilted), ctypes.byref(det), dummy,
                                      dummy, 1 << 30, None) == _native.PRISM_EINVAL
    assert b"half-band" in L.prism_last_error()
    # tilt: semi-angle + tilt beyond the beam set's alpha_max
    t5 = _native.PrismOptics(20.0, 0.0, 0.0, 3.0, 4.0)
    r = L.prism_probe_outputs(h, 2, 24.0, dummy, SBIG, dummy, 4, ctypes.byref(t5), ctypes.byref(det),
                              dummy, dummy, 1 << 30, None)
    assert r == _native.PRISM_EINVAL and b"tilt" in L.prism_last_error()
    nan_tilt = _native.PrismOptics(20.0, 0.0, 0.0, float("nan"), 0.0)
    assert L.prism_multislice_outputs(h, dummy, 4, ctypes.byref(nan_tilt), ctypes.byref(det),
                                      dummy, dummy, 1 << 30, None) == _native.PRISM_EINVAL
    # probe step: semi-angle beyond the beam set's alpha_max
    wider = _native.PrismOptics(amax + 1.0, 0.0, 0.0)
    r = L.prism_probe_outputs(h, 2, amax, dummy, SBIG, dummy, 4, ctypes.byref(wider), ctypes.byref(det),
                              dummy, dummy, 1 << 30, None)
    assert r == _native.PRISM_EINVAL and b"alpha_max" in L.prism_last_error()
    # CBED output: null output buffer, and the same checks as the detector path
    r = L.prism_probe_cbed(h, 2, amax, dummy, SBIG, dummy, 4, ctypes.byref(optics), None, dummy,
                           1 << 30, None)
    assert r == _native.PRISM_EINVAL
    r = L.prism_probe_cbed(h, 2, amax, dummy, SBIG, dummy, 4, ctypes.byref(wider), dummy, dummy,
                           1 << 30, None)
    assert r == _native.PRISM_EINVAL
    assert L.prism_probe_cbed(h, 2, amax, None, 0, None, 0, ctypes.byref(optics), None, None, 0,
                              None) == _native.PRISM_OK
    # probe step: too small workspace
    r = L.prism_probe_outputs(h, 2, amax, dummy, SBIG, dummy, 4, ctypes.byref(optics), ctypes.byref(det),
                              dummy, dummy, 128, None)
    assert r == _native.PRISM_ENOSPACE
    # accumulating forms: weight must be finite; otherwise the checks of the
    # call they extend, and zero probes is a no-op
    for wgt in (float("nan"), float("inf")):
        r = L.prism_probe_outputs_accumulate(h, 2, amax, dummy, SBIG, dummy, 4, ctypes.byref(optics),
                                             ctypes.byref(det), wgt, dummy, dummy, 1 << 30, None)
        assert r == _native.PRISM_EINVAL and b"weight" in L.prism_last_error()
        r = L.prism_probe_cbed_accumulate(h, 2, amax, dummy, SBIG, dummy, 4, ctypes.byref(optics), wgt,
                                          dummy, dummy, 1 << 30, None)
        assert r == _native.PRISM_EINVAL and b"weight" in L.prism_last_error()
        r = L.prism_multislice_outputs_accumulate(h, dummy, 4, ctypes.byref(optics),
                                                  ctypes.byref(det), wgt, dummy, dummy, 1 << 30,
                                                  None)
        assert r == _native.PRISM_EINVAL and b"weight" in L.prism_last_error()
    r = L.prism_probe_outputs_accumulate(h, 2, amax, dummy, SBIG, dummy, 4, ctypes.byref(optics),
                                         None, 0.5, dummy, dummy, 1 << 30, None)
    assert r == _native.PRISM_EINVAL
    r = L.prism_probe_cbed_accumulate(h, 2, amax, dummy, SBIG, dummy, 4, ctypes.byref(wider), 0.5,
                                      dummy, dummy, 1 << 30, None)
    assert r == _native.PRISM_EINVAL and b"alpha_max" in L.prism_last_error()
    r = L.prism_multislice_outputs_accumulate(h, dummy, 4, ctypes.byref(optics), ctypes.byref(det),
                                              0.5, dummy, dummy, 64, None)
    assert r == _native.PRISM_ENOSPACE
    assert L.prism_probe_outputs_accumulate(h, 2, amax, None, 0, None, 0, ctypes.byref(optics),
                                            ctypes.byref(det), 0.5, None, None, 0,
                                            None) == _native.PRISM_OK


def test_null_plan_and_pointers():
    L = _native.lib()
    n = ctypes.c_int()
    assert L.prism_beam_count(None, 2, 30.0, ctypes.byref(n)) == _native.PRISM_EINVAL
    assert L.prism_plan_create(None, None) == _native.PRISM_EINVAL
    L.prism_plan_destroy(None)


def test_tile_order_roundtrip():
    perm = tile_order(16, 12, 8, 4)
    assert sorted(perm.tolist()) == list(range(16 * 12))
    assert perm[:8].tolist() == list(range(8))
    assert perm[8:16].tolist() == list(range(16, 24))
    vals = np.arange(16 * 12)[perm] * 3
    assert np.array_equal(untile(vals, perm), np.arange(16 * 12) * 3)
    odd = tile_order(19, 7, 8, 8)
    assert sorted(odd.tolist()) == list(range(19 * 7))


def test_batch_build_validation():
    from paper_1702_01904_amd import build_batch_workspace_bytes
    L = _native.lib()
    a = Plan(128, 12.8, 80.0, [2.0] * 4)
    b = Plan(128, 12.8, 80.0, [2.0] * 6)      # same medium, more slices: one group
    c = Plan(128, 12.8, 120.0, [2.0] * 4)     # other energy: own group
    fa, fb, fc = 2, 1, 2
    items = [(a, fa, a.alpha_max_default(20.0, fa)), (b, fb, b.alpha_max_default(20.0, fb)),
             (c, fc, c.alpha_max_default(20.0, fc))]
    pref, mn = build_batch_workspace_bytes(items)
    # one group's minimum: the transmissions of both members (10 slices of
    # 128^2 complex64) dominate
    assert mn >= 10 * 128 * 128 * 8 and pref >= mn
    p1, m1 = build_batch_workspace_bytes(items[:2])
    p2, m2 = build_batch_workspace_bytes(items[2:])
    assert pref == max(p1, p2) and mn == max(m1, m2)
    arr = (_native.PrismBuildItem * 3)()
    dummy = ctypes.c_void_p(0x1000)
    for k, (p, f, am) in enumerate(items):
        arr[k] = _native.PrismBuildItem(p._h, f, am, dummy, SBIG)
    # potential slices not set (checked per item, before any launch)
    r = L.prism_build_smatrix_batch(arr, 3, dummy, 1 << 30, None)
    assert r == _native.PRISM_ENOTREADY and b"item 0" in L.prism_last_error()
    # bad items
    assert L.prism_build_smatrix_batch(arr, -1, dummy, 1 << 30, None) == _native.PRISM_EINVAL
    assert L.prism_build_smatrix_batch(None, 2, dummy, 1 << 30, None) == _native.PRISM_EINVAL
    assert L.prism_build_smatrix_batch(arr, 0, None, 0, None) == _native.PRISM_OK
    bad = (_native.PrismBuildItem * 2)()
    bad[0] = arr[0]
    bad[1] = _native.PrismBuildItem(b._h, 3, 30.0, dummy, SBIG)  # 128 % 6 != 0
    r = L.prism_build_smatrix_batch(bad, 2, dummy, 1 << 30, None)
    assert r == _native.PRISM_EINVAL and b"item 1" in L.prism_last_error()
    bad[1] = _native.PrismBuildItem(None, 1, 30.0, dummy, SBIG)
    assert L.prism_build_smatrix_batch(bad, 2, dummy, 1 << 30, None) == _native.PRISM_EINVAL
    pref_q, min_q = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.prism_build_batch_workspace_bytes(bad, 2, ctypes.byref(pref_q),
                                               ctypes.byref(min_q)) == _native.PRISM_EINVAL
    for p in (a, b, c):
        L.prism_set_potential_slices(p._h, dummy)
    nulls = (_native.PrismBuildItem * 1)()
    nulls[0] = _native.PrismBuildItem(a._h, fa, items[0][2], None, 0)
    r = L.prism_build_smatrix_batch(nulls, 1, dummy, 1 << 30, None)
    assert r == _native.PRISM_EINVAL and b"S-matrix" in L.prism_last_error()
    assert L.prism_build_smatrix_batch(arr, 3, None, 1 << 30, None) == _native.PRISM_EINVAL
    # workspace below the minimum of the first group
    r = L.prism_build_smatrix_batch(arr, 3, dummy, mn // 2, None)
    assert r == _native.PRISM_ENOSPACE


def test_server_sizes_and_checks_before_any_stream():
    from paper_1702_01904_amd import Server
    L = _native.lib()
    b = Server.workspace_bytes(4, 1000, 16, 1 << 20)
    # four regions of staged positions (16 B each), outputs (128 B each) and
    # the probe-step workspace, 256-byte aligned
    assert b >= 4 * (1000 * 16 + 1000 * 128 + (1 << 20))
    assert Server.workspace_bytes(1, 1000, 16, 0) < b
    out = ctypes.c_size_t()
    assert L.prism_server_workspace_bytes(0, 10, 1, 0, ctypes.byref(out)) == _native.PRISM_EINVAL
    assert L.prism_server_workspace_bytes(17, 10, 1, 0, ctypes.byref(out)) == _native.PRISM_EINVAL
    assert L.prism_server_workspace_bytes(1, 0, 1, 0, ctypes.byref(out)) == _native.PRISM_EINVAL
    assert L.prism_server_workspace_bytes(1, 10, 33, 0, ctypes.byref(out)) == _native.PRISM_EINVAL
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)
    assert L.prism_server_create(None, 1 << 30, 2, 10, 1, dummy, 1 << 20) == _native.PRISM_EINVAL
    assert L.prism_server_create(ctypes.byref(h), 1 << 30, 2, 10, 1, None,
                                 1 << 20) == _native.PRISM_EINVAL
    r = L.prism_server_create(ctypes.byref(h), 1 << 30, 2, 1000, 16, dummy, 1024)
    assert r == _native.PRISM_ENOSPACE and not h.value
    # calls on a null server fail cleanly
    assert L.prism_server_flush(None) == _native.PRISM_EINVAL
    assert L.prism_server_wait(None, 1) == _native.PRISM_EINVAL
    n = ctypes.c_int()
    assert L.prism_server_poll(None, None, 0, ctypes.byref(n)) == _native.PRISM_EINVAL
    assert L.prism_server_stats(None, None, None, None) == _native.PRISM_EINVAL
    L.prism_server_destroy(None)


def test_probe_order():
    from synth import build_inputs
    d = build_inputs("fcc1024", 0, n_slices=1)
    p = Plan(d["n"], d["cell"], d["energy_keV"], d["thickness"])
    ns = d["n"] // 2
    for f, (tx, ty) in ((4, (8, 8)), (8, (8, 4)), (16, (4, 4))):
        perm = p.probe_order(f, d["probes"])
        assert sorted(perm.tolist()) == list(range(len(d["probes"])))
        # the 256 x 256 raster at two S-pixels comes out as the probe tiles
        G = tx * ty
        t = tile_order(256, 256, tx, ty)
        chunks = lambda q: sorted(tuple(sorted(q[i:i + G])) for i in range(0, len(q), G))
        assert chunks(perm) == chunks(t)
    # scattered positions: runs of 64 consecutive probes get tighter
    rng = np.random.default_rng(3)
    xy = rng.uniform(0.0, d["cell"], (4096, 2))
    perm = p.probe_order(4, xy)
    dxs = d["cell"] / ns

    def spread(q):
        c = np.floor(q / dxs + 0.5)
        return np.mean([np.ptp(c[i:i + 64], axis=0).max() for i in range(0, len(c), 64)])
    assert spread(xy[perm]) < 0.35 * spread(xy)
    assert len(p.probe_order(4, np.zeros((0, 2)))) == 0
    L = _native.lib()
    assert L.prism_probe_order(p._h, 3, None, 0, None) == _native.PRISM_EINVAL   # 1024 % 6
    assert L.prism_probe_order(p._h, 4, None, 5, None) == _native.PRISM_EINVAL
    assert L.prism_probe_order(p._h, 4, None, -1, None) == _native.PRISM_EINVAL


def test_traffic_hash_ignores_comments_only():
    # bench.py reports stored HBM traffic only while the kernel sources hash
    # to the value the counters were taken at; comments do not count, code
    # (string literals included) does
    import bench
    a = 'int a = 1;  // "x"\n/* block\n comment */\nconst char* s = "//kept /* too */";\n'
    b = 'int a = 1;\n\n   \nconst char* s = "//kept /* too */";   \n'
    c = 'int a = 2;\nconst char* s = "//kept /* too */";\n'
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
    assert '"//kept /* too */"' in bench._code_only(a)
    assert len(bench.kernel_source_sha()) == 16


def test_undersized_smatrix_rejected_before_any_launch():
    # an S-matrix built for another f / alpha_max (fewer beams) must not
    # reach the kernels: every call that takes S checks its byte size against
    # prism_smatrix_bytes of its own f and alpha_max
    p = _plan()
    L, h = _raw(p)
    dummy = ctypes.c_void_p(0x1000)
    L.prism_set_potential_slices(h, dummy)
    amax1 = p.alpha_max_default(20.0, 1)
    need = p.smatrix_bytes(1, amax1)
    small = p.smatrix_bytes(2, p.alpha_max_default(20.0, 2))    # the f = 2 set: 49 beams
    assert small < need
    optics = _native.PrismOptics(20.0, 0.0, 0.0)
    edges = (ctypes.c_double * 2)(40.0, 150.0)
    det = _native.PrismDetector(1, edges)
    for nbytes, ok in ((small, False), (need - 1, False), (need, True)):
        calls = [
            L.prism_build_smatrix(h, 1, amax1, dummy, nbytes, dummy, 64, None),
            L.prism_probe_outputs(h, 1, amax1, dummy, nbytes, dummy, 4, ctypes.byref(optics),
                                  ctypes.byref(det), dummy, dummy, 64, None),
            L.prism_probe_outputs_accumulate(h, 1, amax1, dummy, nbytes, dummy, 4,
                                             ctypes.byref(optics), ctypes.byref(det), 0.5, dummy,
                                             dummy, 64, None),
            L.prism_probe_cbed(h, 1, amax1, dummy, nbytes, dummy, 4, ctypes.byref(optics), dummy,
                               dummy, 64, None),
            L.prism_probe_cbed_accumulate(h, 1, amax1, dummy, nbytes, dummy, 4,
                                          ctypes.byref(optics), 0.5, dummy, dummy, 64, None),
        ]
        for r in calls:
            if ok:   # the size passes; the 64-byte workspace is what fails
                assert r == _native.PRISM_ENOSPACE
            else:
                assert r == _native.PRISM_EINVAL
                assert b"prism_smatrix_bytes" in L.prism_last_error()
    item = (_native.PrismBuildItem * 1)()
    item[0] = _native.PrismBuildItem(h, 1, amax1, dummy, small)
    r = L.prism_build_smatrix_batch(item, 1, dummy, 1 << 30, None)
    assert r == _native.PRISM_EINVAL and b"prism_smatrix_bytes" in L.prism_last_error()


@pytest.mark.parametrize("n,cell,E,alpha", [(128, 12.8, 80.0, 20.0), (1024, 40.0, 200.0, 25.0),
                                            (2048, 80.0, 80.0, 20.0), (384, 38.4, 80.0, 11.5)])
def test_alpha_max_and_active_beams_match_the_oracle(n, cell, E, alpha):
    p = Plan(n, cell, E, [2.0])
    lam = O.wavelength(E)
    for f in (1, 2, 4, 8):
        if n % (2 * f):
            continue
        amax = p.alpha_max_default(alpha, f)
        ref = O.default_alpha_max(alpha * 1e-3, f, lam, 1.0 / cell) * 1e3
        assert abs(amax - ref) <= 1e-12 * ref
        beams = O.beam_set(n, cell, lam, f, amax * 1e-3)
        optics = dict(alpha_mrad=alpha)
        _, A = O.prism_coefficients(beams, f, cell, lam, optics, 0.0, 0.0)
        assert p.active_beam_count(f, amax, optics) == int(A.sum())
    L, h = _raw(p)
    v = ctypes.c_double()
    assert L.prism_alpha_max(h, 0, alpha, ctypes.byref(v)) == _native.PRISM_EINVAL
    assert L.prism_alpha_max(h, 1, -1.0, ctypes.byref(v)) == _native.PRISM_EINVAL
    assert L.prism_alpha_max(None, 1, alpha, ctypes.byref(v)) == _native.PRISM_EINVAL


def test_noalloc_rejects_probe_steps_beyond_its_scratch():
    # fcc1024 at f = 4: 305 active beams, a 649 MiB minimum FP32 workspace,
    # more than the 256 MiB library-held scratch; refused before any device call
    p = Plan(1024, 40.0, 200.0, [2.0] * 50)
    L, h = _raw(p)
    amax = p.alpha_max_default(25.0, 4)
    _, mn = p.probe_workspace_bytes(4, amax, dict(alpha_mrad=25.0))
    assert mn > _native.PRISM_NOALLOC_SCRATCH_BYTES
    dummy = ctypes.c_void_p(0x1000)
    optics = _native.PrismOptics(25.0, 0.0, 0.0)
    edges = (ctypes.c_double * 2)(0.0, 200.0)
    det = _native.PrismDetector(1, edges)
    r = L.prism_probe_outputs_noalloc(h, 4, amax, dummy, SBIG, dummy, 16, ctypes.byref(optics),
                                      ctypes.byref(det), dummy, None)
    assert r == _native.PRISM_ENOSPACE and b"library-held" in L.prism_last_error()
    # the probe step's own checks come first
    r = L.prism_probe_outputs_noalloc(h, 3, amax, dummy, SBIG, dummy, 16, ctypes.byref(optics),
                                      ctypes.byref(det), dummy, None)
    assert r == _native.PRISM_EINVAL


def test_tuning_roundtrip_and_validation():
    p = _plan(1024, 40.0, 200.0, 2)
    p.set_tuning({})
    d = p.tuning()
    assert d == dict(row_iters=16, row_min_groups=512, col_iters=8, col_min_groups=256,
                     wave_chunk_mib=256, probe_group=0, window_tile_div=4)
    amax = p.alpha_max_default(25.0, 4)
    pref0, mn0 = p.build_workspace_bytes(4, amax)
    p.set_tuning(dict(row_iters=4, col_min_groups=128, wave_chunk_mib=128, probe_group=32,
                      window_tile_div=2))
    t = p.tuning()
    assert (t["row_iters"], t["col_min_groups"], t["wave_chunk_mib"], t["probe_group"],
            t["window_tile_div"]) == (4, 128, 128, 32, 2)
    pref1, mn1 = p.build_workspace_bytes(4, amax)
    assert mn1 == mn0 and pref1 < pref0          # half the wave state per launch
    assert p.probe_group(4) == (32, 8, 4)
    for bad in (dict(row_iters=3), dict(col_iters=128), dict(wave_chunk_mib=8),
                dict(probe_group=48), dict(window_tile_div=65), dict(row_min_groups=-1)):
        with pytest.raises(PrismError):
            p.set_tuning(bad)
    assert p.tuning() == t                          # a refused setting changes nothing


def _req(p, f, amax, P, optics=None, det=None, S=SBIG):
    o = _native.PrismOptics(20.0, 0.0, 0.0, 0.0, 0.0) if optics is None else optics
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails validation first
    return _native.PrismProbeRequest(p._h, f, amax, dummy, S, dummy, P, ctypes.pointer(o),
                                     ctypes.pointer(det) if det is not None else None, dummy,
                                     dummy, 0, 1.0), o


def test_probe_batch_validation_before_any_launch():
    L = _native.lib()
    p = _plan(256, 25.6)
    edges = np.array([[0.0, 20.0], [20.0, 40.0]])
    det = _native.PrismDetector(2, edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    amax = p.alpha_max_default(20.0, 4)
    arr = (_native.PrismProbeRequest * 3)()
    keep = []
    for k, (f, a) in enumerate(((4, amax), (4, amax), (4, amax))):
        arr[k], o = _req(p, f, a, 10, det=det)
        keep.append(o)
    ws = ctypes.c_void_p(0x1000)
    assert L.prism_probe_batch(arr, -1, ws, 1 << 30, None) == _native.PRISM_EINVAL
    assert L.prism_probe_batch(None, 2, ws, 1 << 30, None) == _native.PRISM_EINVAL
    assert L.prism_probe_batch(arr, 0, None, 0, None) == _native.PRISM_OK
    # request 1: n not divisible by 2 f; nothing runs, the message names it
    arr[1].f = 5
    assert L.prism_probe_batch(arr, 3, ws, 1 << 30, None) == _native.PRISM_EINVAL
    assert b"request 1" in L.prism_last_error()
    arr[1].f = 4
    # request 2: undersized S-matrix
    arr[2].smatrix_bytes = 8
    assert L.prism_probe_batch(arr, 3, ws, 1 << 30, None) == _native.PRISM_EINVAL
    assert b"request 2" in L.prism_last_error() and b"S-matrix" in L.prism_last_error()
    arr[2].smatrix_bytes = SBIG
    # request 0: accumulate with a non-finite weight
    arr[0].accumulate, arr[0].weight = 1, float("nan")
    assert L.prism_probe_batch(arr, 3, ws, 1 << 30, None) == _native.PRISM_EINVAL
    assert b"request 0" in L.prism_last_error()
    arr[0].accumulate, arr[0].weight = 0, 1.0
    # null workspace with probes to run
    assert L.prism_probe_batch(arr, 3, None, 0, None) == _native.PRISM_EINVAL


def test_probe_batch_workspace_and_class():
    L = _native.lib()
    p = _plan(256, 25.6)
    q = _plan(128, 12.8)
    p.set_tuning({})
    q.set_tuning({})
    edges = np.array([[0.0, 20.0]])
    det = _native.PrismDetector(1, edges.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    a4, a2 = p.alpha_max_default(20.0, 4), q.alpha_max_default(20.0, 2)
    # one request with many probes: the sizes of the single call's query
    arr = (_native.PrismProbeRequest * 2)()
    arr[0], o0 = _req(p, 4, a4, 1 << 20, det=det)
    pref, mn = ctypes.c_size_t(), ctypes.c_size_t()
    _native.check(L.prism_probe_batch_workspace_bytes(arr, 1, ctypes.byref(pref), ctypes.byref(mn)))
    sp, sm = p.probe_workspace_bytes(4, a4, dict(alpha_mrad=20.0))
    assert (pref.value, mn.value) == (sp, sm)
    # two specimens of one class: the preferred fill holds both packed S-matrices
    arr[1], o1 = _req(q, 2, a2, 1 << 20, det=det)
    assert p.probe_class(4) == q.probe_class(2) != p.probe_class(2)
    _native.check(L.prism_probe_batch_workspace_bytes(arr, 2, ctypes.byref(pref), ctypes.byref(mn)))
    assert mn.value == max(sm, q.probe_workspace_bytes(2, a2, dict(alpha_mrad=20.0))[1])
    assert pref.value > sp
    # the class key follows the plan's tuning and precision
    p.set_tuning({"window_tile_div": 2})
    assert p.probe_class(4) != q.probe_class(2)
    p.set_tuning({})
    p.set_probe_precision("bf16")
    assert p.probe_class(4) != q.probe_class(2)
    with pytest.raises(PrismError):
        p.probe_class(3)          # 256 not divisible by 6
