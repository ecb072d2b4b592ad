"""Grids with a factor 3 or 9 (n = 3 * 2^k, 9 * 2^k: radix-3/9 LDS FFT
stages in the slice passes, the exit extraction and the multislice probe)
and windows of 12, 18, 24, 36, 48, 72, 96, 144 and 192 pixels, against the
FP64 oracle.

Gate: eps_rel <= 1e-4 (FP32), <= 1e-2 (BF16), per S-matrix beam and over the
outputs.
"""
import numpy as np
import pytest

import oracle as O
from synth import build_inputs

import _gpu as G

pytestmark = pytest.mark.gpu

TOL = 1e-4
TOL16 = 1e-2


def eps(a, ref):
    a = np.asarray(a)
    ref = np.asarray(ref)
    assert np.all(np.isfinite(a))
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


def _amax(d, f):
    lam = O.wavelength(d["energy_keV"])
    return O.default_alpha_max(d["optics"]["alpha_mrad"] * 1e-3, f, lam, 1.0 / d["cell"]) * 1e3


@pytest.fixture(scope="module")
def t192():
    d = build_inputs("tiny192", 0)
    return d, G.make_plan(d)


@pytest.fixture(scope="module")
def m384():
    d = build_inputs("mid384", 0)
    return d, G.make_plan(d)


def test_multislice_192(t192):
    d, plan = t192
    D = G.multislice_outputs(plan, d["probes"], d["optics"], d["edges"])
    ref = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"], d["optics"],
                            d["probes"], d["edges"])
    e = eps(D, ref)
    print(f"n=192 multislice eps_rel={e:.3e}")
    assert e <= TOL


@pytest.mark.parametrize("f", [3, 4, 6])
def test_smatrix_and_prism_192(t192, f):
    d, plan = t192
    amax = _amax(d, f)
    S = G.build_smatrix(plan, f, amax)
    beams, Sref = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f, amax)
    assert np.array_equal(plan.beams(f, amax), beams.astype(np.int32))
    Sh = S.cpu().numpy()
    worst = max(eps(Sh[b], Sref[b]) for b in range(len(beams)))
    print(f"n=192 f={f} B={len(beams)} worst beam eps_rel={worst:.3e}")
    assert worst <= TOL
    D = G.probe_outputs(plan, f, amax, S, d["probes"], d["optics"], d["edges"])
    ref, Cref = O.prism_outputs(Sref, beams, f, d["cell"], d["energy_keV"], d["optics"],
                                d["probes"], d["edges"], return_cbed=True)
    e = eps(D, ref)
    print(f"n=192 prism f={f} W={plan.n // (2 * f)} eps_rel={e:.3e}")
    assert e <= TOL
    C = G.probe_cbed(plan, f, amax, S, d["probes"][::5], d["optics"])
    assert eps(C, Cref[::5]) <= TOL


def test_multislice_384_sampled(m384):
    d, plan = m384
    pr = d["probes"][[0, 76, 152]]
    D = G.multislice_outputs(plan, pr, d["optics"], d["edges"])
    ref = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"], d["optics"],
                            pr, d["edges"])
    e = eps(D, ref)
    print(f"n=384 multislice eps_rel={e:.3e}")
    assert e <= TOL


@pytest.mark.parametrize("f", [3, 4, 6, 8, 12, 16])
def test_prism_384(m384, f):
    d, plan = m384
    amax = _amax(d, f)
    S = G.build_smatrix(plan, f, amax)
    beams, Sref = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f, amax)
    Sh = S.cpu().numpy()
    worst = max(eps(Sh[b], Sref[b]) for b in range(len(beams)))
    assert worst <= TOL
    ref = O.prism_outputs(Sref, beams, f, d["cell"], d["energy_keV"], d["optics"], d["probes"],
                          d["edges"])
    D = G.probe_outputs(plan, f, amax, S, d["probes"], d["optics"], d["edges"])
    e = eps(D, ref)
    print(f"n=384 prism f={f} W={plan.n // (2 * f)} B={len(beams)} worst beam {worst:.3e} "
          f"eps_rel={e:.3e}")
    assert e <= TOL
    plan.set_probe_precision("bf16")
    try:
        D16 = G.probe_outputs(plan, f, amax, S, d["probes"], d["optics"], d["edges"])
    finally:
        plan.set_probe_precision("fp32")
    assert eps(D16, ref) <= TOL16


@pytest.mark.parametrize("n,f,H", [(768, 6, 5), (768, 4, 3), (1536, 12, 3), (576, 4, 3),
                                   (576, 12, 3), (1152, 8, 3), (1152, 6, 2), (576, 16, 3),
                                   (576, 8, 3), (1152, 16, 2), (1152, 4, 2), (1536, 4, 2)])
def test_large_3x2k_grids_sampled(n, f, H):
    # 576^2 .. 1536^2 (0.1 A pixels, random atoms; windows 18 .. 192): one
    # multislice probe and PRISM probes (two at 768^2, one elsewhere)
    # against one-probe oracle runs; for W = 144 and 192 (the two-pass
    # window transform over HBM) the diffraction pattern as well
    cfg = dict(
        specimen=dict(kind="random", cell=(0.1 * n, 0.1 * n, 2.0 * H),
                      n_atoms=int(0.015 * (0.1 * n) ** 2 * 2.0 * H), z_choices=(6, 14, 29, 79)),
        n=n, n_slices=H, slice_A=2.0, energy_keV=80.0,
        optics=dict(alpha_mrad=20.0, C1_A=-15.0, C3_A=0.0),
        scan=dict(nx=4, ny=4, step_A=3.1, origin_A=(7.0, 11.0)),
        detectors=[(0.0, 20.0), (40.0, 100.0)], f_values=(f,))
    d = build_inputs(cfg, 5)
    plan = G.make_plan(d)
    pr = d["probes"][[0, 9]]
    Dm = G.multislice_outputs(plan, pr[:1], d["optics"], d["edges"])
    refm = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"], d["optics"],
                             pr[:1], d["edges"])
    em = eps(Dm, refm)
    amax = _amax(d, f)
    S = G.build_smatrix(plan, f, amax)
    D = G.probe_outputs(plan, f, amax, S, d["probes"], d["optics"], d["edges"])
    for k in ((0, 9) if (n, f) == (768, 6) else (9,)):
        x0, y0 = d["probes"][k]
        ref = O.prism_probe_direct(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f,
                                   amax, d["optics"], x0, y0, d["edges"])
        e = eps(D[k], ref)
        print(f"n={n} f={f} probe {k} prism eps_rel={e:.3e} (multislice {em:.3e})")
        assert e <= TOL
    assert em <= TOL
    if n // (2 * f) > 128:
        x0, y0 = d["probes"][9]
        C = G.probe_cbed(plan, f, amax, S, d["probes"][[9]], d["optics"])
        _, Cref = O.prism_probe_direct(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f,
                                       amax, d["optics"], x0, y0, d["edges"], return_cbed=True)
        e = eps(C[0], Cref)
        print(f"n={n} f={f} W={n // (2 * f)} cbed eps_rel={e:.3e}")
        assert e <= TOL


def test_window_12_cbed(m384):
    # the smallest window (W = 12: a radix-4 first row stage, then radix 3)
    d, plan = m384
    f = 16
    amax = _amax(d, f)
    S = G.build_smatrix(plan, f, amax)
    beams, Sref = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f, amax)
    C = G.probe_cbed(plan, f, amax, S, d["probes"], d["optics"])
    _, Cref = O.prism_outputs(Sref, beams, f, d["cell"], d["energy_keV"], d["optics"],
                              d["probes"], d["edges"], return_cbed=True)
    e = eps(C, Cref)
    print(f"n=384 f=16 W=12 cbed eps_rel={e:.3e}")
    assert e <= TOL


@pytest.mark.parametrize("case", ["mid384", "s512"])
def test_binning_slots_w192_w256(case):
    # The W = 144 .. 256 window kernels bin each element in registers, with
    # accumulator slots sized to the detector (4, 8, 16 or 32). A bin's sum
    # does not depend on how many bins there are, so 3, 6 and 12 bins equal
    # the first columns of the 32-bin outputs bit for bit; the first six
    # (overlapping) bins are also checked against the oracle, since PRISM at
    # f = 1 (W = 192 on 384^2, 256 on 512^2) is multislice.
    d = build_inputs(case, 0)
    plan = G.make_plan(d)
    f = 1
    amax = _amax(d, f)
    S = G.build_smatrix(plan, f, amax)
    pr = d["probes"][:6]
    edges = np.array([(5.0 * j, 5.0 * (j + 1) + (2.5 if j % 5 == 0 else 0.0))
                      for j in range(32)])
    D32 = G.probe_outputs(plan, f, amax, S, pr, d["optics"], edges)
    for k in (3, 6, 12):
        Dk = G.probe_outputs(plan, f, amax, S, pr, d["optics"], edges[:k])
        assert np.array_equal(Dk, D32[:, :k]), f"{k} bins differ from the 32-bin columns"
    ref = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"], d["optics"],
                            pr, edges[:6])
    e = eps(D32[:, :6], ref)
    print(f"{case} W={plan.n // 2} bin slots 4/8/16/32 equal; 6 bins eps_rel={e:.3e}")
    assert e <= TOL
