"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

No GPU. Every test checks the oracle against something other than its own
formulas: brute-force DFTs, closed forms for an empty cell, physical
identities (propagation equals defocus, weak-phase contrast, translation),
exact linear-algebra identities of the PRISM construction, and values the
paper prints (Eq. TimeRatio worked example).
"""
import math
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle as O
from synth import build_inputs, phonon_configurations

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(v) for v in line.split()])
    return np.asarray(rows)


# ---------------------------------------------------------------- P1, P2

@pytest.mark.parametrize("n", [4, 6, 8, 12, 16])
def test_p1_fft_matches_dft_matrix(n):
    rng = np.random.default_rng(n)
    a = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    # explicit double sum, no matrices shared with the oracle's DftMatrix
    j = np.arange(n)
    ref = np.zeros((n, n), dtype=complex)
    for ky in range(n):
        for kx in range(n):
            ph = np.exp(-2j * np.pi * (ky * j[:, None] + kx * j[None, :]) / n)
            ref[ky, kx] = (a * ph).sum()
    for F in (O.ScipyFFT(workers=1), O.DftMatrix()):
        assert np.abs(F.fft2(a) - ref).max() <= 1e-13 * np.abs(ref).max()
        assert np.abs(F.ifft2(ref) - a).max() <= 1e-13 * np.abs(a).max()


def test_p2_sign_convention_peak_at_plus_m():
    n = 32
    for m, nn in [(3, 0), (0, 5), (-4, 7), (2, -9)]:
        psi = O.plane_wave(n, m, nn, 1)
        Psi = O.ScipyFFT(1).fft2(psi)
        ky, kx = np.unravel_index(np.argmax(np.abs(Psi)), Psi.shape)
        assert (kx, ky) == (m % n, nn % n)
        assert abs(abs(Psi[ky, kx]) - n * n) < 1e-9


# ---------------------------------------------------------------- constants

def test_wavelength_matches_tabulated_values():
    for kv, lam in _read_golden("electron_wavelengths.txt"):
        assert abs(O.wavelength(kv) - lam) < 0.6e-5


# ---------------------------------------------------------------- P3 empty cell, multislice

def _empty(n, H):
    return np.zeros((H, n, n)), np.full(H, 2.0)


def test_p3_empty_cell_detectors_are_aperture_fractions():
    n, cell, E, H = 128, 12.8, 80.0, 4
    phase, th = _empty(n, H)
    optics = dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0)
    edges = [(0.0, 21.0), (40.0, 150.0), (0.0, 10.0)]
    probes = np.array([[0.0, 0.0], [3.3, 7.1]])
    D = O.multislice_stem(phase, th, cell, E, optics, probes, edges)
    # independent brute-force count of aperture pixels by angle
    lam = O.wavelength(E)
    cnt_all = cnt_10 = 0
    for ky in range(-n // 2, n // 2):
        for kx in range(-n // 2, n // 2):
            th_k = lam * math.hypot(kx, ky) / cell
            if th_k <= 0.020 + 1e-15:
                cnt_all += 1
                cnt_10 += th_k < 0.010
    assert np.allclose(D[:, 0], 1.0, atol=1e-13)
    assert np.allclose(D[:, 1], 0.0, atol=1e-13)
    assert np.allclose(D[:, 2], cnt_10 / cnt_all, atol=1e-13)


def test_p3_propagation_equals_defocus():
    # Free-space propagation through thickness z is a defocus change of z:
    # exit(C1=0, C3) == entrance(C1=z, C3). A wrong relative sign between
    # the propagator and chi would match C1 = -z instead (C3 != 0 breaks
    # the +/- symmetry).
    n, cell, E, H = 64, 16.0, 80.0, 5
    phase, th = _empty(n, H)
    lam = O.wavelength(E)
    o0 = dict(alpha_mrad=25.0, C1_A=0.0, C3_A=2.0e5)
    psi0 = O.entrance_probe(n, cell, lam, o0, 5.0, 9.0)
    exit_ = O.multislice(psi0, phase, th, lam, 1.0 / cell)
    oz = dict(o0, C1_A=float(th.sum()))
    om = dict(o0, C1_A=-float(th.sum()))
    ref = O.entrance_probe(n, cell, lam, oz, 5.0, 9.0)
    wrong = O.entrance_probe(n, cell, lam, om, 5.0, 9.0)
    assert np.abs(exit_ - ref).max() < 1e-13
    assert np.abs(np.abs(exit_) ** 2 - np.abs(wrong) ** 2).max() > 1e-4


def test_entrance_probe_centred_on_r0_with_unit_intensity():
    n, cell, lam = 64, 12.8, O.wavelength(80.0)
    optics = dict(alpha_mrad=20.0)
    for (x0, y0) in [(0.0, 0.0), (4.0, 6.2), (11.8, 0.6)]:
        psi = O.entrance_probe(n, cell, lam, optics, x0, y0)
        iy, ix = np.unravel_index(np.argmax(np.abs(psi)), psi.shape)
        assert (ix, iy) == (round(x0 / (cell / n)) % n, round(y0 / (cell / n)) % n)
        assert abs((np.abs(psi) ** 2).sum() - 1.0) < 1e-13


def test_weak_phase_object_contrast_sign():
    # psi = exp(i eps cos(2 pi q0 x)) then Fresnel propagation over t gives
    # I = 1 + 2 eps sin(pi lambda q0^2 t) cos(2 pi q0 x) + O(eps^2).
    n, cell, t, E, eps, k0 = 64, 16.0, 50.0, 80.0, 1e-7, 5
    lam = O.wavelength(E)
    x = np.arange(n) * cell / n
    phi = np.broadcast_to(eps * np.cos(2 * np.pi * k0 * x / cell), (n, n))
    out = O.slice_step(np.ones((n, n), complex), O.transmission(phi),
                       O.propagator(n, lam, 1.0 / cell, t, band_limit=False))
    gamma = np.pi * lam * (k0 / cell) ** 2 * t
    ref = 1 + 2 * eps * np.sin(gamma) * np.cos(2 * np.pi * k0 * x / cell)
    assert np.abs(np.abs(out) ** 2 - ref[None, :]).max() < 1e-13
    assert abs(np.sin(gamma)) > 0.1


# ---------------------------------------------------------------- P4 empty cell, PRISM

@pytest.mark.parametrize("f", [1, 2, 4])
def test_p4_empty_cell_prism_closed_form(f):
    n, cell, E, H = 128, 12.8, 80.0, 3
    phase, th = _empty(n, H)
    lam = O.wavelength(E)
    optics = dict(alpha_mrad=20.0, C1_A=150.0, C3_A=1e4)
    amax = O.default_alpha_max(0.020, f, lam, 1 / cell) * 1e3
    beams, S = O.smatrix(phase, th, cell, E, f, amax)
    probes = np.array([[0.0, 0.0], [2.6, 5.0], [12.4, 0.2]])
    D, cbed = O.prism_outputs(S, beams, f, cell, E, optics, probes, [(0, 10), (10, 21)],
                              return_cbed=True)
    w = n // (2 * f)
    act = [(m, k) for m, k in beams if lam * math.hypot(m * f, k * f) / cell <= 0.020]
    ref = np.zeros((w, w))
    for m, k in act:
        ref[k % w, m % w] = 1.0 / len(act)
    for p in range(len(probes)):
        assert np.abs(cbed[p] - ref).max() < 1e-13
    assert np.allclose(D.sum(axis=1), 1.0, atol=1e-13)
    # each active beam lands in the detector bin of its own angle
    inner = sum(lam * math.hypot(m * f, k * f) / cell < 0.010 for m, k in act)
    assert np.allclose(D[:, 0], inner / len(act), atol=1e-13)
    assert 0 < inner < len(act)


def test_scherzer_defocus_fixes_c3_term():
    # Textbook Scherzer condition: with C1 = -sqrt(4 lambda C3 / 3) the
    # minimum of chi(q) over q is exactly -2 pi / 3. Both the q^4 power and
    # the pi/2 prefactor of the C3 term enter that value.
    lam, C3, dq = O.wavelength(200.0), 1.2e7, 1e-5
    C1 = -math.sqrt(4.0 * lam * C3 / 3.0)
    k = np.arange(0, 200000)
    chi = O.chi_of_k2(k.astype(np.int64) ** 2, lam, dq, C1, C3)
    assert abs(chi.min() + 2 * np.pi / 3) < 1e-6
    assert chi[0] == 0.0


# ---------------------------------------------------------------- P5 conservation

def test_p5_conservation_without_band_limit():
    d = build_inputs("tiny", 1)
    _, cbed = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"],
                                d["optics"], d["probes"][:3], [(0, 1)],
                                band_limit=False, return_cbed=True)
    assert np.abs(cbed.sum(axis=(1, 2)) - 1.0).max() < 1e-12


def test_p5_band_limit_never_increases_intensity():
    d = build_inputs("tiny", 2)
    lam = O.wavelength(d["energy_keV"])
    n, dq = d["n"], 1.0 / d["cell"]
    psi = O.entrance_probe(n, d["cell"], lam, d["optics"], 6.0, 6.0)
    prop = O.propagator(n, lam, dq, 2.0)
    last = (np.abs(psi) ** 2).sum()
    for p in range(d["phase"].shape[0]):
        psi = O.slice_step(psi, O.transmission(d["phase"][p]), prop)
        now = (np.abs(psi) ** 2).sum()
        assert now <= last + 1e-13
        last = now


def test_p5_smooth_weak_slices_conserve_with_band_limit():
    n, cell, E = 128, 12.8, 80.0
    x = np.arange(n) * cell / n
    X, Y = np.meshgrid(x, x)
    phase = np.stack([0.05 * np.cos(2 * np.pi * (X + 2 * Y) / cell + p) for p in range(4)])
    _, cbed = O.multislice_stem(phase, np.full(4, 2.0), cell, E, dict(alpha_mrad=20.0),
                                np.array([[1.0, 2.0]]), [(0, 1)], return_cbed=True)
    assert abs(cbed.sum() - 1.0) < 1e-12


# ---------------------------------------------------------------- P6 PRISM f=1 == multislice

def test_p6_prism_f1_equals_multislice():
    d = build_inputs("tiny", 0)
    lam = O.wavelength(d["energy_keV"])
    optics = dict(alpha_mrad=20.0, C1_A=30.0, C3_A=0.0)
    probes = d["probes"][::17]
    Dm = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"],
                           optics, probes, d["edges"])
    amax = O.default_alpha_max(0.020, 1, lam, 1 / d["cell"]) * 1e3
    beams, S = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], 1, amax)
    k2 = beams[:, 0] ** 2 + beams[:, 1] ** 2
    assert int(O.aperture_of_k2(k2, lam, 1 / d["cell"], 0.020).sum()) == 121
    Dp = O.prism_outputs(S, beams, 1, d["cell"], d["energy_keV"], optics, probes, d["edges"])
    assert O.rel_l2(Dp, Dm) < 1e-12


# ---------------------------------------------------------------- probe tilt

def _tilted(optics, tx, ty):
    return dict(optics, tilt_x_mrad=tx, tilt_y_mrad=ty)


def test_tilt_empty_cell_detectors_are_shifted_aperture_fractions():
    n, cell, E, H = 128, 12.8, 80.0, 3
    phase, th = _empty(n, H)
    lam = O.wavelength(E)
    tx, ty = 7.3, -4.1
    optics = _tilted(dict(alpha_mrad=20.0, C1_A=40.0, C3_A=1e4), tx, ty)
    edges = [(0.0, 10.0), (10.0, 20.0), (20.0, 40.0)]
    D = O.multislice_stem(phase, th, cell, E, optics, np.array([[3.0, 5.5]]), edges)
    # brute force: aperture centred on the tilt, pixels binned by their own angle
    cnt = np.zeros(3)
    na = 0
    for ky in range(-n // 2, n // 2):
        for kx in range(-n // 2, n // 2):
            if math.hypot(lam * kx / cell - tx * 1e-3, lam * ky / cell - ty * 1e-3) <= 0.020:
                na += 1
                a = lam * math.hypot(kx, ky) / cell * 1e3
                cnt += [lo <= a < hi for lo, hi in edges]
    assert np.allclose(D[0], cnt / na, atol=1e-12)
    assert cnt[2] > 0  # the tilt pushes part of the disc beyond 20 mrad


def test_tilt_by_whole_pixels_rolls_the_diffraction_pattern():
    # a tilt of exactly (3, -2) Fourier pixels shifts |Psi(k)|^2 by (3, -2)
    n, cell, E, H = 64, 12.8, 80.0, 2
    phase, th = _empty(n, H)
    lam = O.wavelength(E)
    lq = lam / cell
    o0 = dict(alpha_mrad=15.5, C1_A=25.0, C3_A=3e4)
    ot = _tilted(o0, 3 * lq * 1e3, -2 * lq * 1e3)
    _, c0 = O.multislice_stem(phase, th, cell, E, o0, np.array([[6.0, 6.0]]), [(0, 1)],
                              return_cbed=True)
    _, ct = O.multislice_stem(phase, th, cell, E, ot, np.array([[6.0, 6.0]]), [(0, 1)],
                              return_cbed=True)
    assert np.abs(np.roll(np.roll(c0[0], -2, axis=0), 3, axis=1) - ct[0]).max() < 1e-13


def test_tilt_height_term_returns_exit_probe_to_r0():
    # a tilted probe drifts by about h theta through the specimen; the
    # coefficient equation's -h tan(theta) entrance offset brings the exit
    # probe back to r0 (a sign error would leave it 2 h theta away)
    n, cell, E, H = 256, 25.6, 80.0, 10
    phase = np.zeros((H, n, n))
    th = np.full(H, 20.0)                    # h = 200 A
    lam = O.wavelength(E)
    optics = _tilted(dict(alpha_mrad=20.0), 8.0, -5.0)
    x0, y0 = 12.8, 12.8
    psi0 = O.entrance_probe(n, cell, lam, optics, x0, y0, height=float(th.sum()))
    ex = O.multislice(psi0, phase, th, lam, 1.0 / cell)
    I = np.abs(ex) ** 2
    x = np.arange(n) * cell / n
    m = (np.abs(x - x0) < 6.0)
    sub = I[np.ix_(m, m)]
    cx = (sub.sum(axis=0) * x[m]).sum() / sub.sum()
    cy = (sub.sum(axis=1) * x[m]).sum() / sub.sum()
    assert math.hypot(cx - x0, cy - y0) < 0.1
    # without the height term the exit probe sits about h theta away
    psi_no = O.entrance_probe(n, cell, lam, optics, x0, y0, height=0.0)
    I2 = np.abs(O.multislice(psi_no, phase, th, lam, 1.0 / cell)) ** 2
    sub2 = I2[np.ix_(m, m)]
    cx2 = (sub2.sum(axis=0) * x[m]).sum() / sub2.sum()
    assert abs(cx2 - x0 - 200.0 * 8e-3) < 0.2


def test_tilt_prism_f1_equals_multislice():
    d = build_inputs("tiny", 1)
    lam = O.wavelength(d["energy_keV"])
    optics = _tilted(dict(alpha_mrad=18.0, C1_A=-25.0, C3_A=0.0), 4.0, 2.5)
    probes = d["probes"][::23]
    Dm = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"],
                           optics, probes, d["edges"])
    amax = O.default_alpha_max(0.018 + math.hypot(4.0, 2.5) * 1e-3, 1, lam, 1 / d["cell"]) * 1e3
    beams, S = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], 1, amax)
    Dp = O.prism_outputs(S, beams, 1, d["cell"], d["energy_keV"], optics, probes, d["edges"],
                         height=float(np.sum(d["thickness"])))
    assert O.rel_l2(Dp, Dm) < 1e-12
    # the tilt matters: the untilted result differs
    Du = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"],
                           dict(optics, tilt_x_mrad=0.0, tilt_y_mrad=0.0), probes, d["edges"])
    assert O.rel_l2(Du, Dm) > 1e-3


# ---------------------------------------------------------------- P7 periodised-probe identity

@pytest.mark.parametrize("f", [2, 4])
def test_p7_prism_equals_cropped_multislice_of_periodised_probe(f):
    d = build_inputs("tiny", 3)
    n, cell, E = d["n"], d["cell"], d["energy_keV"]
    lam = O.wavelength(E)
    optics = dict(alpha_mrad=20.0, C1_A=-20.0, C3_A=0.0)
    amax = O.default_alpha_max(0.020, f, lam, 1 / cell) * 1e3
    beams, S = O.smatrix(d["phase"], d["thickness"], cell, E, f, amax)
    w = n // (2 * f)
    probes = np.array([[0.0, 0.0], [5.2, 9.6], [12.6, 3.0]])
    _, cbed = O.prism_outputs(S, beams, f, cell, E, optics, probes, [(0, 1)], return_cbed=True)
    for p, (x0, y0) in enumerate(probes):
        alpha, A = O.prism_coefficients(beams, f, cell, lam, optics, x0, y0)
        coef = alpha / (w * math.sqrt(A.sum()))
        psi0 = sum(c * O.plane_wave(n, m, k, f) for c, (m, k) in zip(coef, beams) if c != 0)
        ex = O.multislice(psi0, d["phase"], d["thickness"], lam, 1 / cell)[::2, ::2]
        # crop by rolling the window start to the origin (independent of window_indices)
        ds = 2 * cell / n
        cx = int(np.floor(x0 / ds + 0.5))
        cy = int(np.floor(y0 / ds + 0.5))
        win = np.roll(np.roll(ex, -(cy - w // 2), axis=0), -(cx - w // 2), axis=1)[:w, :w]
        I = np.abs(np.fft.fft2(win)) ** 2 / (w * w)
        assert np.abs(I - cbed[p]).max() < 1e-12 * max(1.0, I.max())


def test_p7_direct_single_probe_route_matches_prism_outputs():
    d = build_inputs("tiny", 6)
    cell, E, f = d["cell"], d["energy_keV"], 2
    lam = O.wavelength(E)
    optics = dict(alpha_mrad=20.0, C1_A=10.0, C3_A=2e4)
    amax = O.default_alpha_max(0.020, f, lam, 1 / cell) * 1e3
    beams, S = O.smatrix(d["phase"], d["thickness"], cell, E, f, amax)
    pr = np.array([[0.4, 12.6], [6.3, 6.5]])
    ref = O.prism_outputs(S, beams, f, cell, E, optics, pr, d["edges"])
    for p, (x0, y0) in enumerate(pr):
        got = O.prism_probe_direct(d["phase"], d["thickness"], cell, E, f, amax, optics, x0, y0,
                                   d["edges"])
        assert np.abs(got - ref[p]).max() <= 1e-12 * max(1.0, np.abs(ref).max())


# ---------------------------------------------------------------- P8 translation

def test_p8_multislice_one_pixel_shift():
    d = build_inputs("tiny", 4)
    n, cell = d["n"], d["cell"]
    dx = cell / n
    shifted = np.roll(d["phase"].astype(np.float64), 1, axis=2)
    pr = np.array([[1.6, 2.4], [7.2, 0.0]])
    D0 = O.multislice_stem(d["phase"], d["thickness"], cell, d["energy_keV"], d["optics"],
                           pr, d["edges"])
    D1 = O.multislice_stem(shifted, d["thickness"], cell, d["energy_keV"], d["optics"],
                           pr + [dx, 0.0], d["edges"])
    assert np.abs(D1 - D0).max() <= 1e-10 * np.abs(D0).max()


def test_p8_prism_two_pixel_shift():
    d = build_inputs("tiny", 5)
    n, cell, E, f = d["n"], d["cell"], d["energy_keV"], 2
    dx = cell / n
    lam = O.wavelength(E)
    amax = O.default_alpha_max(0.020, f, lam, 1 / cell) * 1e3
    shifted = np.roll(d["phase"].astype(np.float64), 2, axis=1)    # +2 fine pixels in y
    pr = np.array([[1.6, 2.4], [7.2, 0.0], [3.0, 11.8]])
    b0, S0 = O.smatrix(d["phase"], d["thickness"], cell, E, f, amax)
    b1, S1 = O.smatrix(shifted, d["thickness"], cell, E, f, amax)
    D0 = O.prism_outputs(S0, b0, f, cell, E, d["optics"], pr, d["edges"])
    D1 = O.prism_outputs(S1, b1, f, cell, E, d["optics"], pr + [0.0, 2 * dx], d["edges"])
    assert np.abs(D1 - D0).max() <= 1e-10 * np.abs(D0).max()


def test_p6_prism_f1_equals_multislice_on_a_3x2k_grid():
    # the same identity on a grid with a factor 3 (192 = 3 * 64), the oracle's
    # FFTs being mixed radix there
    d = build_inputs("tiny192", 1)
    cell, E = d["cell"], d["energy_keV"]
    lam = O.wavelength(E)
    amax = O.default_alpha_max(0.020, 1, lam, 1 / cell) * 1e3
    pr = d["probes"][::29]
    beams, S = O.smatrix(d["phase"], d["thickness"], cell, E, 1, amax)
    Dp = O.prism_outputs(S, beams, 1, cell, E, d["optics"], pr, d["edges"])
    Dm = O.multislice_stem(d["phase"], d["thickness"], cell, E, d["optics"], pr, d["edges"])
    assert O.rel_l2(Dp, Dm) < 1e-12


# ---------------------------------------------------------------- frozen phonons

def test_frozen_phonon_prism_f1_equals_multislice_average():
    # per configuration PRISM f = 1 is multislice (P6), so the averages agree
    d = phonon_configurations("tiny", 2, 3)
    cell, E = d["cell"], d["energy_keV"]
    lam = O.wavelength(E)
    amax = O.default_alpha_max(0.020, 1, lam, 1 / cell) * 1e3
    pr = d["probes"][::37]
    Dp = O.frozen_phonon_prism(d["phase_configs"], d["thickness"], cell, E, 1, amax, d["optics"],
                               pr, d["edges"])
    Dm = O.frozen_phonon_multislice(d["phase_configs"], d["thickness"], cell, E, d["optics"], pr,
                                    d["edges"])
    assert O.rel_l2(Dp, Dm) < 1e-12
    # the configurations differ, so the average is not any single one
    D0 = O.multislice_stem(d["phase_configs"][0], d["thickness"], cell, E, d["optics"], pr,
                           d["edges"])
    assert O.rel_l2(D0, Dm) > 1e-4


def test_frozen_phonon_prism_mean_of_translated_configurations():
    # configuration B is configuration A moved by one S-pixel (2 fine pixels),
    # so its image at r equals A's at r - s (P8); the incoherent mean is then
    # (D_A(r) + D_A(r - s)) / 2, computed from A's S-matrix alone
    d = build_inputs("tiny", 8)
    n, cell, E, f = d["n"], d["cell"], d["energy_keV"], 2
    dx = cell / n
    lam = O.wavelength(E)
    amax = O.default_alpha_max(0.020, f, lam, 1 / cell) * 1e3
    A = d["phase"].astype(np.float64)
    B = np.roll(A, 2, axis=2)                       # +2 fine pixels in x
    pr = np.array([[1.6, 2.4], [7.2, 0.0], [3.0, 11.8], [12.4, 6.6]])
    D, C = O.frozen_phonon_prism([A, B], d["thickness"], cell, E, f, amax, d["optics"], pr,
                                 d["edges"], return_cbed=True)
    bA, SA = O.smatrix(A, d["thickness"], cell, E, f, amax)
    D0, C0 = O.prism_outputs(SA, bA, f, cell, E, d["optics"], pr, d["edges"], return_cbed=True)
    D1, C1 = O.prism_outputs(SA, bA, f, cell, E, d["optics"], pr - [2 * dx, 0.0], d["edges"],
                             return_cbed=True)
    assert np.abs(D - 0.5 * (D0 + D1)).max() <= 1e-10 * np.abs(D).max()
    assert np.abs(C - 0.5 * (C0 + C1)).max() <= 1e-10 * np.abs(C).max()
    assert np.abs(D1 - D0).max() > 1e-3 * np.abs(D0).max()   # the two terms differ


def test_frozen_phonon_multislice_mean_of_translated_configurations():
    d = build_inputs("tiny", 9)
    n, cell, E = d["n"], d["cell"], d["energy_keV"]
    dx = cell / n
    A = d["phase"].astype(np.float64)
    B = np.roll(A, 1, axis=1)                       # +1 fine pixel in y
    pr = np.array([[1.6, 2.4], [7.2, 0.0], [3.0, 11.8]])
    D = O.frozen_phonon_multislice([A, B], d["thickness"], cell, E, d["optics"], pr, d["edges"])
    D0 = O.multislice_stem(A, d["thickness"], cell, E, d["optics"], pr, d["edges"])
    D1 = O.multislice_stem(A, d["thickness"], cell, E, d["optics"], pr - [0.0, dx], d["edges"])
    assert np.abs(D - 0.5 * (D0 + D1)).max() <= 1e-10 * np.abs(D).max()


# ---------------------------------------------------------------- P9 tiny brute force

@pytest.mark.parametrize("n", [8, 12])
def test_p9_dft_matrix_oracle_agrees(n):
    rng = np.random.default_rng(n)
    cell, E, H = n * 0.25, 80.0, 2
    phase = rng.uniform(0, 0.8, size=(H, n, n))
    th = np.full(H, 2.0)
    # aperture inside the half-band limit, so f = 1 PRISM uses the same waves
    optics = dict(alpha_mrad=35.0, C1_A=3.0, C3_A=0.0)
    probes = np.array([[0.0, 0.0], [0.75, 1.25]])
    edges = [(0, 20), (20, 2000)]
    Dm_f = O.multislice_stem(phase, th, cell, E, optics, probes, edges)
    Dm_d = O.multislice_stem(phase, th, cell, E, optics, probes, edges, fft=O.DftMatrix())
    assert np.abs(Dm_f - Dm_d).max() < 1e-13
    lam = O.wavelength(E)
    for f in (1, 2):
        if n % (2 * f):
            continue
        amax = O.default_alpha_max(0.035, f, lam, 1 / cell) * 1e3
        b, S = O.smatrix(phase, th, cell, E, f, amax)
        b2, S2 = O.smatrix(phase, th, cell, E, f, amax, fft=O.DftMatrix())
        assert np.abs(S - S2).max() < 1e-13
        Dp = O.prism_outputs(S, b, f, cell, E, optics, probes, edges)
        Dp2 = O.prism_outputs(S2, b2, f, cell, E, optics, probes, edges, fft=O.DftMatrix())
        assert np.abs(Dp - Dp2).max() < 1e-13
        if f == 1:
            assert np.abs(Dp - Dm_f).max() < 1e-13


def test_p9_bloch_form_full_smatrix_n8():
    # Eq. 2: the exit wave is a fixed linear map of the entrance wave. Build
    # that map column by column from every Fourier basis wave, then apply it
    # to a probe and compare with a direct multislice run.
    n, cell, E, H = 8, 2.0, 80.0, 3
    rng = np.random.default_rng(7)
    phase = rng.uniform(0, 1.0, size=(H, n, n))
    th = np.full(H, 2.0)
    lam = O.wavelength(E)
    cols = []
    for ky in range(n):
        for kx in range(n):
            basis = O.plane_wave(n, kx, ky, 1)
            cols.append(O.multislice(basis, phase, th, lam, 1 / cell).ravel())
    Smat = np.stack(cols, axis=1)                     # [pixel][k]
    psi0 = O.entrance_probe(n, cell, lam, dict(alpha_mrad=400.0, C1_A=1.0), 0.5, 0.75)
    coef = np.fft.fft2(psi0).ravel() / (n * n)        # psi0 = sum_k coef_k e^{2 pi i k r / n}
    direct = O.multislice(psi0, phase, th, lam, 1 / cell).ravel()
    assert np.abs(Smat @ coef - direct).max() < 1e-13


# ---------------------------------------------------------------- P10 beam set

def _brute_beams(n, cell, lam, f, amax):
    out = set()
    R = n  # generous search range
    for m in range(-R, R + 1):
        for k in range(-R, R + 1):
            if math.sqrt(m * m + k * k) * f * lam / cell <= amax * (1 + 1e-15) and \
                    (m * f) ** 2 + (k * f) ** 2 < (n / 4) ** 2:
                out.add((m, k))
    return out


@pytest.mark.parametrize("name,f,count", [("tiny", 1, 161), ("tiny", 2, 49),
                                          ("fcc1024", 4, 373), ("fcc1024", 8, 109),
                                          ("fcc1024", 16, 37)])
def test_p10_beam_count_matches_brute_force(name, f, count):
    from synth import get_config
    cfg = get_config(name)
    n, cell = cfg["n"], cfg["specimen"]["cell"][0]
    lam = O.wavelength(cfg["energy_keV"])
    amax = O.default_alpha_max(cfg["optics"]["alpha_mrad"] * 1e-3, f, lam, 1 / cell)
    b = O.beam_set(n, cell, lam, f, amax)
    assert len(b) == count
    assert set(map(tuple, b.tolist())) == _brute_beams(n, cell, lam, f, amax)
    assert len(set(map(tuple, b.tolist()))) == len(b)
    assert [tuple(x) for x in b.tolist()] == sorted(tuple(x) for x in b.tolist())


@settings(max_examples=25, deadline=None)
@given(st.integers(3, 9).map(lambda e: 2 ** e), st.sampled_from([1, 2, 4]),
       st.floats(5.0, 60.0))
def test_p10_beam_set_properties(n, f, alpha_mrad):
    if n % (2 * f) or n < 16:
        return
    cell = n * 0.1
    lam = O.wavelength(80.0)
    a = alpha_mrad * 1e-3
    b = O.beam_set(n, cell, lam, f, O.default_alpha_max(a, f, lam, 1 / cell))
    s = set(map(tuple, b.tolist()))
    assert all((-m, -k) in s for m, k in s)           # inversion symmetry
    assert (0, 0) in s
    b2 = O.beam_set(n, cell, lam, f, O.default_alpha_max(a * 1.3, f, lam, 1 / cell))
    assert s <= set(map(tuple, b2.tolist()))          # monotone in alpha_max


# ---------------------------------------------------------------- P11 cost model

def test_p11_cost_model_reproduces_printed_speedups():
    rows = _read_golden("cost_model_speedups.txt")
    exact = {2: 0.5055, 4: 7.793, 8: 108.79, 16: 1152.8}
    for f, printed in rows:
        r = O.time_ratio(40, 1e5, 1e4, int(f))
        assert abs(r - exact[int(f)]) / exact[int(f)] < 1e-3
        assert abs(r - printed) / printed < 0.06          # "approximately" in the text


def test_p11_ratio_is_quotient_of_large_n_forms():
    # Eq. TimeRatio equals 2 H P N^2 divided by B N^2 (2H/f^2 + P/(4 f^4)).
    for H, P, B, f in [(40, 1e5, 1e4, 4), (50, 65536, 305, 8), (10, 100, 7, 3)]:
        N = 1024
        ratio = (2 * H * P * N * N) / (B * N * N * (2 * H / f ** 2 + P / (4 * f ** 4)))
        assert abs(O.time_ratio(H, P, B, f) / ratio - 1) < 1e-12
        # the exact forms converge to it as N grows
        big = O.t_multi(H, P, 2 ** 40) / O.t_prism(H, P, 2 ** 40, B, f)
        assert abs(big / ratio - 1) < 1e-9


# ---------------------------------------------------------------- metrics

def test_error_metrics():
    a = np.array([1.0, 2.0, 3.0, 4.0])
    assert O.rel_l2(a, a) == 0.0
    assert abs(O.rel_l2(2 * a, a) - 1.0) < 1e-15
    assert abs(O.one_minus_r2(a, 3 * a + 1)) < 1e-15
    assert O.one_minus_r2(a, a[::-1]) == pytest.approx(0.0, abs=1e-15)


# ---------------------------------------------------------------- detectors

def test_detector_bins_are_half_open_and_additive():
    # A detector bin [inner, outer) counts every pixel whose scattering angle
    # lies in it (the annular detectors of the probe-output step): adjacent
    # bins add up to their union, a bin reaching past every angle holds the
    # whole pattern, inner == outer holds nothing, overlapping bins are summed
    # independently, and a pixel exactly on an edge goes to the upper bin.
    rng = np.random.default_rng(7)
    inten = rng.random((3, 9, 9))
    theta = np.abs(rng.normal(0.0, 0.05, (9, 9)))
    theta[4, 4] = 0.02  # exactly on the 20 mrad edge
    D = O.detector_sums(inten, theta, [(0, 20), (20, 60), (0, 60), (10, 30), (30, 30),
                                       (0, 1e9), (20, 20.000001)])
    assert np.allclose(D[:, 0] + D[:, 1], D[:, 2], rtol=1e-13, atol=0)
    assert np.allclose(D[:, 5], inten.sum(axis=(1, 2)), rtol=1e-13, atol=0)
    assert np.all(D[:, 4] == 0.0)
    brute = [sum(inten[p, i, j] for i in range(9) for j in range(9) if 0.01 <= theta[i, j] < 0.03)
             for p in range(3)]
    assert np.allclose(D[:, 3], brute, rtol=1e-13, atol=0)
    assert np.allclose(D[:, 6], inten[:, 4, 4], rtol=0, atol=0)


def test_window_bounds_worked_cases():
    # Eq. RegionBounds on an n_S = 16 grid with 0.5 A S-pixels and W = 4: the
    # centre pixel is the nearest S-pixel (halves round up), the window runs
    # from centre - W/2 for W pixels, and both wrap with the cell
    cases = [(0.0, [14, 15, 0, 1]), (0.74, [15, 0, 1, 2]), (0.75, [0, 1, 2, 3]),
             (-0.3, [13, 14, 15, 0]), (7.8, [14, 15, 0, 1]), (8.0 + 0.74, [15, 0, 1, 2])]
    for x0, want in cases:
        assert list(O.window_indices(x0, 16, 4, 0.5)) == want, x0
    # a 3 * 2^k width: W = 24 on n_S = 48
    assert list(O.window_indices(0.0, 48, 24, 1.0)) == list(range(36, 48)) + list(range(0, 12))
