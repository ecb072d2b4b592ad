"""Plain FP64 oracle of multislice STEM and of the PRISM algorithm.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing in the
product path may import this module.

Source: C. Ophus, "A Fast Image Simulation Algorithm for Scanning
Transmission Electron Microscopy" (arXiv:1702.01904). Each function names
the section or equation it follows. Everything is complex128 / float64,
FFTs come from ``scipy.fft`` (or, for brute-force checks, from explicit DFT
matrices passed in as ``fft=DftMatrix()``).

Conventions (fixed here because the paper leaves them implicit):
  * arrays are indexed [y][x]; pixel (i, j) sits at (i dx, j dx), dx = d/n;
  * integer frequencies k run over fftfreq order, q = k dq with dq = 1/d;
  * the forward FFT uses exp(-2 pi i k x / n) and is unnormalised, the
    inverse carries 1/n per axis (NumPy convention);
  * scattering angle of a full-grid frequency k is
    theta = (lambda * dq) * sqrt(kx^2 + ky^2), evaluated in that order;
  * the anti-aliasing aperture keeps kx^2 + ky^2 < (n/4)^2 (half the
    maximum frequency, strict), applied with the propagator every slice.
"""
import math
import os

import numpy as np
import scipy.fft as sfft

__all__ = [
    "HC_KEV_A", "ME_C2_KEV", "wavelength", "kfreq", "k2_grid", "theta_of_k2",
    "tilt_k", "tilted_k2", "tilt_shift",
    "band_mask", "propagator", "transmission", "aperture_of_k2", "chi_of_k2",
    "detector_sums", "ScipyFFT", "DftMatrix", "slice_step", "multislice",
    "entrance_probe", "multislice_stem", "default_alpha_max", "beam_set",
    "plane_wave", "smatrix", "window_origin", "window_indices",
    "prism_coefficients", "prism_probe_wave", "prism_outputs", "prism_probe_direct",
    "frozen_phonon_multislice", "frozen_phonon_prism",
    "t_multi", "t_prism", "time_ratio", "rel_l2", "one_minus_r2",
]

# Physical constants (CODATA 2018).
HC_KEV_A = 12.398419843320026      # h c in keV * Angstrom
ME_C2_KEV = 510.99895000           # electron rest energy m_e c^2 in keV


def wavelength(energy_keV):
    """Relativistic electron wavelength lambda (A) of Eq. 1.

    lambda = h c / sqrt(E (E + 2 m_e c^2)) for kinetic energy E.
    """
    E = float(energy_keV)
    return HC_KEV_A / math.sqrt(E * (E + 2.0 * ME_C2_KEV))


# --------------------------------------------------------------------------
# Grids and Fourier-space functions (Eqs. 3-5, aperture and chi equations)
# --------------------------------------------------------------------------

def kfreq(n):
    """Integer frequencies of an n-point FFT in fftfreq order."""
    return np.rint(np.fft.fftfreq(n) * n).astype(np.int64)


def k2_grid(n, scale=1):
    """Integer |k|^2 on an n x n grid indexed [ky][kx]; k multiplied by ``scale``."""
    k = kfreq(n) * int(scale)
    return k[:, None] ** 2 + k[None, :] ** 2


def theta_of_k2(k2, lam, dq):
    """Scattering angle (rad) of integer full-grid |k|^2 (small-angle theta = lambda |q|)."""
    return (lam * dq) * np.sqrt(np.asarray(k2, dtype=np.float64))


def band_mask(n, enabled=True):
    """Anti-aliasing aperture at half the maximum frequency (compact S-matrix paragraph)."""
    if not enabled:
        return np.ones((n, n), dtype=bool)
    return 16 * k2_grid(n) < n * n


def propagator(n, lam, dq, t, band_limit=True):
    """Fresnel propagator of Eq. 3 over thickness t, times the band limit."""
    q2 = k2_grid(n).astype(np.float64) * (dq * dq)
    return np.exp(-1j * np.pi * lam * q2 * t) * band_mask(n, band_limit)


def transmission(phase):
    """Transmission function of Eq. 4, exp(i sigma V_p), from the phase sigma V_p."""
    return np.exp(1j * np.asarray(phase, dtype=np.float64))


def aperture_of_k2(k2, lam, dq, alpha_rad):
    """Hard probe aperture A(q): 1 where lambda |q| <= alpha, else 0."""
    return theta_of_k2(k2, lam, dq) <= alpha_rad


def chi_of_k2(k2, lam, dq, C1, C3):
    """Aberration phase chi(q) = pi lambda q^2 C1 + (pi/2) lambda^3 q^4 C3."""
    q2 = np.asarray(k2, dtype=np.float64) * (dq * dq)
    return np.pi * lam * q2 * C1 + 0.5 * np.pi * lam ** 3 * q2 * q2 * C3


def tilt_k(optics, lam, dq):
    """Probe tilt as a full-grid frequency offset (kx_t, ky_t) = theta_t / (lambda dq).

    The tilted probe's aperture and aberrations are centred on q_t = theta_t /
    lambda (the paper's closing discussion: the probe centre moves away from
    q = 0). ``optics`` keys ``tilt_x_mrad``, ``tilt_y_mrad`` (default 0).
    """
    lq = lam * dq
    return (optics.get("tilt_x_mrad", 0.0) * 1e-3 / lq, optics.get("tilt_y_mrad", 0.0) * 1e-3 / lq)


def tilted_k2(kx, ky, optics, lam, dq):
    """|k - k_t|^2 (float64) for integer full-grid frequencies kx, ky."""
    ktx, kty = tilt_k(optics, lam, dq)
    dx = np.asarray(kx, dtype=np.float64) - ktx
    dy = np.asarray(ky, dtype=np.float64) - kty
    return dx * dx + dy * dy


def tilt_shift(optics, height):
    """Entrance-position offset h tan(theta_t) of the coefficient equation (Angstrom)."""
    return (height * math.tan(optics.get("tilt_x_mrad", 0.0) * 1e-3),
            height * math.tan(optics.get("tilt_y_mrad", 0.0) * 1e-3))


def detector_sums(intensity, theta, edges_mrad):
    """Virtual annular detectors: sum of intensity with inner <= theta < outer.

    ``intensity`` has shape [..., ny, nx]; returns [..., n_det] float64.
    """
    edges = np.asarray(edges_mrad, dtype=np.float64).reshape(-1, 2) * 1e-3
    out = np.empty(intensity.shape[:-2] + (edges.shape[0],), dtype=np.float64)
    for j, (lo, hi) in enumerate(edges):
        m = (theta >= lo) & (theta < hi)
        out[..., j] = (intensity * m).sum(axis=(-2, -1))
    return out


# --------------------------------------------------------------------------
# FFT primitives
# --------------------------------------------------------------------------

class ScipyFFT:
    """2D FFT pair on the last two axes (pocketfft via scipy)."""

    def __init__(self, workers=None):
        self.workers = workers if workers is not None else (os.cpu_count() or 1)

    def fft2(self, a):
        return sfft.fft2(a, axes=(-2, -1), workers=self.workers)

    def ifft2(self, a):
        return sfft.ifft2(a, axes=(-2, -1), workers=self.workers)


class DftMatrix:
    """2D DFT by explicit O(n^2) matrices (brute force, for tiny grids)."""

    @staticmethod
    def _mat(n, sign):
        j = np.arange(n)
        return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)

    def fft2(self, a):
        ny, nx = a.shape[-2:]
        return self._mat(ny, -1) @ a @ self._mat(nx, -1).T

    def ifft2(self, a):
        ny, nx = a.shape[-2:]
        return (self._mat(ny, 1) @ a @ self._mat(nx, 1).T) / (nx * ny)


_DEFAULT_FFT = None


def _fft(fft):
    global _DEFAULT_FFT
    if fft is not None:
        return fft
    if _DEFAULT_FFT is None:
        _DEFAULT_FFT = ScipyFFT()
    return _DEFAULT_FFT


# --------------------------------------------------------------------------
# Multislice (Eqs. 3-5)
# --------------------------------------------------------------------------

def slice_step(psi, trans_p, prop_p, fft=None):
    """One multislice step, Eq. 5: iFFT{ FFT{psi t_p} P_p }."""
    F = _fft(fft)
    return F.ifft2(F.fft2(psi * trans_p) * prop_p)


def multislice(psi, phase, thickness, lam, dq, band_limit=True, fft=None):
    """Apply Eq. 5 for every slice p = 0 .. H-1 (the last step propagates to the exit face)."""
    n = psi.shape[-1]
    props = {}
    for p in range(phase.shape[0]):
        t = float(thickness[p])
        if t not in props:
            props[t] = propagator(n, lam, dq, t, band_limit)
        psi = slice_step(psi, transmission(phase[p]), props[t], fft)
    return psi


def entrance_probe(n, cell, lam, optics, x0, y0, fft=None, height=0.0):
    """Incident STEM probe on the full grid, normalised to unit total intensity.

    Psi_0(q) = A(q - q_t) exp(-i chi(q - q_t)) exp(-2 pi i q . (r0 - h tan theta_t));
    psi_0 = iFFT(Psi_0) n / sqrt(N_A). Without tilt this is the untilted probe
    centred on r0; ``height`` h is the specimen thickness (coefficient equation).
    """
    F = _fft(fft)
    dq = 1.0 / cell
    k = kfreq(n)
    dk2 = tilted_k2(k[None, :], k[:, None], optics, lam, dq)
    A = aperture_of_k2(dk2, lam, dq, optics["alpha_mrad"] * 1e-3)
    NA = int(A.sum())
    chi = chi_of_k2(dk2, lam, dq, optics.get("C1_A", 0.0), optics.get("C3_A", 0.0))
    sx, sy = tilt_shift(optics, height)
    x0, y0 = x0 - sx, y0 - sy
    shift = np.exp(-2j * np.pi * (k[None, :] * x0 + k[:, None] * y0) * dq)
    Psi0 = A * np.exp(-1j * chi) * shift
    return F.ifft2(Psi0) * (n / math.sqrt(NA))


def multislice_stem(phase, thickness, cell, energy_keV, optics, probes, edges_mrad,
                    band_limit=True, fft=None, batch=16, return_cbed=False):
    """Conventional multislice STEM: one full Eq. 5 run per probe position.

    Output per probe: I(k) = |FFT(psi_H)|^2 / n^2 summed over each detector.
    Returns float64 [P][n_det] (and the CBED stack [P][n][n] if asked).
    """
    F = _fft(fft)
    phase = np.asarray(phase, dtype=np.float64)
    n = phase.shape[-1]
    lam = wavelength(energy_keV)
    dq = 1.0 / cell
    theta = theta_of_k2(k2_grid(n), lam, dq)
    probes = np.asarray(probes, dtype=np.float64).reshape(-1, 2)
    P = probes.shape[0]
    out = np.zeros((P, np.asarray(edges_mrad).reshape(-1, 2).shape[0]))
    cbed = np.zeros((P, n, n)) if return_cbed else None
    for s in range(0, P, batch):
        pr = probes[s:s + batch]
        psi = np.stack([entrance_probe(n, cell, lam, optics, x0, y0, F, height=float(np.sum(thickness)))
                        for x0, y0 in pr])
        psi = multislice(psi, phase, thickness, lam, dq, band_limit, F)
        I = np.abs(F.fft2(psi)) ** 2 / float(n * n)
        out[s:s + len(pr)] = detector_sums(I, theta, edges_mrad)
        if return_cbed:
            cbed[s:s + len(pr)] = I
    return (out, cbed) if return_cbed else out


# --------------------------------------------------------------------------
# PRISM: beam set, compact S-matrix, coefficients, window sum (Fig. 1c-f)
# --------------------------------------------------------------------------

def default_alpha_max(alpha_rad, f, lam, dq):
    """alpha_max = largest probe semi-angle + f lambda dq (choice of alpha_max paragraph)."""
    return alpha_rad + f * (lam * dq)


def beam_set(n, cell, lam, f, alpha_max_rad):
    """Plane-wave indices (m, n) of the PRISM beam set, lexicographic order.

    Keeps sqrt(m^2+n^2) f lambda dq <= alpha_max (the plane-wave set
    equation) and, so that every beam survives the half-band aperture,
    (m f)^2 + (n f)^2 < (n/4)^2. Returns int64 [B][2].
    """
    dq = 1.0 / cell
    lim = n // (4 * f) + 1
    out = []
    for m in range(-lim, lim + 1):
        for nn in range(-lim, lim + 1):
            k2 = (m * f) ** 2 + (nn * f) ** 2
            if 16 * k2 >= n * n:
                continue
            if theta_of_k2(k2, lam, dq) <= alpha_max_rad:
                out.append((m, nn))
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


def plane_wave(n, m, nn, f):
    """Tilted plane wave exp(2 pi i (m f x + n f y) / d) on the n x n grid (exact phase index)."""
    i = np.arange(n, dtype=np.int64)
    idx = (m * f * i[None, :] + nn * f * i[:, None]) % n
    return np.exp(2j * np.pi * idx.astype(np.float64) / n)


def smatrix(phase, thickness, cell, energy_keV, f, alpha_max_mrad, fft=None,
            band_limit=True, beams=None):
    """Compact S-matrix: multislice of every beam, stored band-limited at 1/4 size.

    Each S_{m,n}(r) is the exit wave of plane wave (m, n), Fourier-cropped to
    k in [-n/4, n/4)^2 and inverse-transformed on the (n/2)^2 grid with the
    factor 1/4, so that S(i', j') equals the exit wave at fine pixel
    (2 i', 2 j'). Returns (beams int64 [B][2], S complex128 [B][n/2][n/2]).
    """
    F = _fft(fft)
    phase = np.asarray(phase, dtype=np.float64)
    n = phase.shape[-1]
    if n % (2 * f) or n % 4:
        raise ValueError("n must be divisible by 2 f and by 4")
    lam = wavelength(energy_keV)
    dq = 1.0 / cell
    if beams is None:
        beams = beam_set(n, cell, lam, f, alpha_max_mrad * 1e-3)
    ns = n // 2
    keep = np.concatenate([np.arange(0, n // 4), np.arange(n - n // 4, n)])
    S = np.empty((len(beams), ns, ns), dtype=np.complex128)
    for b, (m, nn) in enumerate(beams):
        psi = multislice(plane_wave(n, m, nn, f), phase, thickness, lam, dq, band_limit, F)
        Psi = F.fft2(psi)
        S[b] = 0.25 * F.ifft2(Psi[np.ix_(keep, keep)])
    return beams, S


def window_origin(x0, ns, w, dxs):
    """First S-pixel of the cut-out region of Eq. RegionBounds along one axis.

    The centre pixel is floor(x0 / dx_S + 1/2) mod n_S; the window covers
    centre - w//2 ... centre - w//2 + w - 1, wrapped periodically.
    """
    c = int(math.floor(x0 / dxs + 0.5)) % ns
    return (c - w // 2) % ns


def window_indices(x0, ns, w, dxs):
    return (window_origin(x0, ns, w, dxs) + np.arange(w)) % ns


def prism_coefficients(beams, f, cell, lam, optics, x0, y0, height=0.0):
    """Probe coefficients alpha_{m,n}(r0) (coefficient equation).

    alpha = A(q - q_t) exp(-i chi(q - q_t)) exp(-2 pi i q . (r0 - h tan theta_t))
    at q = (m f dq, n f dq) (q_t = 0 without tilt; ``height`` h is the
    specimen thickness). Returns (alpha complex128 [B], active bool [B]); the
    normalisation 1 / (W sqrt(B_A)) is applied through ``prism_probe_wave``.
    """
    dq = 1.0 / cell
    m = beams[:, 0].astype(np.float64)
    nn = beams[:, 1].astype(np.float64)
    dk2 = tilted_k2(beams[:, 0] * f, beams[:, 1] * f, optics, lam, dq)
    A = aperture_of_k2(dk2, lam, dq, optics["alpha_mrad"] * 1e-3)
    chi = chi_of_k2(dk2, lam, dq, optics.get("C1_A", 0.0), optics.get("C3_A", 0.0))
    sx, sy = tilt_shift(optics, height)
    shift = np.exp(-2j * np.pi * (m * f * (x0 - sx) + nn * f * (y0 - sy)) * dq)
    return A * np.exp(-1j * chi) * shift, A


def prism_probe_wave(S, beams, f, cell, lam, optics, x0, y0, height=0.0):
    """Eq. PRISMfinal inside the Eq. RegionBounds window; returns psi [W][W] (indexed [v][u])."""
    ns = S.shape[-1]
    w = ns // f
    dxs = cell / ns
    alpha, A = prism_coefficients(beams, f, cell, lam, optics, x0, y0, height)
    BA = int(A.sum())
    act = np.nonzero(A)[0]                       # beams with alpha = 0 are skipped
    rows = window_indices(y0, ns, w, dxs)
    cols = window_indices(x0, ns, w, dxs)
    win = S[np.ix_(act, rows, cols)]
    coef = alpha[act] / (w * math.sqrt(BA))
    return np.tensordot(coef, win, axes=(0, 0))


def prism_outputs(S, beams, f, cell, energy_keV, optics, probes, edges_mrad, fft=None,
                  return_cbed=False, height=0.0):
    """PRISM probe step: window sum, FFT, |Psi|^2 / W^2 and detector sums (Fig. 1d-f).

    The window's Fourier pixel is f dq, so window frequency kw maps to the
    full-grid frequency f kw for the detector angles. Returns float64 [P][n_det].
    """
    F = _fft(fft)
    lam = wavelength(energy_keV)
    dq = 1.0 / cell
    ns = S.shape[-1]
    w = ns // f
    theta = theta_of_k2(k2_grid(w, scale=f), lam, dq)
    probes = np.asarray(probes, dtype=np.float64).reshape(-1, 2)
    n_det = np.asarray(edges_mrad).reshape(-1, 2).shape[0]
    out = np.zeros((probes.shape[0], n_det))
    cbed = np.zeros((probes.shape[0], w, w)) if return_cbed else None
    for p, (x0, y0) in enumerate(probes):
        psi = prism_probe_wave(S, beams, f, cell, lam, optics, x0, y0, height)
        I = np.abs(F.fft2(psi)) ** 2 / float(w * w)
        out[p] = detector_sums(I, theta, edges_mrad)
        if return_cbed:
            cbed[p] = I
    return (out, cbed) if return_cbed else out


def prism_probe_direct(phase, thickness, cell, energy_keV, f, alpha_max_mrad, optics, x0, y0,
                       edges_mrad, fft=None, return_cbed=False):
    """PRISM output of one probe without forming the S-matrix.

    By linearity of Eq. 5, the window sum of Eq. PRISMfinal equals the window
    of the quarter-size exit wave of the periodised probe
    psi0 = sum_b alpha_b exp(2 pi i q_b . r). One multislice run per probe
    therefore gives PRISM's output exactly (identity checked against
    ``prism_outputs``); this is how single probes of large grids are sampled.
    Returns float64 [n_det] (and the window intensity [W][W] when
    ``return_cbed``).
    """
    F = _fft(fft)
    phase = np.asarray(phase, dtype=np.float64)
    n = phase.shape[-1]
    lam = wavelength(energy_keV)
    dq = 1.0 / cell
    beams = beam_set(n, cell, lam, f, alpha_max_mrad * 1e-3)
    ns = n // 2
    w = ns // f
    alpha, A = prism_coefficients(beams, f, cell, lam, optics, x0, y0,
                                  float(np.sum(thickness)))
    coef = alpha / (w * math.sqrt(int(A.sum())))
    psi0 = np.zeros((n, n), dtype=np.complex128)
    for c, (m, nn) in zip(coef, beams):
        if c != 0:
            psi0 += c * plane_wave(n, m, nn, f)
    exit_ = multislice(psi0, phase, thickness, lam, dq, True, F)[::2, ::2]
    dxs = cell / ns
    rows = window_indices(y0, ns, w, dxs)
    cols = window_indices(x0, ns, w, dxs)
    win = exit_[np.ix_(rows, cols)]
    I = np.abs(F.fft2(win)) ** 2 / float(w * w)
    theta = theta_of_k2(k2_grid(w, scale=f), lam, dq)
    D = detector_sums(I, theta, edges_mrad)
    return (D, I) if return_cbed else D


# --------------------------------------------------------------------------
# Frozen phonons ("Simulation and Analysis Implementation")
# --------------------------------------------------------------------------
# Thermal scattering: the whole simulation is repeated for K configurations
# of randomly displaced atoms and the intensities are added incoherently;
# the result reported here is their mean (sum / K).

def frozen_phonon_multislice(phase_configs, thickness, cell, energy_keV, optics, probes,
                             edges_mrad, fft=None, return_cbed=False):
    """Mean over configurations of multislice STEM outputs (detector sums, CBED)."""
    K = len(phase_configs)
    D, C = 0.0, 0.0
    for ph in phase_configs:
        r = multislice_stem(ph, thickness, cell, energy_keV, optics, probes, edges_mrad,
                            fft=fft, return_cbed=return_cbed)
        if return_cbed:
            D, C = D + r[0], C + r[1]
        else:
            D = D + r
    return (D / K, C / K) if return_cbed else D / K


def frozen_phonon_prism(phase_configs, thickness, cell, energy_keV, f, alpha_max_mrad, optics,
                        probes, edges_mrad, fft=None, return_cbed=False):
    """Mean over configurations of PRISM outputs, one S-matrix per configuration."""
    K = len(phase_configs)
    height = float(np.sum(thickness))
    D, C = 0.0, 0.0
    for ph in phase_configs:
        beams, S = smatrix(ph, thickness, cell, energy_keV, f, alpha_max_mrad, fft=fft)
        r = prism_outputs(S, beams, f, cell, energy_keV, optics, probes, edges_mrad, fft=fft,
                          return_cbed=return_cbed, height=height)
        if return_cbed:
            D, C = D + r[0], C + r[1]
        else:
            D = D + r
    return (D / K, C / K) if return_cbed else D / K


# --------------------------------------------------------------------------
# Cost model (Eqs. TimeMulti, TimePRISM, TimeRatio) and error metrics
# --------------------------------------------------------------------------

def t_multi(H, P, N):
    """Eq. TimeMulti, exact form: H P [6 N log2 N + 2 N^2]."""
    return H * P * (6 * N * math.log2(N) + 2 * N * N)


def t_prism(H, P, N, B, f):
    """Eq. TimePRISM, exact form: (H B / f^2)[6 N log2 N + 2 N^2] + P B N^2 / (4 f^4)."""
    return H * B / f ** 2 * (6 * N * math.log2(N) + 2 * N * N) + P * B * N * N / (4.0 * f ** 4)


def time_ratio(H, P, B, f):
    """Eq. TimeRatio: 8 H P f^4 / (B (8 H f^2 + P)) (large-N form)."""
    return 8.0 * H * P * f ** 4 / (B * (8.0 * H * f ** 2 + P))


def rel_l2(a, ref):
    """||a - ref||_2 / ||ref||_2 over all entries."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def one_minus_r2(a, b):
    """Error estimate 1 - R^2 between two images (Fig. 4e discussion), R the Pearson correlation."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    r = np.corrcoef(a, b)[0, 1]
    return float(1.0 - r * r)
