"""Reader of the FP64 reference files under tests/golden/ (written by
tests/golden/make_goldens.py from the oracle alone) and the per-bin gates
the GPU parity tests apply to them."""
import os
import re

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    """(header dict, probe indices int64 [P], positions [P][2], values [P][n_det])."""
    path = os.path.join(GOLDEN, name)
    head = {}
    rows = []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                m = re.search(r"alpha_max = ([0-9.eE+-]+) mrad", line)
                if m:
                    head["alpha_max_mrad"] = float(m.group(1))
                m = re.search(r"f = (\d+),", line)
                if m:
                    head["f"] = int(m.group(1))
                continue
            if line.strip():
                rows.append([float(x) for x in line.split()])
    a = np.asarray(rows, dtype=np.float64)
    return head, a[:, 0].astype(np.int64), a[:, 1:3], a[:, 3:]


def exists(name):
    return os.path.exists(os.path.join(GOLDEN, name))


def per_bin(D, ref):
    """Per-bin eps_rel over the probes, and max |dD| (units of total probe intensity)."""
    D = np.asarray(D, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.linalg.norm(D - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    eps = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return eps, float(np.abs(D - ref).max())


def gate(D, ref, edges_mrad, half_band_mrad, tol, label, floor=None):
    """Gate the whole-array eps_rel and max |dD| (units of the probe's total
    intensity, which is 1) at ``tol``, and eps_rel per bin for the bins that
    lie entirely below the half-band angle and are not near-empty: their
    reference mean is at least ``floor`` of the probe's intensity (default
    1e-6 for tol <= 1e-4, else 1e-4). Near-empty bins, where the arithmetic's
    absolute error floor dominates a relative figure, and bins reaching past
    the half-band limit (crop leakage only in PRISM) are reported, not gated
    per bin. Returns the report string (all bins listed)."""
    assert np.all(np.isfinite(D)), label
    if floor is None:
        floor = 1e-6 if tol <= 1e-4 else 1e-4
    eps, dmax = per_bin(D, ref)
    edges = np.asarray(edges_mrad, dtype=np.float64).reshape(-1, 2)
    mean = np.abs(np.asarray(ref)).mean(axis=0)
    gated = (edges[:, 1] <= half_band_mrad) & (mean >= floor)
    whole = float(np.linalg.norm(D - ref) / np.linalg.norm(ref))
    rep = (f"{label}: eps_rel {whole:.2e}, max|dD| {dmax:.2e}, worst gated bin "
           f"{eps[gated].max():.2e}; per bin (eps_rel, mean, * = gated): " + " ".join(
               f"[{lo:g},{hi:g}){'*' if g else ''} {e:.1e} {m:.0e}"
               for (lo, hi), e, m, g in zip(edges, eps, mean, gated)))
    print(rep)
    assert whole <= tol, rep
    assert dmax <= tol, rep
    assert np.all(eps[gated] <= tol), rep
    return rep
