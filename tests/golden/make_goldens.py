#!/usr/bin/env python3
"""Write the FP64 reference outputs of the full-size workloads into tests/golden/.

Every value comes from the oracle (``oracle/``) on the seeded inputs of
``synth/``; nothing else is imported. The GPU parity tests and the benchmark
compare the library's outputs against these files probe by probe and bin by
bin.

  PRISM (Eq. PRISMfinal summed over the window of Eq. RegionBounds, then the
  window's |FFT|^2 / W^2 integrated over each detector bin): the whole
  compact S-matrix is built by the oracle (every beam of the set through all
  slices, Eq. 5, quarter-size storage), then the probe step runs on the
  chosen probes.
    fcc1024 (1024^2, 50 slices, 200 keV, 25 mrad, 16 bins): f = 4, 8, 16 on
      128 probes of the 256 x 256 scan: scan corners and edge midpoints
      (windows that wrap through the cell boundary), the four corners of
      seeded 8 x 8, 8 x 4 and 4 x 4 blocks of the raster, the first and last
      probes of 8-row bands, and seeded uniform picks.
    np2048 (2048^2 nanoparticle on carbon, 35 slices, 80 keV, 20 mrad,
      [40, 150) mrad): f = 4 and 8 on all 1024 sub-pixel probes.
  Multislice STEM (Eq. 5 once per probe): fcc1024 on 32 of the PRISM probes.

Usage: python tests/golden/make_goldens.py [--only fcc1024,np2048,multislice]
Takes about 2 hours on 8 cores (the np2048 S-matrices dominate).
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import build_inputs  # noqa: E402

SCAN = 256  # fcc1024 raster side


def fcc_probe_indices(seed=1702):
    """128 raster indices p = j * 256 + i of the fcc1024 scan, sorted."""
    rng = np.random.default_rng(seed)
    sel = []

    def add(i, j):
        p = (j % SCAN) * SCAN + (i % SCAN)
        if p not in sel:
            sel.append(p)

    for i, j in ((0, 0), (255, 0), (0, 255), (255, 255), (128, 0), (0, 128), (255, 128),
                 (128, 255)):
        add(i, j)
    for bx, by, count in ((8, 8, 6), (8, 4, 4), (4, 4, 6)):
        for _ in range(count):
            i0 = int(rng.integers(0, SCAN // bx)) * bx
            j0 = int(rng.integers(0, SCAN // by)) * by
            for di, dj in ((0, 0), (bx - 1, 0), (0, by - 1), (bx - 1, by - 1)):
                add(i0 + di, j0 + dj)
    for r in (0, 15, 31):
        add(255, 8 * r + 7)
        add(0, (8 * r + 8) % SCAN)
    while len(sel) < 128:
        add(int(rng.integers(0, SCAN)), int(rng.integers(0, SCAN)))
    return np.sort(np.asarray(sel[:128], dtype=np.int64))


def write(path, header, idx, xy, values):
    with open(path, "w") as fh:
        for line in header:
            fh.write("# " + line + "\n")
        for k in range(len(idx)):
            vals = " ".join(repr(float(v)) for v in np.atleast_1d(values[k]))
            fh.write(f"{int(idx[k])} {float(xy[k, 0])!r} {float(xy[k, 1])!r} {vals}\n")
    print(f"wrote {path} ({len(idx)} rows)", flush=True)


def amax_of(d, f):
    lam = O.wavelength(d["energy_keV"])
    return O.default_alpha_max(d["optics"]["alpha_mrad"] * 1e-3, f, lam, 1.0 / d["cell"]) * 1e3


def prism_goldens(name, f_values, idx, tag):
    d = build_inputs(name, 0)
    xy = d["probes"][idx]
    for f in f_values:
        amax = amax_of(d, f)
        t0 = time.time()
        beams, S = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f, amax)
        print(f"{name} f={f}: S-matrix of {len(beams)} beams in {time.time() - t0:.0f} s",
              flush=True)
        t0 = time.time()
        D = O.prism_outputs(S, beams, f, d["cell"], d["energy_keV"], d["optics"], xy, d["edges"],
                            height=float(np.sum(d["thickness"])))
        print(f"{name} f={f}: {len(idx)} probes in {time.time() - t0:.0f} s", flush=True)
        del S
        edges = ", ".join(f"[{lo:g}, {hi:g})" for lo, hi in d["edges"])
        header = [
            f"FP64 oracle, PRISM probe step: {name} seed 0, f = {f}, "
            f"alpha_max = {amax!r} mrad (alpha + f lambda dq), {len(beams)} beams",
            "Eq. PRISMfinal over the window of Eq. RegionBounds, |FFT_W psi|^2 / W^2 "
            "summed per detector bin (inner <= theta < outer)",
            f"bins (mrad): {edges}",
            f"probes: {tag}",
            "written by tests/golden/make_goldens.py from oracle/ and synth/ only",
            "columns: probe_index x_A y_A D_0 ... D_{n_det-1}",
        ]
        write(os.path.join(HERE, f"{name}_prism_f{f}.txt"), header, idx, xy, D)


def multislice_goldens(idx):
    d = build_inputs("fcc1024", 0)
    xy = d["probes"][idx]
    t0 = time.time()
    D = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"], d["optics"], xy,
                          d["edges"])
    print(f"fcc1024 multislice: {len(idx)} probes in {time.time() - t0:.0f} s", flush=True)
    header = [
        "FP64 oracle, multislice STEM: fcc1024 seed 0 (Eq. 5 once per probe, "
        "|FFT psi_H|^2 / n^2 summed per detector bin)",
        "probes: 32 of the PRISM golden probes (seeded pick)",
        "written by tests/golden/make_goldens.py from oracle/ and synth/ only",
        "columns: probe_index x_A y_A D_0 ... D_15",
    ]
    write(os.path.join(HERE, "fcc1024_multislice.txt"), header, idx, xy, D)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--only", default="fcc1024,multislice,np2048")
    args = ap.parse_args()
    parts = set(x.strip() for x in args.only.split(",") if x.strip())
    idx = fcc_probe_indices()
    if "fcc1024" in parts:
        prism_goldens("fcc1024", (16, 8, 4), idx,
                      "128 raster indices p = j * 256 + i (corners, edges, block corners, "
                      "band ends, seeded picks)")
    if "multislice" in parts:
        rng = np.random.default_rng(7)
        multislice_goldens(np.sort(rng.choice(idx, 32, replace=False)))
    if "np2048" in parts:
        prism_goldens("np2048", (8, 4), np.arange(1024),
                      "all 1024 seeded sub-pixel probes over the particle disc")


if __name__ == "__main__":
    main()
