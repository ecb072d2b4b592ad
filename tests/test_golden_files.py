"""The committed full-size FP64 references (tests/golden/*_prism_f*.txt,
fcc1024_multislice.txt) against the inputs they name and against an
independent oracle route.

Each file comes from tests/golden/make_goldens.py (the oracle's full
S-matrix and probe step). Here a few of its rows are recomputed without any
S-matrix: by linearity of Eq. 5 the window sum of Eq. PRISMfinal equals the
window of the multislice exit wave of the periodised probe (the
``prism_probe_direct`` route, itself pinned in test_oracle_pins.py), and the
multislice rows by the oracle's multislice STEM.
"""
import numpy as np
import pytest

import oracle as O
from synth import build_inputs

import _golden as GD

FILES = [("fcc1024", 16), ("fcc1024", 8), ("fcc1024", 4), ("np2048", 8), ("np2048", 4)]


@pytest.fixture(scope="module")
def inputs():
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = build_inputs(name, 0)
        return cache[name]
    return get


@pytest.mark.parametrize("name,f", FILES)
def test_golden_file_matches_its_inputs(inputs, name, f):
    fn = f"{name}_prism_f{f}.txt"
    if not GD.exists(fn):
        pytest.skip(f"{fn} not generated")
    head, idx, xy, D = GD.load(fn)
    d = inputs(name)
    assert head["f"] == f
    lam = O.wavelength(d["energy_keV"])
    amax = O.default_alpha_max(d["optics"]["alpha_mrad"] * 1e-3, f, lam, 1.0 / d["cell"]) * 1e3
    assert abs(head["alpha_max_mrad"] - amax) <= 1e-12 * amax
    assert len(np.unique(idx)) == len(idx)
    assert np.array_equal(xy, d["probes"][idx])
    assert D.shape == (len(idx), len(d["edges"]))
    assert np.all(np.isfinite(D)) and np.all(D >= 0.0)


@pytest.mark.slow
@pytest.mark.parametrize("f,rows", [(16, (0, 77)), (8, (5,))])
def test_fcc1024_golden_rows_by_the_direct_route(inputs, f, rows):
    fn = f"fcc1024_prism_f{f}.txt"
    if not GD.exists(fn):
        pytest.skip(f"{fn} not generated")
    head, idx, xy, D = GD.load(fn)
    d = inputs("fcc1024")
    for r in rows:
        ref = O.prism_probe_direct(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f,
                                   head["alpha_max_mrad"], d["optics"], xy[r, 0], xy[r, 1],
                                   d["edges"])
        assert np.abs(ref - D[r]).max() <= 1e-10 * np.abs(ref).max(), r


@pytest.mark.slow
def test_fcc1024_multislice_golden_rows(inputs):
    if not GD.exists("fcc1024_multislice.txt"):
        pytest.skip("fcc1024_multislice.txt not generated")
    _, idx, xy, D = GD.load("fcc1024_multislice.txt")
    d = inputs("fcc1024")
    assert np.array_equal(xy, d["probes"][idx])
    ref = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"], d["optics"],
                            xy[:1], d["edges"])
    assert np.abs(ref[0] - D[0]).max() <= 1e-10 * np.abs(ref).max()
