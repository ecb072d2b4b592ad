"""Frozen-phonon averaging on the GPU (the accumulating probe-step and
multislice calls) against the FP64 oracle's configuration means.

Each configuration of displaced atoms gets its own potential slices and its
own S-matrix; the outputs are summed incoherently with weight 1/K in the
output buffer. Gate: eps_rel <= 1e-4 (FP32 window sum), <= 1e-2 (BF16).
"""
import numpy as np
import pytest

import oracle as O
from synth import build_inputs, phonon_configurations

import _gpu as G

pytestmark = pytest.mark.gpu

TOL = 1e-4
TOL16 = 1e-2
K = 3


def eps(a, ref):
    a = np.asarray(a)
    ref = np.asarray(ref)
    assert np.all(np.isfinite(a))
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


def _amax(d, f, alpha_mrad=None):
    lam = O.wavelength(d["energy_keV"])
    a = (alpha_mrad if alpha_mrad is not None else d["optics"]["alpha_mrad"]) * 1e-3
    return O.default_alpha_max(a, f, lam, 1.0 / d["cell"]) * 1e3


@pytest.fixture(scope="module")
def phonons():
    d = phonon_configurations("tiny", 4, K)
    plan = G.make_plan(d)
    return d, plan


@pytest.mark.parametrize("f", [1, 2])
def test_frozen_phonon_prism_tiny(phonons, f):
    d, plan = phonons
    amax = _amax(d, f)
    pr = d["probes"][::5]
    D = G.frozen_phonon_prism(plan, f, amax, d["phase_configs"], pr, d["optics"], d["edges"])
    ref, Cref = O.frozen_phonon_prism(d["phase_configs"], d["thickness"], d["cell"],
                                      d["energy_keV"], f, amax, d["optics"], pr, d["edges"],
                                      return_cbed=True)
    e = eps(D, ref)
    print(f"frozen phonon prism tiny f={f} K={K} P={len(pr)} eps_rel={e:.3e}")
    assert e <= TOL
    C = G.frozen_phonon_prism(plan, f, amax, d["phase_configs"], pr, d["optics"], d["edges"],
                              cbed=True)
    e = eps(C, Cref)
    print(f"frozen phonon cbed tiny f={f} eps_rel={e:.3e}")
    assert e <= TOL


def test_frozen_phonon_multislice_tiny(phonons):
    d, plan = phonons
    pr = d["probes"][::11]
    D = G.frozen_phonon_multislice(plan, d["phase_configs"], pr, d["optics"], d["edges"])
    ref = O.frozen_phonon_multislice(d["phase_configs"], d["thickness"], d["cell"],
                                     d["energy_keV"], d["optics"], pr, d["edges"])
    e = eps(D, ref)
    print(f"frozen phonon multislice tiny K={K} P={len(pr)} eps_rel={e:.3e}")
    assert e <= TOL


def test_frozen_phonon_prism_tiny_bf16(phonons):
    d, plan = phonons
    f = 2
    amax = _amax(d, f)
    pr = d["probes"]
    plan.set_probe_precision("bf16")
    try:
        D = G.frozen_phonon_prism(plan, f, amax, d["phase_configs"], pr, d["optics"], d["edges"])
    finally:
        plan.set_probe_precision("fp32")
    ref = O.frozen_phonon_prism(d["phase_configs"], d["thickness"], d["cell"], d["energy_keV"],
                                f, amax, d["optics"], pr, d["edges"])
    e = eps(D, ref)
    print(f"frozen phonon prism tiny bf16 f={f} eps_rel={e:.3e}")
    assert e <= TOL16


def test_accumulate_splits_like_overwrite_w256():
    # W = 256 (two-pass window FFT, per-tile partials): out = 0.25 R + 0.75 R
    # through two accumulating calls equals the overwriting call's R, for the
    # detector sums and the CBED patterns
    import torch
    d = build_inputs("s512", 1)
    plan = G.make_plan(d)
    f = 1
    amax = _amax(d, f)
    S = G.build_smatrix(plan, f, amax)
    pr = d["probes"][[0, 77, 300, 575]]
    R = G.probe_outputs(plan, f, amax, S, pr, d["optics"], d["edges"])
    Rc = G.probe_cbed(plan, f, amax, S, pr, d["optics"])
    xy = G.upload(pr)
    wsp = G.workspace(plan.probe_workspace_bytes(f, amax, d["optics"])[0])
    out = torch.zeros((len(pr), len(d["edges"])), dtype=torch.float64, device=G.device())
    outc = torch.zeros((len(pr), 256, 256), dtype=torch.float32, device=G.device())
    G.say("accumulate W=256 detector and CBED, weights 0.25 then 0.75")
    for wgt in (0.25, 0.75):
        plan.probe_outputs_accumulate(f, amax, S, xy, d["optics"], d["edges"], wgt, out, wsp)
        plan.probe_cbed_accumulate(f, amax, S, xy, d["optics"], wgt, outc, wsp)
    torch.cuda.synchronize()
    A, Ac = out.cpu().numpy(), outc.cpu().numpy()
    assert np.abs(A - R).max() <= 1e-13 * np.abs(R).max()
    assert np.abs(Ac - Rc).max() <= 1e-6 * np.abs(Rc).max()
    # and the result itself against the oracle for one probe (PRISM at f = 1
    # is multislice on the same grid)
    ref = O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"], d["optics"],
                            pr[1:2], d["edges"])[0]
    e = eps(A[1], ref)
    print(f"s512 f=1 W=256 accumulate probe 77 eps_rel={e:.3e}")
    assert e <= TOL
