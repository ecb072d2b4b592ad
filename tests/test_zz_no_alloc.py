"""prism_probe_outputs_noalloc (library-held scratch, no workspace argument)
against prism_probe_outputs on the same inputs, through the C ABI.

Two calls in a row on one GPU, the second with fewer probes, so the second
runs on scratch that still holds the first call's contents. The outputs must
equal the workspace call's bit for bit (same kernels, same probe groups) and
stay within the FP32 gate of the FP64 oracle (eps_rel <= 1e-4).
"""
import numpy as np
import pytest

import oracle as O
from synth import build_inputs

import _gpu as G

pytestmark = pytest.mark.gpu


def _amax(d, f):
    lam = O.wavelength(d["energy_keV"])
    return O.default_alpha_max(d["optics"]["alpha_mrad"] * 1e-3, f, lam, 1.0 / d["cell"]) * 1e3


def _noalloc(plan, f, amax, S, probes, optics, edges):
    import torch
    xy = G.upload(np.asarray(probes, dtype=np.float64))
    n_det = np.asarray(edges).reshape(-1, 2).shape[0]
    out = torch.full((len(probes), n_det), float("nan"), dtype=torch.float64, device=G.device())
    G.say(f"probe_outputs_noalloc n={plan.n} f={f} P={len(probes)}")
    plan.probe_outputs_noalloc(f, amax, S, xy, optics, edges, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("name,f,picks", [("tiny", 2, (256, 37)), ("mid256", 4, (133, 20))])
def test_noalloc_matches_workspace_call(name, f, picks):
    d = build_inputs(name, 0)
    plan = G.make_plan(d)
    amax = _amax(d, f)
    S = G.build_smatrix(plan, f, amax)
    beams, Sref = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f, amax)
    for P in picks:
        pr = d["probes"][:P]
        got = _noalloc(plan, f, amax, S, pr, d["optics"], d["edges"])
        ref_ws = G.probe_outputs(plan, f, amax, S, pr, d["optics"], d["edges"])
        assert np.array_equal(got, ref_ws), P
        ref = O.prism_outputs(Sref, beams, f, d["cell"], d["energy_keV"], d["optics"], pr,
                              d["edges"])
        e = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"noalloc {name} f={f} P={P} eps_rel={e:.3e}")
        assert e <= 1e-4


def test_noalloc_full_size_window_then_smaller():
    # fcc1024 at f = 16 (64 MiB of scratch): 4096 probes, then 1000
    d = build_inputs("fcc1024", 0)
    plan = G.make_plan(d)
    f = 16
    amax = _amax(d, f)
    S = G.build_smatrix(plan, f, amax)
    for P in (4096, 1000):
        pr = d["probes"][:P]
        got = _noalloc(plan, f, amax, S, pr, d["optics"], d["edges"])
        ref_ws = G.probe_outputs(plan, f, amax, S, pr, d["optics"], d["edges"])
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref_ws), P
