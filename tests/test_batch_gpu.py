"""Batched S-matrix build of several specimens (shared launches, per-wave
transmission) against the FP64 oracle and against one-specimen builds.

Gate: eps_rel <= 1e-4 per beam against the oracle's S-matrix; every
batched S-matrix equals the specimen's own prism_build_smatrix bit for bit
(the per-wave arithmetic is the same; only the launches are shared).
"""
import numpy as np
import pytest

import oracle as O
from synth import batch_shapes, batch_workload, build_inputs
from paper_1702_01904_amd import Plan, build_batch_workspace_bytes, build_smatrix_batch

import _gpu as G

pytestmark = pytest.mark.gpu

TOL = 1e-4


def eps(a, ref):
    a = np.asarray(a)
    ref = np.asarray(ref)
    assert np.all(np.isfinite(a))
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


def _amax(d, f):
    lam = O.wavelength(d["energy_keV"])
    return O.default_alpha_max(d["optics"]["alpha_mrad"] * 1e-3, f, lam, 1.0 / d["cell"]) * 1e3


def _plans(specs):
    out = []
    for d in specs:
        ph = G.upload(np.asarray(d["phase"], dtype=np.float32))
        plan = G.make_plan(d, ph)
        out.append((d, plan, ph))
    return out


def _batch(entries, ws_bytes=None):
    import torch
    items = []
    for d, plan, _ in entries:
        f = d["f"]
        amax = _amax(d, f)
        B = plan.beam_count(f, amax)
        S = torch.full((B, plan.n // 2, plan.n // 2), float("nan"), dtype=torch.complex64,
                       device=G.device())
        items.append((plan, f, amax, S))
    pref, mn = build_batch_workspace_bytes(items)
    ws = G.workspace(pref if ws_bytes is None else max(mn, mn + ws_bytes))
    G.say(f"batched build of {len(items)} specimens: "
          + ", ".join(f"n={p.n} H={p.n_slices} f={f} B={S.shape[0]}" for p, f, _, S in items)
          + f" ws={ws.numel()}")
    build_smatrix_batch(items, ws)
    torch.cuda.synchronize()
    return [it[3].cpu().numpy() for it in items]


@pytest.fixture(scope="module")
def small():
    return _plans(batch_workload("batch_small", 0))


def test_batch_small_against_oracle_and_single_builds(small):
    Sb = _batch(small)
    for (d, plan, _), S in zip(small, Sb):
        f = d["f"]
        amax = _amax(d, f)
        beams, Sref = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f, amax)
        worst = max(eps(S[b], Sref[b]) for b in range(len(beams)))
        print(f"batch {d['name']} n={d['n']} H={len(d['thickness'])} f={f} B={len(beams)} "
              f"worst beam eps_rel={worst:.3e}")
        assert worst <= TOL
        S1 = G.build_smatrix(plan, f, amax).cpu().numpy()
        assert np.array_equal(S, S1)


def test_batch_small_workspace_splits_members(small):
    # a workspace of 7 waves beyond the minimum: chunks cut through members
    Sb = _batch(small, ws_bytes=7 * 256 * 128 * 8)
    for (d, plan, _), S in zip(small, Sb):
        S1 = G.build_smatrix(plan, d["f"], _amax(d, d["f"])).cpu().numpy()
        assert np.array_equal(S, S1)


def test_batch_groups_by_medium():
    # different energy / slice thickness / grid: separate groups, one call
    base = build_inputs("tiny", 3)
    other_e = dict(build_inputs("tiny", 4), energy_keV=120.0)
    other_t = dict(build_inputs("tiny", 5))
    other_t["thickness"] = np.full(len(other_t["thickness"]), 1.5)
    mid = build_inputs("mid256", 1)
    specs = []
    for d, f in ((base, 2), (other_e, 1), (other_t, 2), (mid, 4), (build_inputs("tiny", 6), 1)):
        specs.append(dict(d, f=f, name=f"n{d['n']}"))
    entries = _plans(specs)
    Sb = _batch(entries)
    for (d, plan, _), S in zip(entries, Sb):
        S1 = G.build_smatrix(plan, d["f"], _amax(d, d["f"])).cpu().numpy()
        assert np.array_equal(S, S1)
    # and the 120 keV member against the oracle
    d = specs[1]
    beams, Sref = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], 1,
                            _amax(d, 1))
    worst = max(eps(Sb[1][b], Sref[b]) for b in range(len(beams)))
    print(f"batch 120 keV member worst beam eps_rel={worst:.3e}")
    assert worst <= TOL


def test_batch_full_size_members():
    # members of the 32-specimen mix at their real sizes (n = 1024 with
    # f = 4, n = 512, n = 768, n = 256): batched S equals single builds, and sampled
    # probes of the n = 256 member through the batched S against the oracle
    shapes = batch_shapes("batch32", 0)
    pick = [i for i, (n, _, f) in enumerate(shapes) if n == 1024 and f == 4][:1]
    pick += [i for i, (n, _, _) in enumerate(shapes) if n == 512][:1]
    pick += [i for i, (n, _, _) in enumerate(shapes) if n == 768][:1]   # a 3 * 2^k grid
    pick += [i for i, (n, _, _) in enumerate(shapes) if n == 256][:2]
    chosen = batch_workload("batch32", 0, indices=pick)
    entries = _plans(chosen)
    Sb = _batch(entries)
    for (d, plan, _), S in zip(entries, Sb):
        S1 = G.build_smatrix(plan, d["f"], _amax(d, d["f"])).cpu().numpy()
        assert np.array_equal(S, S1), d["name"]
    import torch
    d, plan, _ = entries[-1]
    f = d["f"]
    amax = _amax(d, f)
    Sdev = torch.from_numpy(Sb[-1]).to(G.device())
    pr = d["probes"][[0, 1111, 4095]]
    D = G.probe_outputs(plan, f, amax, Sdev, pr, d["optics"], d["edges"])
    for k, (x0, y0) in enumerate(pr):
        ref = O.prism_probe_direct(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f,
                                   amax, d["optics"], x0, y0, d["edges"])
        e = eps(D[k], ref)
        print(f"batch32 member {d['name']} n=256 H={len(d['thickness'])} f={f} probe {k} "
              f"eps_rel={e:.3e}")
        assert e <= TOL
