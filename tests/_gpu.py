"""Drive libprism through the Python binding for GPU tests (no oracle here)."""
import sys

import numpy as np


def say(*args):
    """Name the case before a GPU step (flushed, so a fault still shows it)."""
    print("[gpu]", *args, flush=True)
    sys.stdout.flush()


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def upload_phase(inputs):
    import torch
    return torch.from_numpy(np.ascontiguousarray(inputs["phase"], dtype=np.float32)).to(device())


def make_plan(inputs, phase_dev=None):
    from paper_1702_01904_amd import Plan
    plan = Plan(inputs["n"], inputs["cell"], inputs["energy_keV"], inputs["thickness"])
    plan.set_potential_slices(phase_dev if phase_dev is not None else upload_phase(inputs))
    return plan


def workspace(nbytes):
    import torch
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device())


def build_smatrix(plan, f, amax, ws_bytes=None):
    import torch
    B = plan.beam_count(f, amax)
    ns = plan.n // 2
    S = torch.empty((B, ns, ns), dtype=torch.complex64, device=device())
    pref, mn = plan.build_workspace_bytes(f, amax)
    ws = workspace(pref if ws_bytes is None else max(mn, ws_bytes))
    say(f"build_smatrix n={plan.n} H={plan.n_slices} f={f} B={B} ws={ws.numel()}")
    plan.build_smatrix(f, amax, S, ws)
    torch.cuda.synchronize()
    return S


def probe_outputs(plan, f, amax, S, probes, optics, edges, ws_bytes=None):
    import torch
    xy = torch.from_numpy(np.ascontiguousarray(probes, dtype=np.float64)).to(device())
    n_det = np.asarray(edges).reshape(-1, 2).shape[0]
    out = torch.full((len(probes), n_det), float("nan"), dtype=torch.float64, device=device())
    pref, mn = plan.probe_workspace_bytes(f, amax, optics)
    ws = workspace(pref if ws_bytes is None else max(mn, ws_bytes))
    say(f"probe_outputs n={plan.n} f={f} P={len(probes)} n_det={n_det} ws={ws.numel()}")
    plan.probe_outputs(f, amax, S, xy, optics, edges, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def probe_cbed(plan, f, amax, S, probes, optics):
    import torch
    xy = torch.from_numpy(np.ascontiguousarray(probes, dtype=np.float64)).to(device())
    w = plan.n // (2 * f)
    out = torch.full((len(probes), w, w), float("nan"), dtype=torch.float32, device=device())
    pref, _ = plan.probe_workspace_bytes(f, amax, optics)
    ws = workspace(pref)
    say(f"probe_cbed n={plan.n} f={f} P={len(probes)} W={w} ws={ws.numel()}")
    plan.probe_cbed(f, amax, S, xy, optics, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def multislice_outputs(plan, probes, optics, edges, ws_bytes=None):
    import torch
    xy = torch.from_numpy(np.ascontiguousarray(probes, dtype=np.float64)).to(device())
    n_det = np.asarray(edges).reshape(-1, 2).shape[0]
    out = torch.full((len(probes), n_det), float("nan"), dtype=torch.float64, device=device())
    pref, mn = plan.multislice_workspace_bytes(n_det)
    ws = workspace(pref if ws_bytes is None else max(mn, ws_bytes))
    say(f"multislice_outputs n={plan.n} H={plan.n_slices} P={len(probes)} ws={ws.numel()}")
    plan.multislice_outputs(xy, optics, edges, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def upload(a, dtype=None):
    """Host array to a device tensor (float64 unless dtype is given)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device(), dtype=dtype if dtype is not None else t.dtype)


def frozen_phonon_prism(plan, f, amax, phase_configs, probes, optics, edges, cbed=False):
    """Mean over configurations through the accumulating probe step: one
    potential upload and S-matrix build per configuration, weight 1/K."""
    import torch
    K = len(phase_configs)
    xy = upload(np.asarray(probes, dtype=np.float64))
    B = plan.beam_count(f, amax)
    ns = plan.n // 2
    S = torch.empty((B, ns, ns), dtype=torch.complex64, device=device())
    wsb = workspace(plan.build_workspace_bytes(f, amax)[0])
    wsp = workspace(plan.probe_workspace_bytes(f, amax, optics)[0])
    if cbed:
        w = plan.n // (2 * f)
        out = torch.zeros((len(probes), w, w), dtype=torch.float32, device=device())
    else:
        n_det = np.asarray(edges).reshape(-1, 2).shape[0]
        out = torch.zeros((len(probes), n_det), dtype=torch.float64, device=device())
    phases = [upload(np.asarray(ph, dtype=np.float32)) for ph in phase_configs]
    for k, ph in enumerate(phases):
        say(f"frozen phonon prism config {k + 1}/{K} n={plan.n} f={f} B={B} "
            f"P={len(probes)} cbed={cbed}")
        plan.set_potential_slices(ph)
        plan.build_smatrix(f, amax, S, wsb)
        if cbed:
            plan.probe_cbed_accumulate(f, amax, S, xy, optics, 1.0 / K, out, wsp)
        else:
            plan.probe_outputs_accumulate(f, amax, S, xy, optics, edges, 1.0 / K, out, wsp)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def frozen_phonon_multislice(plan, phase_configs, probes, optics, edges):
    import torch
    K = len(phase_configs)
    xy = upload(np.asarray(probes, dtype=np.float64))
    n_det = np.asarray(edges).reshape(-1, 2).shape[0]
    out = torch.zeros((len(probes), n_det), dtype=torch.float64, device=device())
    ws = workspace(plan.multislice_workspace_bytes(n_det)[0])
    phases = [upload(np.asarray(ph, dtype=np.float32)) for ph in phase_configs]
    for k, ph in enumerate(phases):
        say(f"frozen phonon multislice config {k + 1}/{K} n={plan.n} P={len(probes)}")
        plan.set_potential_slices(ph)
        plan.multislice_outputs_accumulate(xy, optics, edges, 1.0 / K, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()
