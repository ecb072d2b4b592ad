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
