#!/usr/bin/env python3
"""Throughput benchmark: PRISM vs multislice STEM probe positions per second.

Workload (fcc1024): 40 x 40 x 100 A Au FCC crystal (a = 4.08 A, 10,000
atoms, 0.08 A seeded jitter), 1024^2 grid, 50 slices of 2 A, 200 keV,
25 mrad probe, 256 x 256 scan at 0.15625 A, 16 radial bins to 200 mrad.

One timed step = the whole PRISM path for one specimen: build the compact
S-matrix (every beam through all 50 slices, quarter-size extraction) and
compute the detector outputs of all 65,536 probe positions. ``value`` is
65,536 / step time. The multislice baseline runs the same slice kernels on
a seeded subset of probes in its own timed region (its rate per probe does
not depend on the scan size) and is reported beside it with the speed-up.

Per-kernel durations come from HIP events that the library records on the
launch stream during the timed steps; the dominant kernel's roofline is
derived from them. ``--no-cpu-baseline`` skips the FP64 oracle timing.
"""
import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix
F16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 / FP16 matrix
CONFIG = "fcc1024"

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE on this
# workload (f = 4), calibrated with a 256 MiB device copy (fetch x2.0,
# write x1.0), as in the HBM-traffic summary under profiles/. Valid only for
# the kernel sources with this hash (of their code, comments aside); reported
# as null otherwise.
TRAFFIC_SRC_SHA = "a81852979c72bdc3"
TRAFFIC_BYTES = {"row_pass": 563499446, "col_pass": 521796428, "contract": 9375558529,
                 "s32_pack": 1310732154, "window_detect": 1079331347, "contract16": 4706686928,
                 "s16_pack": 975213709}


# Sources that decide the profiled kernels and their launch shapes (the
# serving layer and the binding do not).
KERNEL_SOURCES = ("slice_kernels.hip", "probe_kernels.hip", "probe16_kernels.hip", "fft_lds.hpp",
                  "fft_reg.hpp", "kernels.hpp", "plan.cpp")


_TOKENS = re.compile(r'("(?:\\.|[^"\\\n])*"|\'(?:\\.|[^\'\\\n])*\')|//[^\n]*|/\*.*?\*/', re.S)


def _code_only(text):
    """C++ source without comments, trailing blanks and empty lines (string
    and character literals kept), so that comment edits keep the hash."""
    text = _TOKENS.sub(lambda m: m.group(1) or "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def kernel_source_sha():
    """Hash of the code of the kernel sources and of the launch-shape table
    (both decide the kernels' HBM traffic)."""
    import hashlib
    src = os.path.join(ROOT, "paper_1702_01904_amd", "csrc")
    text = "".join(_code_only(open(os.path.join(src, f)).read()) for f in KERNEL_SOURCES)
    table = os.path.join(ROOT, "paper_1702_01904_amd", "tuning_gfx950.json")
    if os.path.exists(table):
        text += open(table).read()
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--f", type=int, default=4, help="interpolation factor of the headline run")
    ap.add_argument("--other-f", default="8,16", help="extra f values timed (comma list, '' none)")
    ap.add_argument("--ms-probes", type=int, default=128,
                    help="multislice probes timed (0: skip the multislice baseline)")
    ap.add_argument("--precisions", default="bf16,fp16",
                    help="16-bit window-sum variants timed at the headline f ('' none)")
    ap.add_argument("--phonon-configs", type=int, default=2,
                    help="frozen-phonon configurations timed at the headline f (0: skip the "
                         "probe-side variants: resident-S step, CBED output, frozen phonons)")
    ap.add_argument("--batch", default="batch32",
                    help="mixed specimen batch timed with the batched build ('' none)")
    ap.add_argument("--serve-rates", default="50,150,250",
                    help="query arrival rates (per s) of the serving run ('' none)")
    ap.add_argument("--serve-queries", type=int, default=200)
    ap.add_argument("--serve-build-rate", type=float, default=2.0,
                    help="S-matrix build arrivals per s in the serving run")
    ap.add_argument("--serve-resident-gb", type=float, default=110.0,
                    help="byte budget of resident S-matrices in the serving run (GB)")
    ap.add_argument("--np2048", type=int, default=1,
                    help="time the precision forms on the np2048 nanoparticle case (0: skip)")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip the copy / GEMM peak measurement (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (reference for HBM counters)")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic work per kernel (units summed over the launches of one step)

def kernel_work(name, g):
    """(kind, amount) of algorithmic work for all launches of ``name`` in one step."""
    N, H, B, P, W, BA = g["N"], g["H"], g["B"], g["P"], g["W"], g["BA"]
    state = 4.0 * N * N           # compact wave: N x N/2 complex64
    if name == "row_pass":
        # read + write the wave state, plus the slice's transmission once per launch
        return "hbm", B * H * 2 * state + g["launches"] * 8.0 * N * N
    if name == "col_pass":
        return "hbm", B * H * 2 * state
    if name == "extract":
        return "hbm", B * (state / 2 + 2.0 * N * N)
    if name == "beam_init":
        return "hbm", B * state
    if name in ("contract", "contract16"):
        return "mfma", 8.0 * BA * W * W * P
    if name in ("s32_pack", "s16_pack"):
        # read the active S planes, write the pixel-major copy (8 or 4 bytes per beam-pixel)
        return "hbm", BA * g["NS"] ** 2 * (16.0 if name == "s32_pack" else 12.0)
    if name == "window_detect":
        return "hbm", 8.0 * W * W * P + 8.0 * P * g["n_det"]
    if name == "transmission":
        return "hbm", H * N * N * (4.0 + 8.0)
    return None, 0.0


def roofline(prof, g, steps, name=None):
    """Roofline entry for ``name`` (default: the kernel with the largest total time)."""
    if name is None:
        name = max(prof, key=lambda k: prof[k]["total_ms"])
    ent = dict(prof[name])
    launches = ent["launches"] / steps
    g = dict(g, launches=launches)
    kind, amount = kernel_work(name, g)
    per_launch_ms = ent["total_ms"] / ent["launches"]
    per_launch_units = amount / launches
    if kind == "mfma":
        achieved = per_launch_units / (per_launch_ms * 1e-3) / 1e12
        peak = F16_MFMA_PEAK_TFLOPS if name.endswith("16") else FP32_MFMA_PEAK_TFLOPS
        unit = "TFLOP/s"
    else:
        achieved = per_launch_units / (per_launch_ms * 1e-3) / 1e9
        peak, unit = HBM_PEAK_GBS, "GB/s"
    traffic = None
    if name in TRAFFIC_BYTES and kernel_source_sha() == TRAFFIC_SRC_SHA:
        traffic = TRAFFIC_BYTES[name]
    return name, {
        "bound": kind, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
        "frac": round(achieved / peak, 4), "traffic": traffic,
        "kernel": name, "launches_per_step": launches,
        "avg_launch_ms": round(per_launch_ms, 4),
        "algorithmic_per_launch": per_launch_units,
    }


# ---------------------------------------------------------------------------
# accuracy of the timed outputs against the committed FP64 oracle outputs
# (tests/golden/, written from the oracle alone by tests/golden/make_goldens.py)

GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def golden(name):
    """(probe indices, values [P][n_det]) of a golden file, or None if absent."""
    path = os.path.join(GOLDEN_DIR, name)
    if not os.path.exists(path):
        return None
    a = np.loadtxt(path, comments="#", ndmin=2)
    return a[:, 0].astype(np.int64), a[:, 3:]


def accuracy(D, ref, edges, half_band_mrad, floor):
    """eps_rel over the sample, max |dD| (units of total probe intensity) and
    per-bin eps_rel: the worst over the bins the parity tests gate (entirely
    below the half-band angle, mean at least ``floor`` of the intensity),
    and each other bin's figure beside its mean (near-empty or past the band
    limit)."""
    D = np.asarray(D, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    num = np.linalg.norm(D - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    per = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
    edges = np.asarray(edges)
    mean = np.abs(ref).mean(axis=0)
    gated = (edges[:, 1] <= half_band_mrad) & (mean >= floor)
    return {"eps_rel": float(np.linalg.norm(D - ref) / np.linalg.norm(ref)),
            "max_abs_dD": float(np.abs(D - ref).max()),
            "worst_gated_bin_eps_rel": float(per[gated].max()),
            "ungated_bins": {f"{lo:g}-{hi:g} mrad": {"eps_rel": float(e), "mean": float(m)}
                             for (lo, hi), e, m, g in zip(edges, per, mean, gated) if not g},
            "probes": int(D.shape[0])}


def floor_of(prec):
    """Near-empty floor of the per-bin gate (fraction of the probe's intensity)."""
    return 1e-6 if prec in ("fp32", "multislice") else 1e-4


def method_error(D_prism, D_multi, edges, half_band_mrad):
    """PRISM against multislice on the same probes (the method's own error,
    not a parity figure): 1 - R^2 per detector bin (R the Pearson correlation
    over the probes, as the paper's image comparison) and rel-L2 overall."""
    out = []
    for j, (lo, hi) in enumerate(np.asarray(edges)):
        a, b = D_prism[:, j], D_multi[:, j]
        if lo >= half_band_mrad or np.std(a) == 0 or np.std(b) == 0:
            out.append(None)
            continue
        r = np.corrcoef(a, b)[0, 1]
        out.append(round(float(1.0 - r * r), 6))
    return {"one_minus_r2_per_bin": out,
            "rel_l2": round(float(np.linalg.norm(D_prism - D_multi) / np.linalg.norm(D_multi)), 6)}


def host_cpu():
    """Model name of the host CPU (first entry of /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(d, f, amax, P_full):
    """Time the FP64 oracle on a bounded sample (on every host core it may
    use) and scale to the full build + scan in probes/s."""
    import oracle as O
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    F = O.ScipyFFT(workers=cores)
    lam = O.wavelength(d["energy_keV"])
    beams = O.beam_set(d["n"], d["cell"], lam, f, amax * 1e-3)
    B = len(beams)
    nb = 8
    pick = np.linspace(0, B - 1, nb).astype(np.int64)
    t0 = time.perf_counter()
    _, S1 = O.smatrix(d["phase"], d["thickness"], d["cell"], d["energy_keV"], f, amax, fft=F,
                      beams=beams[pick])
    t_beam = (time.perf_counter() - t0) / nb
    S = np.repeat(S1, -(-B // nb), axis=0)[:B]      # right shape for timing the probe step
    del S1
    npr = 256
    sel = np.linspace(0, P_full - 1, npr).astype(np.int64)
    t0 = time.perf_counter()
    O.prism_outputs(S, beams, f, d["cell"], d["energy_keV"], d["optics"], d["probes"][sel],
                    d["edges"], fft=F)
    t_probe = (time.perf_counter() - t0) / npr
    del S
    nms = 2
    t0 = time.perf_counter()
    O.multislice_stem(d["phase"], d["thickness"], d["cell"], d["energy_keV"], d["optics"],
                      d["probes"][:nms], d["edges"], fft=F)
    t_ms = (time.perf_counter() - t0) / nms
    total = t_beam * B + t_probe * P_full
    return {
        "value": round(P_full / total, 3), "unit": "probes/s", "cores": cores, "kind": "oracle",
        "sample": (f"FP64 oracle (scipy.fft, {cores} workers), f={f}: S-matrix of {nb} of {B} "
                   f"beams ({t_beam:.2f} s/beam), probe step of {npr} of {P_full} probes "
                   f"({t_probe * 1e3:.1f} ms/probe), scaled to the full build + scan; "
                   f"multislice on {nms} probes ({t_ms:.2f} s/probe)"),
        "os_cpu_count": os.cpu_count(), "host_cpu": host_cpu(),
        "multislice_probes_per_s": round(1.0 / t_ms, 4),
    }


def measured_peaks(dev):
    """What this GPU reaches on plain work: a 1 GiB device copy (GB/s, bytes
    read + written) and square FP32 / BF16 library GEMMs (TFLOP/s)."""
    import torch

    def ev(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    x = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    copy_gbs = 2.0 * x.numel() * 4 / (ev(lambda: y.copy_(x)) * 1e-3) / 1e9
    del x, y
    out = {"copy_GBps": round(copy_gbs, 1)}
    n = 8192
    for name, dt in (("gemm_fp32_TFLOPs", torch.float32), ("gemm_bf16_TFLOPs", torch.bfloat16)):
        a = torch.randn(n, n, dtype=dt, device=dev)
        b = torch.randn(n, n, dtype=dt, device=dev)
        out[name] = round(2.0 * n ** 3 / (ev(lambda: torch.mm(a, b)) * 1e-3) / 1e12, 1)
        del a, b
    torch.cuda.synchronize()
    return out


def run_precision_np2048(args, dev):
    """Window-sum precision forms on the 2048^2 nanoparticle-on-carbon case
    (1024 sub-pixel probes, f = 4 and 8): probe-step time per precision and
    eps_rel of the 16-bit outputs against the FP32 outputs of the same S
    (their FP64-oracle parity is a GPU test)."""
    import torch
    from synth import build_inputs
    from paper_1702_01904_amd import Plan
    d = build_inputs("np2048", args.seed)
    p = Plan(d["n"], d["cell"], d["energy_keV"], d["thickness"])
    ph = torch.from_numpy(d["phase"]).to(dev)
    p.set_potential_slices(ph)
    P, nd = len(d["probes"]), len(d["edges"])
    res = {}
    for f in (4, 8):
        # the library's compact order for scattered probes (results do not
        # depend on it); the as-given order is timed once for comparison
        perm = p.probe_order(f, d["probes"])
        xy = torch.from_numpy(d["probes"][perm]).to(dev)
        xy_given = torch.from_numpy(d["probes"]).to(dev)
        amax = p.alpha_max_default(d["optics"]["alpha_mrad"], f)
        B = p.beam_count(f, amax)
        S = torch.empty((B, d["n"] // 2, d["n"] // 2), dtype=torch.complex64, device=dev)
        wsb = torch.empty(p.build_workspace_bytes(f, amax)[0], dtype=torch.uint8, device=dev)
        p.build_smatrix(f, amax, S, wsb)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        p.build_smatrix(f, amax, S, wsb)
        e1.record()
        torch.cuda.synchronize()
        n = d["n"]
        bms = e0.elapsed_time(e1)
        gbs = B * len(d["thickness"]) * 16.0 * n * n / (bms * 1e-3) / 1e9
        ent = {"beams": B, "window": n // (2 * f), "build_ms": round(bms, 3),
               "build_hbm_GBps": round(gbs, 1), "build_hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        ba = p.active_beam_count(f, amax, d["optics"])
        flops = 8.0 * ba * (n // (2 * f)) ** 2 * P     # useful window-sum flops per probe step
        del wsb
        outs = {}
        for prec in ("fp32", "bf16", "fp16"):
            p.set_probe_precision(prec)
            wsp = torch.empty(p.probe_workspace_bytes(f, amax, d["optics"])[0],
                              dtype=torch.uint8, device=dev)
            out = torch.empty((P, nd), dtype=torch.float64, device=dev)
            p.probe_outputs(f, amax, S, xy, d["optics"], d["edges"], out, wsp)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                p.probe_outputs(f, amax, S, xy, d["optics"], d["edges"], out, wsp)
            e1.record()
            torch.cuda.synchronize()
            outs[prec] = out.cpu().numpy()
            ent[f"{prec}_probe_ms"] = round(e0.elapsed_time(e1) / args.steps, 3)
            if prec == "fp32":
                e0.record()
                p.probe_outputs(f, amax, S, xy_given, d["optics"], d["edges"], out, wsp)
                e1.record()
                torch.cuda.synchronize()
                ent["fp32_probe_ms_input_order"] = round(e0.elapsed_time(e1), 3)
            del wsp
        p.set_probe_precision("fp32")
        ent["active_beams"] = ba
        for prec, peak in (("fp32", FP32_MFMA_PEAK_TFLOPS), ("bf16", F16_MFMA_PEAK_TFLOPS),
                           ("fp16", F16_MFMA_PEAK_TFLOPS)):
            tf = flops / (ent[f"{prec}_probe_ms"] * 1e-3) / 1e12
            ent[f"{prec}_window_sum_TFLOPs_whole_step"] = round(tf, 2)
            ent[f"{prec}_mfma_frac_whole_step"] = round(tf / peak, 4)
        for prec in ("bf16", "fp16"):
            ref = outs["fp32"]
            ent[f"eps_rel_{prec}_vs_fp32"] = float(np.linalg.norm(outs[prec] - ref)
                                                   / np.linalg.norm(ref))
        g = golden(f"np2048_prism_f{f}.txt")
        if g is not None:
            hb = p.wavelength / d["cell"] * (n / 4) * 1e3
            inv = np.empty_like(perm)
            inv[perm] = np.arange(len(perm))
            ent["accuracy_vs_fp64_oracle"] = {
                prec: accuracy(outs[prec][inv][g[0]], g[1], d["edges"], hb, floor_of(prec))
                for prec in ("fp32", "bf16", "fp16")}
        res[str(f)] = ent
        log(f"np2048 f={f}: build {ent['build_ms']} ms, probe step fp32/bf16/fp16 "
            f"{ent['fp32_probe_ms']}/{ent['bf16_probe_ms']}/{ent['fp16_probe_ms']} ms")
        del S, xy, xy_given
    del ph
    torch.cuda.synchronize()
    return {"workload": "np2048: Au r=20 A particle on 30 A carbon, 2048^2, 35 slices, 80 keV, "
                        "20 mrad, 1024 sub-pixel probes, one bin [40,150) mrad",
            "probe_order": "prism_probe_order (compact runs of the scattered probes)",
            "per_f": res, "tolerance": "eps_rel <= 1e-4 (FP32), 1e-2 (BF16/FP16) vs the FP64 "
                                       "oracle (accuracy_vs_fp64_oracle: all 1024 probes)"}


def run_batch(args, dev):
    """Mixed batch of specimens: batched S-matrix build (shared launches)
    against one build call per specimen, then every specimen's probe step."""
    import torch
    from synth import batch_workload
    from paper_1702_01904_amd import (Plan, build_batch_workspace_bytes, build_smatrix_batch,
                                      probe_batch, probe_batch_workspace_bytes, tile_order)
    t0 = time.perf_counter()
    specs = batch_workload(args.batch, args.seed)
    log(f"batch {args.batch}: {len(specs)} specimens generated in {time.perf_counter() - t0:.1f} s")
    ents = []
    for d in specs:
        f = d["f"]
        p = Plan(d["n"], d["cell"], d["energy_keV"], d["thickness"])
        ph = torch.from_numpy(d["phase"]).to(dev)
        p.set_potential_slices(ph)
        amax = p.alpha_max_default(d["optics"]["alpha_mrad"], f)
        B = p.beam_count(f, amax)
        S = torch.empty((B, d["n"] // 2, d["n"] // 2), dtype=torch.complex64, device=dev)
        _, tx, ty = p.probe_group(f)
        xy = torch.from_numpy(d["probes"][tile_order(d["n"] // 4, d["n"] // 4, tx, ty)]).to(dev)
        out = torch.empty((len(d["probes"]), len(d["edges"])), dtype=torch.float64, device=dev)
        ents.append(dict(d=d, f=f, plan=p, ph=ph, amax=amax, B=B, S=S, xy=xy, out=out))
    items = [(e["plan"], e["f"], e["amax"], e["S"]) for e in ents]
    wsb = torch.empty(build_batch_workspace_bytes(items)[0], dtype=torch.uint8, device=dev)
    ws1 = torch.empty(max(e["plan"].build_workspace_bytes(e["f"], e["amax"])[0] for e in ents),
                      dtype=torch.uint8, device=dev)
    wsp = torch.empty(max(e["plan"].probe_workspace_bytes(e["f"], e["amax"], e["d"]["optics"])[0]
                          for e in ents), dtype=torch.uint8, device=dev)

    def ev_ms(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    ms_batched = ev_ms(lambda: build_smatrix_batch(items, wsb))
    ms_single = ev_ms(lambda: [e["plan"].build_smatrix(e["f"], e["amax"], e["S"], ws1)
                               for e in ents])
    ms_probe = ev_ms(lambda: [e["plan"].probe_outputs(e["f"], e["amax"], e["S"], e["xy"],
                                                      e["d"]["optics"], e["d"]["edges"],
                                                      e["out"], wsp) for e in ents])
    # every specimen's probe step in one call: specimens of one launch class
    # share the window-sum and window launches
    reqs = [dict(plan=e["plan"], f=e["f"], alpha_max_mrad=e["amax"], smatrix=e["S"],
                 probe_xy=e["xy"], optics=e["d"]["optics"], edges_mrad=e["d"]["edges"],
                 out=torch.empty_like(e["out"])) for e in ents]
    pb_pref, pb_min = probe_batch_workspace_bytes(reqs)
    wspb = torch.empty(max(pb_min, min(pb_pref, 32 << 30)), dtype=torch.uint8, device=dev)
    ms_probe_batched = ev_ms(lambda: probe_batch(reqs, wspb))
    probe_batch_equal = all(bool(torch.equal(r["out"], e["out"])) for r, e in zip(reqs, ents))
    classes = len({e["plan"].probe_class(e["f"]) for e in ents})
    del reqs, wspb
    per_n = {}
    for n in sorted({e["d"]["n"] for e in ents}):
        sub = [e for e in ents if e["d"]["n"] == n]
        its = [(e["plan"], e["f"], e["amax"], e["S"]) for e in sub]
        mb = ev_ms(lambda: build_smatrix_batch(its, wsb))
        m1 = ev_ms(lambda: [e["plan"].build_smatrix(e["f"], e["amax"], e["S"], ws1) for e in sub])
        bs_n = sum(e["B"] * len(e["d"]["thickness"]) for e in sub)
        gbs = bs_n * 16.0 * n * n / (mb * 1e-3) / 1e9   # two passes, 4 n^2 B each way
        per_n[str(n)] = {"specimens": len(sub), "beam_slices": bs_n,
                         "build_batched_ms": round(mb, 3), "build_per_specimen_ms": round(m1, 3),
                         "build_hbm_GBps": round(gbs, 1),
                         "build_hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
    finite = all(bool(torch.isfinite(e["out"]).all()) for e in ents)
    bsl = sum(e["B"] * len(e["d"]["thickness"]) for e in ents)
    P = sum(len(e["d"]["probes"]) for e in ents)
    log(f"batch: batched build {ms_batched:.1f} ms, one call per specimen {ms_single:.1f} ms, "
        f"probe steps {ms_probe:.1f} ms (one batched call {ms_probe_batched:.1f} ms, "
        f"{classes} launch classes, equal {probe_batch_equal})")
    del ents, items, wsb, ws1, wsp
    torch.cuda.synchronize()
    return {
        "workload": f"{args.batch}: {len(specs)} random specimens, 0.1 A pixels, n in "
                    f"{sorted({d['n'] for d in specs})}, 20-120 slices, f in "
                    f"{sorted({d['f'] for d in specs})}, 80 keV, 20 mrad, (n/4)^2 probes each",
        "specimens": len(specs), "beam_slices": bsl, "probes": P,
        "build_batched_ms": round(ms_batched, 3), "build_per_specimen_ms": round(ms_single, 3),
        "beam_slices_per_s_batched": round(bsl / (ms_batched * 1e-3), 1),
        "beam_slices_per_s_per_specimen": round(bsl / (ms_single * 1e-3), 1),
        "probe_steps_ms": round(ms_probe, 3),
        "probes_per_s_probe_steps": round(P / (ms_probe * 1e-3), 1),
        "probe_batch_ms": round(ms_probe_batched, 3),
        "probes_per_s_probe_batch": round(P / (ms_probe_batched * 1e-3), 1),
        "probe_batch_launch_classes": classes,
        "probe_batch_equals_per_specimen_calls": probe_batch_equal,
        "probes_per_s_end_to_end": round(P / ((ms_batched + min(ms_probe, ms_probe_batched)) * 1e-3), 1),
        "by_grid": per_n,
        "outputs_finite": finite,
    }


def run_serving(args, plan_fcc, d_fcc, dev):
    """Continuous batching: Poisson arrivals of probe queries and S-matrix
    builds against a large resident set, with memory-based admission.

    Resident at the start: S-matrices of seeded random specimens on 2048^2
    and 1024^2 grids (80 and 40 A cells, 80 keV, 20 mrad; f = 4 and 8) plus the
    fcc1024 specimen at f = 4, 8, 16, filling --serve-resident-gb. Queries
    (Poisson, rate swept) pick a resident S-matrix and a probe count
    log-uniform in [64, 65536] (a run of its (n/4)^2 scan raster in
    probe-tile order); builds (Poisson, --serve-build-rate per s) are new
    S-matrices of n in {512, 1024, 2048} and f in {4, 8, 16}, admitted by
    the server once they fit its budget, releasing least recently used idle
    S-matrices (LRU eviction). The driver submits requests as they arrive,
    flushes whenever something arrived and polls for completions. Latency =
    completion seen - arrival, per request type.
    """
    import math
    import torch
    from synth import build_inputs
    from paper_1702_01904_amd import Plan, Server, tile_order
    edges = [(0.0, 20.0), (20.0, 40.0), (40.0, 100.0)]
    optics = dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0)

    def specimen(n, seed, H):
        side = {512: 25.6, 1024: 40.0, 2048: 80.0}[n]    # the tests' cells at these grids
        cfg = dict(specimen=dict(kind="random", cell=(side, side, 2.0 * H),
                                 n_atoms=int(round(0.015 * side * side * 2.0 * H)),
                                 z_choices=(6, 14, 29, 79)),
                   n=n, n_slices=H, slice_A=2.0, energy_keV=80.0, optics=dict(optics),
                   scan=dict(nx=4, ny=4, step_A=1.0, origin_A=(0.0, 0.0)),
                   detectors=edges, f_values=(4,))
        d = build_inputs(cfg, seed)
        p = Plan(n, d["cell"], d["energy_keV"], d["thickness"])
        ph = torch.from_numpy(d["phase"]).to(dev)
        p.set_potential_slices(ph)
        return dict(p=p, d=d, ph=ph)

    t0 = time.perf_counter()
    kinds = {512: [specimen(512, 11, 20)], 1024: [specimen(1024, 12 + k, 30) for k in range(2)],
             2048: [specimen(2048, 20 + k, 35) for k in range(2)]}
    kinds["fcc"] = [dict(p=plan_fcc, d=d_fcc, ph=None)]
    torch.cuda.synchronize()
    log(f"serving: specimens ready in {time.perf_counter() - t0:.1f} s")
    # three query streams and the build stream: one hardware queue each (HIP
    # maps streams onto 4 hardware queues by default; a fifth stream would
    # share a queue with the build stream and wait behind its launches)
    max_probes, n_streams = 65536, 3
    max_det = max(len(edges), len(d_fcc["edges"]))
    shapes = [(n, f) for n in (512, 1024, 2048) for f in (4, 8, 16)] + [("fcc", 4), ("fcc", 8),
                                                                        ("fcc", 16)]
    probe_ws = 0
    ws_build = 0
    for key, f in shapes:
        sp = kinds[key][0]
        amax = sp["p"].alpha_max_default(sp["d"]["optics"]["alpha_mrad"], f)
        probe_ws = max(probe_ws, sp["p"].probe_workspace_bytes(f, amax, sp["d"]["optics"])[0])
        ws_build = max(ws_build, sp["p"].build_workspace_bytes(f, amax)[0])
    ws = torch.empty(Server.workspace_bytes(n_streams, max_probes, max_det, probe_ws),
                     dtype=torch.uint8, device=dev)
    wsb = torch.empty(ws_build, dtype=torch.uint8, device=dev)
    budget = int(args.serve_resident_gb * 1e9)
    srv = Server(budget, ws, n_streams=n_streams, max_probes=max_probes, max_det=max_det)
    srv.set_lru_eviction(True)
    # one call in flight per slot: queries that arrive while every slot is
    # busy wait and leave together (merged by launch class) when one frees
    srv.set_dispatch_limit(1)
    free_bufs = {}      # (n, f) shape -> S buffers released by eviction
    live = {}           # specimen id -> entry

    def s_buffer(sp, f, amax):
        key = (sp["p"].n, sp["p"].beam_count(f, amax))
        if free_bufs.get(key):
            return free_bufs[key].pop()
        return torch.empty((key[1], sp["p"].n // 2, sp["p"].n // 2), dtype=torch.complex64,
                           device=dev)

    def reclaim():
        for sid in srv.evictions():
            e = live.pop(sid)
            free_bufs.setdefault((e["sp"]["p"].n, e["S"].shape[0]), []).append(e["S"])

    def submit_build(key, f, rng_pick):
        sp = kinds[key][rng_pick % len(kinds[key])]
        amax = sp["p"].alpha_max_default(sp["d"]["optics"]["alpha_mrad"], f)
        S = s_buffer(sp, f, amax)
        sid, t = srv.submit_build(sp["p"], f, amax, S, wsb)
        live[sid] = dict(sp=sp, f=f, amax=amax, S=S, n=sp["p"].n)
        return t

    # fill the resident set: fcc1024 at f = 4, 8, 16, then 2048^2 and 1024^2
    # S-matrices at f = 4 and 8, one after another, until the budget is used
    def bytes_of(key, f):
        p = kinds[key][0]["p"]
        return p.smatrix_bytes(f, p.alpha_max_default(optics["alpha_mrad"] if key != "fcc"
                                                      else d_fcc["optics"]["alpha_mrad"], f))

    fill = [("fcc", 4), ("fcc", 8), ("fcc", 16)]
    planned = sum(bytes_of(key, f) for key, f in fill)
    k = 0
    while True:
        key, f = ((2048, 4), (1024, 4), (2048, 8), (1024, 8))[k % 4]
        if planned + bytes_of(key, f) > 0.95 * budget:
            break
        fill.append((key, f))
        planned += bytes_of(key, f)
        k += 1
    t0 = time.perf_counter()
    for i, (key, f) in enumerate(fill):
        t = submit_build(key, f, i)
        srv.flush()
        srv.wait(t)
        reclaim()
    torch.cuda.synchronize()
    resident0 = srv.stats()[0]
    log(f"serving: {len(fill)} S-matrices resident ({resident0 / 1e9:.1f} GB) in "
        f"{time.perf_counter() - t0:.1f} s")

    rng = np.random.default_rng(args.seed + 99)
    pools = {}
    for key in kinds:
        n = kinds[key][0]["p"].n
        for f in (4, 8, 16):
            _, tx, ty = kinds[key][0]["p"].probe_group(f)
            n4 = n // 4
            step = kinds[key][0]["d"]["cell"] / n4
            i = np.arange(n4, dtype=np.float64) * step
            ras = np.stack([np.tile(i, n4), np.repeat(i, n4)], axis=1)[tile_order(n4, n4, tx, ty)]
            reps = -(-max_probes // len(ras))
            pools[(key, f)] = torch.from_numpy(
                np.ascontiguousarray(np.tile(ras, (reps, 1))[:max_probes])).to(dev)

    def run(rate, n_q, build_rate, warm=False):
        # merged, time-sorted arrivals of queries and builds
        qa = np.cumsum(rng.exponential(1.0 / rate, n_q))
        span_q = qa[-1]
        nb = max(1, int(rng.poisson(build_rate * span_q)))
        ba = np.sort(rng.uniform(0.0, span_q, nb))
        events = sorted([(t, "q") for t in qa] + [(t, "b") for t in ba])
        t_first = events[0][0]
        P = np.exp(rng.uniform(math.log(64), math.log(65536), n_q)).astype(np.int64)
        outs = []
        torch.cuda.synchronize()
        kind_of, arrive, done_at = {}, {}, {}
        flushes, qi = 0, 0
        calls0 = srv.call_stats()
        t0 = time.perf_counter()
        ev = 0
        while ev < len(events) or len(done_at) < len(arrive):
            now = time.perf_counter() - t0
            sub = False
            while ev < len(events) and events[ev][0] - t_first <= now:
                typ = events[ev][1]
                if typ == "q":
                    sid = list(live)[int(rng.integers(0, len(live)))]
                    e = live[sid]
                    key = "fcc" if e["sp"]["p"] is plan_fcc else e["n"]
                    pool = pools[(key, e["f"])]
                    p = int(P[qi])
                    st = int(rng.integers(0, max_probes - p + 1))
                    outs.append(torch.empty((p, len(e["sp"]["d"]["edges"])),
                                            dtype=torch.float64, device=dev))
                    t = srv.submit(sid, pool[st:st + p], e["sp"]["d"]["optics"],
                                   e["sp"]["d"]["edges"], outs[-1])
                    kind_of[t] = ("query", p)
                    qi += 1
                else:
                    key = (512, 1024, 2048)[int(rng.integers(0, 3))]
                    f = (4, 8, 16)[int(rng.integers(0, 3))]
                    t = submit_build(key, f, int(rng.integers(0, 4)))
                    kind_of[t] = ("build", 0)
                arrive[t] = events[ev][0] - t_first
                ev += 1
                sub = True
            if sub:
                srv.flush()
                reclaim()
                flushes += 1
            for t in srv.poll():
                done_at[t] = time.perf_counter() - t0
            if not sub and srv.stats()[1] > 0:
                srv.flush()       # builds (and their queries) waiting for memory
                reclaim()
        span = max(done_at.values())
        if warm:
            return None
        calls1 = srv.call_stats()
        res = {"offered_queries_per_s": rate, "offered_builds_per_s": build_rate,
               "flushes": flushes, "resident_GB_end": round(srv.stats()[0] / 1e9, 2),
               "probe_calls": calls1[0] - calls0[0],
               "probe_calls_over_several_specimens": calls1[1] - calls0[1]}
        for kind in ("query", "build"):
            ts = [t for t in arrive if kind_of[t][0] == kind]
            if not ts:
                continue
            lat = np.array([done_at[t] - arrive[t] for t in ts]) * 1e3
            res[kind] = {"count": len(ts),
                         "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                         "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                         "latency_ms_max": round(float(lat.max()), 3)}
        probes = int(sum(kind_of[t][1] for t in arrive))
        res["query"]["probes"] = probes
        res["probes_per_s"] = round(probes / span, 1)
        return res

    run(1000.0, 20, 0.0, warm=True)
    rates = [float(x) for x in args.serve_rates.split(",") if x.strip()]
    sweep = []
    for r in rates:
        rec = run(r, args.serve_queries, args.serve_build_rate)
        log(f"serving at {r:g} queries/s + {args.serve_build_rate:g} builds/s: query p50 "
            f"{rec['query']['latency_ms_p50']} ms, p99 {rec['query']['latency_ms_p99']} ms; "
            f"build p50 {rec.get('build', {}).get('latency_ms_p50')} ms; "
            f"{rec['probes_per_s']:.0f} probes/s, {rec['resident_GB_end']} GB resident")
        sweep.append(rec)
    srv.close()
    del srv, ws, wsb, live, free_bufs, pools, kinds
    torch.cuda.synchronize()
    return {"resident": f"{len(fill)} S-matrices at the start ({resident0 / 1e9:.1f} GB; budget "
                        f"{budget / 1e9:.0f} GB, LRU eviction): random specimens on 2048^2 and "
                        f"1024^2 grids at f = 4, 8 and fcc1024 at f = 4, 8, 16",
            "queries": "Poisson arrivals, probes per query log-uniform in [64, 65536], "
                       "a run of the (n/4)^2 scan raster in probe-tile order",
            "builds": f"Poisson arrivals at {args.serve_build_rate:g}/s, n in {{512, 1024, "
                      f"2048}}, f in {{4, 8, 16}}, admitted by the server's byte budget",
            "slots": f"{n_streams} query streams (first free slot, one call in flight each; "
                     f"queries arriving meanwhile merge into the next call) + 1 build stream",
            "sweep": sweep}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU (sharding over several is a design only); --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from synth import build_inputs
    from paper_1702_01904_amd import Plan, tile_order, untile

    dev = torch.device("cuda:0")
    if args.calibration_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 256 MiB read + 256 MiB written")
        del src, dst
    t_setup = time.perf_counter()
    d = build_inputs(CONFIG, args.seed)
    N, H, P = d["n"], d["phase"].shape[0], len(d["probes"])
    log(f"inputs ready ({time.perf_counter() - t_setup:.1f} s): N={N} H={H} P={P}")
    plan = Plan(N, d["cell"], d["energy_keV"], d["thickness"])
    phase = torch.from_numpy(d["phase"]).to(dev)
    plan.set_potential_slices(phase)
    optics, edges = d["optics"], d["edges"]
    n_det = edges.shape[0]

    def setup_f(f):
        amax = plan.alpha_max_default(optics["alpha_mrad"], f)
        B = plan.beam_count(f, amax)
        S = torch.empty((B, N // 2, N // 2), dtype=torch.complex64, device=dev)
        wsb = torch.empty(plan.build_workspace_bytes(f, amax)[0], dtype=torch.uint8, device=dev)
        wsp = torch.empty(plan.probe_workspace_bytes(f, amax, optics)[0], dtype=torch.uint8,
                          device=dev)
        _, tx, ty = plan.probe_group(f)
        perm = tile_order(256, 256, tx, ty)
        xy = torch.from_numpy(d["probes"][perm]).to(dev)
        out = torch.empty((P, n_det), dtype=torch.float64, device=dev)
        ba = plan.active_beam_count(f, amax, optics)
        return dict(f=f, amax=amax, B=B, BA=ba, S=S, wsb=wsb, wsp=wsp, perm=perm, xy=xy, out=out)

    def step(c):
        plan.build_smatrix(c["f"], c["amax"], c["S"], c["wsb"])
        plan.probe_outputs(c["f"], c["amax"], c["S"], c["xy"], optics, edges, c["out"], c["wsp"])

    def timed(c, steps, warmup, profile):
        for i in range(warmup):
            step(c)
            torch.cuda.synchronize()
            log(f"f={c['f']} warmup {i + 1}/{warmup} done")
        if profile:
            plan.profile(True)
        torch.cuda.synchronize()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        evs[0].record()
        for i in range(steps):
            step(c)
            evs[i + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        prof = plan.profile_report() if profile else None
        plan.profile(False)
        ms = evs[0].elapsed_time(evs[-1]) / steps
        per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
        log(f"f={c['f']} timed {steps} steps: {ms:.2f} ms/step (wall {wall:.2f} s)")
        timed.median = float(np.median(per))
        return ms, prof

    # The headline steps run as a user runs them. The per-kernel HIP events
    # (two per launch, about 1,600 per step) add gaps between launches, so
    # the kernel breakdown and the roofline come from the same steps run
    # again, back to back, with the events on.
    main_c = setup_f(args.f)
    ms, _ = timed(main_c, args.steps, args.warmup, False)
    ms_median = timed.median
    ms_events, prof = timed(main_c, args.steps, 0, True)
    value = P / (ms * 1e-3)
    geo = dict(N=N, NS=N // 2, H=H, B=main_c["B"], BA=main_c["BA"], P=P, W=N // (2 * args.f),
               n_det=n_det)
    dom, roof = roofline(prof, geo, args.steps)
    kernels = {k: round(v["total_ms"] / args.steps, 3) for k, v in prof.items()}
    out_main = untile(main_c["out"].cpu().numpy(), main_c["perm"])
    finite = bool(np.all(np.isfinite(out_main)))
    half_band = plan.wavelength / d["cell"] * (N / 4) * 1e3   # mrad

    def vs_golden(f, D, prec="fp32"):
        g = golden(f"{CONFIG}_prism_f{f}.txt")
        return None if g is None else accuracy(D[g[0]], g[1], edges, half_band, floor_of(prec))

    accuracy_fp64 = {f"f{args.f}_fp32": vs_golden(args.f, out_main)}
    prism_out = {args.f: out_main}

    # probe-side variants at the headline f: probe step alone on a resident
    # S-matrix, full CBED output, and frozen-phonon averaging (one S-matrix
    # build per configuration, outputs accumulated with weight 1/K)
    probe_side = None
    if args.phonon_configs > 0:
        from synth import phonon_configurations
        c = main_c

        def ev_time(fn, reps):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps

        ms_res = ev_time(lambda: plan.probe_outputs(c["f"], c["amax"], c["S"], c["xy"], optics,
                                                    edges, c["out"], c["wsp"]), args.steps)
        ms_build = ev_time(lambda: plan.build_smatrix(c["f"], c["amax"], c["S"], c["wsb"]),
                           args.steps)
        log(f"resident-S probe step: {ms_res:.2f} ms")
        W = N // (2 * args.f)
        cb = torch.empty((P, W, W), dtype=torch.float32, device=dev)
        ms_cb = ev_time(lambda: plan.probe_cbed(c["f"], c["amax"], c["S"], c["xy"], optics, cb,
                                                c["wsp"]), args.steps)
        del cb
        log(f"CBED probe step: {ms_cb:.2f} ms")
        K = args.phonon_configs
        ph = phonon_configurations(CONFIG, args.seed, K)
        phases = [torch.from_numpy(x).to(dev) for x in ph["phase_configs"]]
        jitter = ph["jitter_A"]
        del ph
        acc = torch.zeros((P, n_det), dtype=torch.float64, device=dev)

        def phonon_run():
            acc.zero_()
            for x in phases:
                plan.set_potential_slices(x)
                plan.build_smatrix(c["f"], c["amax"], c["S"], c["wsb"])
                plan.probe_outputs_accumulate(c["f"], c["amax"], c["S"], c["xy"], optics, edges,
                                              1.0 / K, acc, c["wsp"])

        ms_ph = ev_time(phonon_run, 1)
        plan.set_potential_slices(phase)
        torch.cuda.synchronize()
        del phases, acc
        log(f"frozen phonons, {K} configurations: {ms_ph:.2f} ms")
        probe_side = {
            "phases_ms": {"build": round(ms_build, 3), "probe_step": round(ms_res, 3),
                          "end_to_end": round(ms, 3)},
            "resident_smatrix": {"ms": round(ms_res, 3), "probes_per_s": round(P / (ms_res * 1e-3), 1)},
            "cbed": {"ms": round(ms_cb, 3), "probes_per_s": round(P / (ms_cb * 1e-3), 1),
                     "window": W, "bytes_out": P * W * W * 4},
            "frozen_phonon": {"configs": K, "ms": round(ms_ph, 3),
                              "probes_per_s": round(P / (ms_ph * 1e-3), 1),
                              "jitter_A": jitter},
        }
    del main_c

    # 16-bit window sums at the headline f (tolerance eps_rel <= 1e-2)
    variants = {}
    for prec in [x.strip() for x in args.precisions.split(",") if x.strip()]:
        plan.set_probe_precision(prec)
        c = setup_f(args.f)
        msv, _ = timed(c, args.steps, 1, False)
        accuracy_fp64[f"f{args.f}_{prec}"] = vs_golden(
            args.f, untile(c["out"].cpu().numpy(), c["perm"]), prec)
        msv_events, pv = timed(c, args.steps, 0, True)
        _, rv = roofline(pv, geo, args.steps, "contract16")
        variants[prec] = {"ms_per_step": round(msv, 3), "probes_per_s": round(P / (msv * 1e-3), 1),
                          "ms_per_step_with_kernel_events": round(msv_events, 3),
                          "kernel_ms_per_step": {k: round(v["total_ms"] / args.steps, 3)
                                                 for k, v in pv.items()},
                          "contract16_roofline": rv,
                          "tolerance": "eps_rel <= 1e-2 vs FP64 oracle"}
        plan.set_probe_precision("fp32")
        del c

    per_f = {}
    for f in [int(x) for x in args.other_f.split(",") if x.strip()]:
        c = setup_f(f)
        msf, _ = timed(c, max(1, args.steps), 1, False)
        prism_out[f] = untile(c["out"].cpu().numpy(), c["perm"])
        accuracy_fp64[f"f{f}_fp32"] = vs_golden(f, prism_out[f])
        per_f[str(f)] = {"ms_per_step": round(msf, 3), "probes_per_s": round(P / (msf * 1e-3), 1),
                         "beams": c["B"], "active_beams": c["BA"]}
        del c

    prec2048 = run_precision_np2048(args, dev) if args.np2048 else None
    batch = run_batch(args, dev) if args.batch else None

    serving = run_serving(args, plan, d, dev) if args.serve_rates else None

    # multislice baseline on the same GPU, seeded probe subset
    multi_rate = None
    method_err = None
    if args.ms_probes > 0:
        # the golden multislice probes first, then seeded others
        gm = golden(f"{CONFIG}_multislice.txt")
        first = gm[0][:args.ms_probes] if gm is not None else np.zeros(0, dtype=np.int64)
        rng = np.random.default_rng(args.seed + 7)
        rest = rng.permutation(np.setdiff1d(np.arange(P), first))[:args.ms_probes - len(first)]
        ms_idx = np.concatenate([first, rest])
        sub = d["probes"][ms_idx]
        xy_ms = torch.from_numpy(sub).to(dev)
        out_ms = torch.empty((len(sub), n_det), dtype=torch.float64, device=dev)
        ws_ms = torch.empty(plan.multislice_workspace_bytes(n_det)[0], dtype=torch.uint8,
                            device=dev)
        plan.multislice_outputs(xy_ms[:8], optics, edges, out_ms, ws_ms)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.multislice_outputs(xy_ms, optics, edges, out_ms, ws_ms)
        e1.record()
        torch.cuda.synchronize()
        ms_multi = e0.elapsed_time(e1)
        multi_rate = len(sub) / (ms_multi * 1e-3)
        log(f"multislice: {len(sub)} probes in {ms_multi:.1f} ms -> {multi_rate:.1f} probes/s")
        D_ms = out_ms.cpu().numpy()
        if len(first):
            accuracy_fp64["multislice_fp32"] = accuracy(D_ms[:len(first)], gm[1][:len(first)],
                                                        edges, half_band, floor_of("multislice"))
        method_err = {f"f{f}": method_error(D[ms_idx], D_ms, edges, half_band)
                      for f, D in sorted(prism_out.items())}

    peaks = None
    if not args.no_peaks:
        peaks = measured_peaks(dev)
        log(f"measured peaks: {peaks}")
        mp = peaks["copy_GBps"] if roof["unit"] == "GB/s" else peaks["gemm_fp32_TFLOPs"]
        roof["measured_peak"] = mp
        roof["frac_of_measured"] = round(roof["achieved"] / mp, 4)
        for v in variants.values():   # 16-bit window sums against the BF16 library GEMM
            rv = v["contract16_roofline"]
            rv["measured_peak"] = peaks["gemm_bf16_TFLOPs"]
            rv["frac_of_measured"] = round(rv["achieved"] / peaks["gemm_bf16_TFLOPs"], 4)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample ...")
        cpu = cpu_baseline(d, args.f, plan.alpha_max_default(optics["alpha_mrad"], args.f), P)
        log(f"oracle: {cpu['value']} probes/s on {cpu['cores']} cores ({cpu['host_cpu']}, "
            f"os.cpu_count() = {cpu['os_cpu_count']})")

    rec = {
        "metric": "STEM probe positions/s, PRISM vs multislice, 1 GPU, at stated rel. error",
        "value": round(value, 1),
        "unit": "probes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "ms_per_step_median": round(ms_median, 3),
        "ms_per_step_with_kernel_events": round(ms_events, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{CONFIG}: Au FCC 40x40x100 A, 1024^2 grid, 50 slices, 200 keV, "
                               f"25 mrad, 256x256 scan, 16 bins; PRISM f={args.f} "
                               f"(S-matrix build + all probes)",
                   "f": args.f, "grid": N, "slices": H, "probes": P,
                   "beams": geo["B"], "active_beams": geo["BA"], "window": geo["W"],
                   "tolerance": "eps_rel <= 1e-4 (FP32), 1e-2 (BF16/FP16) vs the FP64 oracle; "
                                "measured on the timed outputs: accuracy_vs_fp64_oracle"},
        "multislice_probes_per_s": round(multi_rate, 2) if multi_rate else None,
        "speedup_vs_gpu_multislice": round(value / multi_rate, 2) if multi_rate else None,
        "speedup_vs_gpu_multislice_per_f": (
            {str(args.f): round(value / multi_rate, 2),
             **{k: round(v["probes_per_s"] / multi_rate, 2) for k, v in per_f.items()}}
            if multi_rate else None),
        "accuracy_vs_fp64_oracle": accuracy_fp64,
        "prism_vs_multislice_method_error": method_err,
        "per_f": per_f,
        "precision_variants": variants,
        "probe_side": probe_side,
        "precision_np2048": prec2048,
        "batch": batch,
        "serving": serving,
        "kernel_ms_per_step": kernels,
        "roofline": roof,
        "measured_peaks": peaks,
        "cpu_baseline": cpu,
        "outputs_finite": finite,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
