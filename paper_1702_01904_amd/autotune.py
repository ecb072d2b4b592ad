"""Launch-shape sweep for libprism on the local GPU (prism_set_tuning).

For every supported grid side n it times, with HIP events, the S-matrix
build and the probe step of a seeded synthetic specimen (random phase
slices, 0.1 A pixels, 80 keV, 20 mrad, 8 slices of 2 A; the (n/4)^2 probe
raster at two S-matrix pixels in probe-tile order) under candidate launch
shapes, one parameter at a time (each starting from the best found so far):

  build: row_iters, row_min_groups, col_iters, col_min_groups (the four-step
         slice passes, n = 256 and 1024), wave_chunk_mib (every n);
  probe: probe_group, window_tile_div.

A candidate is kept only if its S-matrix and probe outputs equal the default
shapes' bit for bit (none of these shapes may change a result). The winners
go to tuning_gfx950.json beside this file, which Plan applies when it is
created for that n.

Usage (on the GPU): python -m paper_1702_01904_amd.autotune [--out PATH] [--n 256,1024]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning_gfx950.json")
GRIDS = (128, 192, 256, 384, 512, 576, 768, 1024, 1152, 1536, 2048)
FIELDS = ("row_iters", "row_min_groups", "col_iters", "col_min_groups", "wave_chunk_mib",
          "probe_group", "window_tile_div")
BUILD_SWEEP = [("row_iters", (2, 4, 8, 16, 32)), ("row_min_groups", (128, 256, 512, 1024)),
               ("col_iters", (2, 4, 8, 16)), ("col_min_groups", (128, 256, 512, 1024)),
               ("wave_chunk_mib", (64, 128, 256, 512))]
PROBE_SWEEP = [("probe_group", (16, 32, 64)), ("window_tile_div", (1, 2, 4, 8))]
FOUR_STEP = (256, 1024)


def interp_factor(n):
    """A factor with a window of 16 .. 128 pixels, 4 where the grid allows."""
    for f in (4, 8, 6, 3, 2, 16, 12):
        if n % (2 * f) == 0 and 16 <= n // (2 * f) <= 128:
            return f
    return 1


def time_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_grid(n, log):
    import torch
    from . import Plan, tile_order
    dev = torch.device("cuda:0")
    H = 8
    plan = Plan(n, 0.1 * n, 80.0, np.full(H, 2.0))
    rng = np.random.default_rng(n)
    phase = torch.from_numpy(rng.uniform(0.0, 0.5, (H, n, n)).astype(np.float32)).to(dev)
    plan.set_potential_slices(phase)
    f = interp_factor(n)
    optics = dict(alpha_mrad=20.0)
    edges = [(0.0, 20.0), (20.0, 40.0), (40.0, 100.0)]
    amax = plan.alpha_max_default(20.0, f)
    B = plan.beam_count(f, amax)
    S = torch.empty((B, n // 2, n // 2), dtype=torch.complex64, device=dev)
    n4 = n // 4
    step = plan.cell / n4
    i = np.arange(n4, dtype=np.float64) * step
    ras = np.stack([np.tile(i, n4), np.repeat(i, n4)], axis=1)
    out = torch.empty((len(ras), len(edges)), dtype=torch.float64, device=dev)

    def run(tune, what):
        plan.set_tuning(tune)
        if what == "build":
            ws = torch.empty(plan.build_workspace_bytes(f, amax)[0], dtype=torch.uint8, device=dev)
            ms = time_ms(lambda: plan.build_smatrix(f, amax, S, ws), 3)
            return ms, S.clone()
        _, tx, ty = plan.probe_group(f)
        perm = tile_order(n4, n4, tx, ty)
        xy = torch.from_numpy(np.ascontiguousarray(ras[perm])).to(dev)
        ws = torch.empty(plan.probe_workspace_bytes(f, amax, optics)[0], dtype=torch.uint8,
                         device=dev)
        ms = time_ms(lambda: plan.probe_outputs(f, amax, S, xy, optics, edges, out, ws), 5)
        res = torch.empty_like(out)
        res[torch.from_numpy(perm).to(dev)] = out
        return ms, res

    best = {k: 0 for k in FIELDS}
    plan.set_tuning(best)
    defaults = plan.tuning()
    ref_ms, ref_S = run(best, "build")
    base_build = ref_ms
    sweeps = [s for s in BUILD_SWEEP if n in FOUR_STEP or s[0] == "wave_chunk_mib"]
    for name, values in sweeps:
        for v in values:
            cand = dict(best, **{name: v})
            ms, Sc = run(cand, "build")
            same = bool(torch.equal(Sc, ref_S))
            log(f"n={n} f={f} build {name}={v}: {ms:.3f} ms{'' if same else ' (differs: dropped)'}")
            if same and ms < ref_ms:
                ref_ms, best = ms, cand
    plan.set_tuning(best)
    plan.build_smatrix(f, amax, S, torch.empty(plan.build_workspace_bytes(f, amax)[0],
                                               dtype=torch.uint8, device=dev))
    ref_pms, ref_out = run(best, "probe")
    base_probe = ref_pms
    for name, values in PROBE_SWEEP:
        for v in values:
            cand = dict(best, **{name: v})
            ms, oc = run(cand, "probe")
            same = bool(torch.equal(oc, ref_out))
            log(f"n={n} f={f} probe {name}={v}: {ms:.3f} ms{'' if same else ' (differs: dropped)'}")
            if same and ms < ref_pms:
                ref_pms, best = ms, cand
    plan.set_tuning(best)
    eff = plan.tuning()
    del S, phase
    torch.cuda.synchronize()
    return {"tuning": eff, "defaults": defaults, "f": f, "beams": B,
            "build_ms": [round(base_build, 4), round(ref_ms, 4)],
            "probe_ms": [round(base_probe, 4), round(ref_pms, 4)]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--n", default=",".join(str(n) for n in GRIDS))
    args = ap.parse_args()

    def log(msg):
        print("[autotune]", msg, file=sys.stderr, flush=True)

    table = {"gpu": None, "written": time.strftime("%Y-%m-%d"), "grids": {}}
    import torch
    table["gpu"] = torch.cuda.get_device_name(0)
    for n in (int(x) for x in args.n.split(",") if x.strip()):
        r = tune_grid(n, log)
        table["grids"][str(n)] = r
        log(f"n={n}: build {r['build_ms'][0]} -> {r['build_ms'][1]} ms, probe "
            f"{r['probe_ms'][0]} -> {r['probe_ms'][1]} ms, {r['tuning']}")
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    print(args.out)


if __name__ == "__main__":
    main()
