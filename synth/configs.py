"""Workload definitions (plain data; no simulation arithmetic).

Each entry fixes the specimen recipe, the sampling grid, the optics, the
probe scan and the detector bins. The parameter ranges follow the paper's
experiments: 80 kV with 2 A slices and 0.1 A pixels (Section "Simulation
and Analysis Implementation"), 20-25 mrad probes (Fig. 3 and Fig. 4
captions), interpolation factors 2-20 (Eq. TimeRatio discussion and
Fig. 4).
"""
import copy

CONFIGS = {
    # Tiny plain-method case: the oracle finishes every path in seconds.
    "tiny": dict(
        specimen=dict(kind="random", cell=(12.8, 12.8, 8.0), n_atoms=20,
                      z_choices=(6, 14, 29, 79)),
        n=128, n_slices=4, slice_A=2.0,
        energy_keV=80.0,
        optics=dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0),
        scan=dict(nx=16, ny=16, step_A=0.8, origin_A=(0.0, 0.0)),
        detectors=[(40.0, 150.0)],
        f_values=(1, 2),
    ),
    # Headline throughput case: one Au FCC specimen on a 1024^2 grid.
    "fcc1024": dict(
        specimen=dict(kind="fcc", cell=(40.0, 40.0, 100.0), a_A=4.08, Z=79,
                      jitter_A=0.08),
        n=1024, n_slices=50, slice_A=2.0,
        energy_keV=200.0,
        optics=dict(alpha_mrad=25.0, C1_A=0.0, C3_A=0.0),
        scan=dict(nx=256, ny=256, step_A=0.15625, origin_A=(0.0, 0.0)),
        detectors=[(12.5 * j, 12.5 * (j + 1)) for j in range(16)],
        f_values=(4, 8, 16),
    ),
    # Mid-size parity case: several FFT/contraction tiles, a ragged probe
    # count, oracle time of a few seconds.
    "mid256": dict(
        specimen=dict(kind="random", cell=(25.6, 25.6, 16.0), n_atoms=150,
                      z_choices=(6, 14, 29, 79)),
        n=256, n_slices=8, slice_A=2.0,
        energy_keV=80.0,
        optics=dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0),
        scan=dict(nx=19, ny=7, step_A=0.4, origin_A=(3.0, 9.2)),
        detectors=[(0.0, 20.0), (20.0, 40.0), (40.0, 80.0), (80.0, 150.0)],
        f_values=(1, 2, 4),
    ),
    # 512^2 case (the radix-8/2 Stockham slice kernels, windows of 128 and
    # 64 at f = 2 and 4); sampled against one-probe oracle runs.
    "s512": dict(
        specimen=dict(kind="random", cell=(51.2, 51.2, 12.0), n_atoms=400,
                      z_choices=(6, 14, 29, 79)),
        n=512, n_slices=6, slice_A=2.0,
        energy_keV=80.0,
        optics=dict(alpha_mrad=20.0, C1_A=10.0, C3_A=0.0),
        scan=dict(nx=24, ny=24, step_A=0.2, origin_A=(20.0, 20.0)),
        detectors=[(0.0, 20.0), (20.0, 50.0), (50.0, 100.0)],
        f_values=(2, 4),
    ),
    # Grids with a factor 3 (radix-3 FFT stages): 192^2 and 384^2 with
    # 0.1 A pixels; windows stay powers of two at f = 3, 6, 12.
    "tiny192": dict(
        specimen=dict(kind="random", cell=(19.2, 19.2, 8.0), n_atoms=30,
                      z_choices=(6, 14, 29, 79)),
        n=192, n_slices=4, slice_A=2.0,
        energy_keV=80.0,
        optics=dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0),
        scan=dict(nx=12, ny=12, step_A=1.6, origin_A=(0.0, 0.0)),
        detectors=[(0.0, 20.0), (40.0, 100.0)],
        f_values=(3, 6),
    ),
    "mid384": dict(
        specimen=dict(kind="random", cell=(38.4, 38.4, 12.0), n_atoms=160,
                      z_choices=(6, 14, 29, 79)),
        n=384, n_slices=6, slice_A=2.0,
        energy_keV=80.0,
        optics=dict(alpha_mrad=20.0, C1_A=20.0, C3_A=0.0),
        scan=dict(nx=17, ny=9, step_A=0.8, origin_A=(5.0, 5.0)),
        detectors=[(0.0, 20.0), (20.0, 50.0), (50.0, 100.0)],
        f_values=(3, 6, 12),
    ),
    # Precision case (nanoparticle on an amorphous carbon slab, 2048^2).
    "np2048": dict(
        specimen=dict(kind="np_on_carbon", cell=(80.0, 80.0, 70.0),
                      np_radius_A=20.0, a_A=4.08, Z=79, slab_A=30.0,
                      carbon_density=0.1, min_spacing_A=1.4),
        n=2048, n_slices=35, slice_A=2.0,
        energy_keV=80.0,
        optics=dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0),
        scan=dict(kind="disc", n_probes=1024),
        detectors=[(40.0, 150.0)],
        f_values=(4, 8),
    ),
}

# Mixed batches of specimens (many small and large specimens built
# together). Each entry is a recipe for ``batch_workload``: grid sizes with
# 0.1 A pixels, slice counts drawn uniformly, interpolation factors drawn
# among those the grid admits (n divisible by 2 f, windows of at least 8
# pixels), random atoms at 0.015 A^-3.
BATCHES = {
    # 32 specimens on 2^k, 3 * 2^k and 9 * 2^k grids, 20-120 slices, f in
    # {4, 6, 8, 12, 16}.
    "batch32": dict(count=32, sizes=(256, 384, 512, 576, 768, 1024, 1152, 1536),
                    h_range=(20, 120), f_choices=(4, 6, 8, 12, 16),
                    pixel_A=0.1, density=0.015, slice_A=2.0, energy_keV=80.0,
                    optics=dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0),
                    detectors=[(0.0, 20.0), (20.0, 40.0), (40.0, 100.0)],
                    z_choices=(6, 14, 29, 79)),
    # Small mix for parity against the oracle.
    "batch_small": dict(count=6, sizes=(128, 192, 256), h_range=(2, 6), f_choices=(1, 2, 3, 4, 6),
                        pixel_A=0.1, density=0.015, slice_A=2.0, energy_keV=80.0,
                        optics=dict(alpha_mrad=20.0, C1_A=0.0, C3_A=0.0),
                        detectors=[(0.0, 20.0), (20.0, 40.0), (40.0, 100.0)],
                        z_choices=(6, 14, 29, 79)),
}


def get_config(name):
    """Return a deep copy of a named workload definition."""
    if name not in CONFIGS:
        raise KeyError(f"unknown workload {name!r}; have {sorted(CONFIGS)}")
    return copy.deepcopy(CONFIGS[name])
