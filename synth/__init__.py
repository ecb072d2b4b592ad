"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package produces *inputs only*: atom lists, projected phase slices,
probe scan positions and detector edges. It holds none of the simulation
method's arithmetic (no propagation, no beams, no FFT of waves); both the
FP64 oracle and the GPU library consume what it returns.

The paper's specimens (a Pt decahedral nanoparticle on amorphous carbon,
a nanoparticle in a nanotube) and its tabulated atomic potentials are not
available, so every specimen here is a seeded synthetic stand-in with the
same shape of workload: 80-200 keV, 20-25 mrad probes, 2 A slices
(Section "Simulation and Analysis Implementation"; Fig. 4 caption).

Projected potentials are given directly as a phase (sigma * V, radians),
each atom a 2D Gaussian of standard deviation 0.3 A and peak phase
0.05 * Z**0.7 rad, summed with minimum-image distances in the periodic
xy cell. The phase is rounded to float32 once here, so the oracle and the
GPU see bit-identical slices.
"""
from .configs import BATCHES, CONFIGS, get_config
from .specimen import (
    random_atoms,
    fcc_atoms,
    nanoparticle_on_carbon,
    phase_slices,
    raster_probes,
    annular_edges,
    build_inputs,
    phonon_configurations,
    batch_workload,
    batch_shapes,
)

__all__ = [
    "CONFIGS",
    "get_config",
    "random_atoms",
    "fcc_atoms",
    "nanoparticle_on_carbon",
    "phase_slices",
    "raster_probes",
    "annular_edges",
    "build_inputs",
    "phonon_configurations",
    "batch_workload",
    "batch_shapes",
    "BATCHES",
]
