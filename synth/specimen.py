"""Seeded specimen, phase-slice, scan and detector generators.

Random draws use ``numpy.random.default_rng(seed)``; for a random specimen
the draw order is x, then y, then z, then atomic number Z. Atoms are cut
into slices of thickness t by floor(z / t) (the slicing of Fig. 1a); atoms
outside [0, H t) are clipped into the first or last slice.
"""
import numpy as np

from .configs import BATCHES, get_config

GAUSS_SIGMA_A = 0.3          # standard deviation of each atom's phase blob


def phase_amplitude(Z):
    """Peak phase shift (rad) of one atom of atomic number Z."""
    return 0.05 * np.asarray(Z, dtype=np.float64) ** 0.7


def random_atoms(cell, n_atoms, z_choices, rng):
    """Uniform random atoms in an orthorhombic cell; returns [n, 4] (x, y, z, Z)."""
    cx, cy, cz = cell
    x = rng.uniform(0.0, cx, n_atoms)
    y = rng.uniform(0.0, cy, n_atoms)
    z = rng.uniform(0.0, cz, n_atoms)
    Z = rng.choice(np.asarray(z_choices), n_atoms)
    return np.stack([x, y, z, Z.astype(np.float64)], axis=1)


def _fcc_sites(a, lo, hi):
    """FCC lattice sites a*(i,j,k)+basis lying in the box [lo, hi)."""
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    imin = np.floor(lo / a).astype(int) - 1
    imax = np.ceil(hi / a).astype(int) + 1
    ii, jj, kk = np.meshgrid(np.arange(imin[0], imax[0]),
                             np.arange(imin[1], imax[1]),
                             np.arange(imin[2], imax[2]), indexing="ij")
    cells = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.float64)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
    keep = np.all((sites >= lo - 1e-9) & (sites < hi - 1e-9), axis=1)
    return sites[keep]


def fcc_atoms(cell, a, Z, jitter, rng):
    """Zone-axis ([001] along the beam) FCC crystal filling the cell.

    Sites a*(i, j, k) + basis are kept inside [0, cx) x [0, cy) x [0, cz);
    each coordinate then gets seeded Gaussian jitter of std ``jitter`` (one
    frozen configuration). Draw order: x jitter, y jitter, z jitter.
    """
    sites = _fcc_sites(a, (0.0, 0.0, 0.0), cell)
    n = sites.shape[0]
    dx = rng.normal(0.0, jitter, n)
    dy = rng.normal(0.0, jitter, n)
    dz = rng.normal(0.0, jitter, n)
    xyz = sites + np.stack([dx, dy, dz], axis=1)
    return np.concatenate([xyz, np.full((n, 1), float(Z))], axis=1)


def nanoparticle_on_carbon(cell, np_radius, a, Z, slab, density, min_spacing, rng):
    """Spherical FCC nanoparticle above an amorphous carbon slab.

    The particle (centre at the cell's xy centre, z = np_radius) is met by
    the beam first; the slab fills z in [cz - slab, cz). Carbon atoms are
    placed by random sequential addition with a minimum spacing, using a
    periodic cell list in x and y.
    """
    cx, cy, cz = cell
    centre = np.array([cx / 2, cy / 2, np_radius])
    sites = _fcc_sites(a, centre - np_radius - a, centre + np_radius + a)
    sites = sites - (sites.mean(axis=0) - centre)
    r = np.linalg.norm(sites - centre, axis=1)
    npart = sites[r <= np_radius]
    atoms = [np.concatenate([npart, np.full((len(npart), 1), float(Z))], axis=1)]

    target = int(round(density * cx * cy * slab))
    z0 = cz - slab
    h = min_spacing
    nbx, nby, nbz = int(cx // h), int(cy // h), max(1, int(slab // h))
    grid = {}
    carbon = []
    tries = 0
    max_tries = 200 * target
    while len(carbon) < target and tries < max_tries:
        tries += 1
        p = np.array([rng.uniform(0, cx), rng.uniform(0, cy), rng.uniform(z0, cz)])
        bx = int(p[0] / cx * nbx) % nbx
        by = int(p[1] / cy * nby) % nby
        bz = min(int((p[2] - z0) / slab * nbz), nbz - 1)
        ok = True
        for ox in (-1, 0, 1):
            for oy in (-1, 0, 1):
                for oz in (-1, 0, 1):
                    key = ((bx + ox) % nbx, (by + oy) % nby, bz + oz)
                    for q in grid.get(key, ()):
                        d = p - q
                        d[0] -= cx * np.round(d[0] / cx)
                        d[1] -= cy * np.round(d[1] / cy)
                        if d @ d < min_spacing * min_spacing:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            grid.setdefault((bx, by, bz), []).append(p)
            carbon.append(p)
    carbon = np.asarray(carbon).reshape(-1, 3)
    atoms.append(np.concatenate([carbon, np.full((len(carbon), 1), 6.0)], axis=1))
    return np.concatenate(atoms, axis=0)


def phase_slices(atoms, cell_xy, n, n_slices, slice_A):
    """Projected phase (rad) of each slice on an n x n grid, float64 [H][n][n].

    Arrays are indexed [y][x]; pixel (i, j) sits at (i d/n, j d/n). Each
    atom adds A_Z exp(-rho^2 / (2 sigma^2)) with rho the minimum-image xy
    distance; the Gaussian is separable, so a slice is GY^T @ GX.
    """
    cx, cy = cell_xy
    if abs(cx - cy) > 1e-12:
        raise ValueError("square cells only")
    d = float(cx)
    xs = np.arange(n, dtype=np.float64) * (d / n)
    out = np.zeros((n_slices, n, n), dtype=np.float64)
    if atoms.shape[0] == 0:
        return out
    sl = np.clip(np.floor(atoms[:, 2] / slice_A).astype(np.int64), 0, n_slices - 1)
    amp = phase_amplitude(atoms[:, 3])
    inv2s2 = 1.0 / (2.0 * GAUSS_SIGMA_A ** 2)
    for p in range(n_slices):
        sel = np.nonzero(sl == p)[0]
        if sel.size == 0:
            continue
        ax = atoms[sel, 0][:, None]
        ay = atoms[sel, 1][:, None]
        dx = np.mod(xs[None, :] - ax + d / 2, d) - d / 2
        dy = np.mod(xs[None, :] - ay + d / 2, d) - d / 2
        gx = np.exp(-dx * dx * inv2s2) * amp[sel][:, None]
        gy = np.exp(-dy * dy * inv2s2)
        out[p] = gy.T @ gx
    return out


def raster_probes(nx, ny, step_A, origin_A=(0.0, 0.0)):
    """Raster scan positions (A), x fastest: probe p = j * nx + i."""
    ox, oy = origin_A
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    X = ox + i[None, :] * step_A
    Y = oy + j[:, None] * step_A
    return np.stack([np.broadcast_to(X, (ny, nx)).ravel(),
                     np.broadcast_to(Y, (ny, nx)).ravel()], axis=1).copy()


def disc_probes(n_probes, centre, radius, rng):
    """Seeded uniform sub-pixel probe positions inside a disc."""
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, n_probes))
    t = rng.uniform(0.0, 2.0 * np.pi, n_probes)
    return np.stack([centre[0] + r * np.cos(t), centre[1] + r * np.sin(t)], axis=1)


def annular_edges(bins):
    """Detector bins as float64 [n_det][2] (inner, outer) in mrad."""
    return np.asarray(bins, dtype=np.float64).reshape(-1, 2)


def make_atoms(cfg, seed):
    spec = cfg["specimen"]
    rng = np.random.default_rng(seed)
    if spec["kind"] == "random":
        return random_atoms(spec["cell"], spec["n_atoms"], spec["z_choices"], rng)
    if spec["kind"] == "fcc":
        return fcc_atoms(spec["cell"], spec["a_A"], spec["Z"], spec["jitter_A"], rng)
    if spec["kind"] == "np_on_carbon":
        return nanoparticle_on_carbon(spec["cell"], spec["np_radius_A"], spec["a_A"],
                                      spec["Z"], spec["slab_A"], spec["carbon_density"],
                                      spec["min_spacing_A"], rng)
    raise ValueError(spec["kind"])


def build_inputs(name_or_cfg, seed=0, n_slices=None):
    """Everything a simulation call needs for one workload and seed.

    Returns a dict with ``phase`` (float32 [H][n][n], rad), ``thickness``
    (float64 [H], A), ``cell`` (A), ``n``, ``energy_keV``, ``optics``,
    ``probes`` (float64 [P][2], A), ``edges`` (float64 [n_det][2], mrad),
    ``f_values`` and ``atoms``. ``n_slices`` optionally truncates H (the
    top slices of the specimen), for quick checks.
    """
    cfg = get_config(name_or_cfg) if isinstance(name_or_cfg, str) else name_or_cfg
    atoms = make_atoms(cfg, seed)
    cell = cfg["specimen"]["cell"]
    H = cfg["n_slices"] if n_slices is None else int(n_slices)
    phase = phase_slices(atoms, cell[:2], cfg["n"], H, cfg["slice_A"]).astype(np.float32)
    scan = cfg["scan"]
    if scan.get("kind") == "disc":
        rng = np.random.default_rng(seed + 1000)
        radius = cfg["specimen"].get("np_radius_A", cell[0] / 4)
        probes = disc_probes(scan["n_probes"], (cell[0] / 2, cell[1] / 2), radius, rng)
    else:
        probes = raster_probes(scan["nx"], scan["ny"], scan["step_A"], scan["origin_A"])
    return dict(
        name=name_or_cfg if isinstance(name_or_cfg, str) else "custom",
        seed=seed,
        atoms=atoms,
        phase=phase,
        thickness=np.full(H, cfg["slice_A"], dtype=np.float64),
        cell=float(cell[0]),
        n=cfg["n"],
        energy_keV=cfg["energy_keV"],
        optics=dict(cfg["optics"]),
        probes=probes,
        edges=annular_edges(cfg["detectors"]),
        f_values=tuple(cfg["f_values"]),
    )


DEFAULT_THERMAL_JITTER_A = 0.08   # rms displacement per Cartesian coordinate


def phonon_configurations(name_or_cfg, seed, n_configs, jitter_A=None, n_slices=None):
    """Frozen-phonon configurations of one specimen (random atomic displacements).

    The undisplaced specimen is the workload's atom list for ``seed`` (an FCC
    crystal on its exact lattice sites); configuration k adds independent
    Gaussian displacements of standard deviation ``jitter_A`` (default: the
    workload's own jitter, else 0.08 A) drawn from
    ``default_rng([seed, k])`` in the order x, y, z. Returns the
    ``build_inputs`` dict of the undisplaced specimen plus ``phase_configs``
    (float32 [K][H][n][n]) and ``atom_configs`` (list of [n_atoms, 4]).
    """
    cfg = get_config(name_or_cfg) if isinstance(name_or_cfg, str) else name_or_cfg
    spec = cfg["specimen"]
    if jitter_A is None:
        jitter_A = spec.get("jitter_A", DEFAULT_THERMAL_JITTER_A)
    base_cfg = dict(cfg, specimen=dict(spec, jitter_A=0.0)) if spec["kind"] == "fcc" else cfg
    d = build_inputs(base_cfg, seed, n_slices)
    d["name"] = name_or_cfg if isinstance(name_or_cfg, str) else "custom"
    cell = spec["cell"]
    H = d["phase"].shape[0]
    base = d["atoms"]
    phases, atoms = [], []
    for k in range(int(n_configs)):
        rng = np.random.default_rng([int(seed), k])
        n = base.shape[0]
        disp = np.stack([rng.normal(0.0, jitter_A, n), rng.normal(0.0, jitter_A, n),
                         rng.normal(0.0, jitter_A, n)], axis=1)
        a = base.copy()
        a[:, :3] += disp
        atoms.append(a)
        phases.append(phase_slices(a, cell[:2], cfg["n"], H, cfg["slice_A"]).astype(np.float32))
    d["phase_configs"] = np.stack(phases)
    d["atom_configs"] = atoms
    d["jitter_A"] = float(jitter_A)
    return d


def _batch_shape(rec, rng):
    n = int(rng.choice(np.asarray(rec["sizes"])))
    H = int(rng.integers(rec["h_range"][0], rec["h_range"][1] + 1))
    def window_ok(f):
        return n % (2 * f) == 0 and n // (2 * f) >= 8
    fs = [f for f in rec["f_choices"] if window_ok(f)]
    return n, H, int(rng.choice(np.asarray(fs)))


def batch_shapes(name_or_recipe, seed=0, count=None):
    """(n, H, f) of every specimen of a batch, without generating atoms."""
    rec = BATCHES[name_or_recipe] if isinstance(name_or_recipe, str) else name_or_recipe
    count = rec["count"] if count is None else int(count)
    return [_batch_shape(rec, np.random.default_rng([int(seed), i])) for i in range(count)]


def batch_workload(name_or_recipe, seed=0, count=None, indices=None):
    """A seeded mixed batch of specimens; returns a list of ``build_inputs``
    dicts, each with its own ``f`` (the interpolation factor drawn for it).

    Per specimen, from ``default_rng([seed, i])``: grid side n from the
    recipe's sizes, slice count H uniform in h_range, f among the recipe's
    factors with n % (2 f) == 0 and n / (2 f) >= 8, then the atoms
    (random, density atoms per A^3 in an n * pixel square cell of
    thickness H * slice). The scan is the (n/4) x (n/4) raster at two
    S-matrix pixels. ``indices`` builds only those specimens of the batch
    (the others are not generated); ``batch_shapes`` lists (n, H, f) of all.
    """
    rec = BATCHES[name_or_recipe] if isinstance(name_or_recipe, str) else name_or_recipe
    count = rec["count"] if count is None else int(count)
    out = []
    for i in (range(count) if indices is None else indices):
        rng = np.random.default_rng([int(seed), i])
        n, H, f = _batch_shape(rec, rng)
        side = n * rec["pixel_A"]
        depth = H * rec["slice_A"]
        n_atoms = int(round(rec["density"] * side * side * depth))
        cfg = dict(
            specimen=dict(kind="random", cell=(side, side, depth), n_atoms=n_atoms,
                          z_choices=tuple(rec["z_choices"])),
            n=n, n_slices=H, slice_A=rec["slice_A"], energy_keV=rec["energy_keV"],
            optics=dict(rec["optics"]),
            scan=dict(nx=n // 4, ny=n // 4, step_A=4 * rec["pixel_A"], origin_A=(0.0, 0.0)),
            detectors=list(rec["detectors"]), f_values=(f,),
        )
        d = build_inputs(cfg, int(rng.integers(0, 2 ** 31)))
        d["name"] = f"{name_or_recipe if isinstance(name_or_recipe, str) else 'batch'}[{i}]"
        d["f"] = f
        out.append(d)
    return out

