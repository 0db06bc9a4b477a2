"""Seeded synthetic atomic systems shaped like the paper's benchmark workloads.

The paper benchmarks bulk Ag, liquid water and a high-entropy alloy from public
DFT sets (Sec. 4.1); none of those are used here.  These generators produce
stand-ins of the same kind: jittered periodic water boxes (the water workload)
and jittered FCC crystals with a Cu-like lattice constant (the Ag workload).

This module only draws positions, species, cells and velocities.  It holds none
of the model's arithmetic and is imported by both the oracle tests and the GPU
path, which is the only code they share.

Every system is returned as a dict with keys
    pos     float64 [n, 3]  Cartesian positions in Angstrom
    species int32   [n]     index into ``elements``
    cell    float64 [3, 3]  row-major lattice vectors (orthorhombic: diagonal)
    pbc     int32   [3]     1 = periodic along that axis
    elements list[str]
"""
from __future__ import annotations

import math

import numpy as np

# Density of the 64-molecule reference box: 64 molecules in a 12.42 A cube.
WATER_BOX_L = 12.42
WATER_MOL_DENSITY = 64.0 / WATER_BOX_L ** 3
R_OH = 0.96
ANGLE_HOH_DEG = 104.5
FCC_A = 3.61

MASS_AMU = {"H": 1.008, "O": 15.999, "Cu": 63.546}


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotation matrices from uniform unit quaternions."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_from_sites(rng, sites: np.ndarray, sigma: float) -> np.ndarray:
    """Place one molecule per O site: O jittered by N(0, sigma^2) per axis,
    two H at R_OH with the H-O-H angle, orientation uniformly random."""
    nm = sites.shape[0]
    o = sites + rng.normal(scale=sigma, size=sites.shape)
    half = math.radians(ANGLE_HOH_DEG) / 2.0
    body = np.array([[math.sin(half), 0.0, math.cos(half)],
                     [-math.sin(half), 0.0, math.cos(half)]]) * R_OH
    R = _random_rotations(rng, nm)
    h = np.einsum("mij,kj->mki", R, body)  # [nm, 2, 3]
    pos = np.empty((nm, 3, 3))
    pos[:, 0] = o
    pos[:, 1] = o + h[:, 0]
    pos[:, 2] = o + h[:, 1]
    return pos.reshape(-1, 3)


def water_box(grid=(4, 4, 4), spacing: float = WATER_BOX_L / 4, sigma: float = 0.2,
              seed: int = 0) -> dict:
    """Periodic water box: one molecule per site of a grid of ``grid`` sites at
    ``spacing`` (sites at (i+1/2)*spacing), O jittered by sigma, random
    orientation.  The default is the 64-molecule, 12.42 A cubic box (192 atoms).
    Atom order is (O, H, H) per molecule; elements are ("H", "O")."""
    rng = np.random.default_rng(seed)
    gx, gy, gz = grid
    idx = np.stack(np.meshgrid(np.arange(gx), np.arange(gy), np.arange(gz), indexing="ij"),
                   axis=-1).reshape(-1, 3)
    sites = (idx + 0.5) * spacing
    pos = _water_from_sites(rng, sites, sigma)
    nm = sites.shape[0]
    species = np.tile(np.array([1, 0, 0], dtype=np.int32), nm)
    cell = np.diag([gx * spacing, gy * spacing, gz * spacing]).astype(np.float64)
    return dict(pos=pos, species=species, cell=cell, pbc=np.ones(3, np.int32),
                elements=["H", "O"])


def water_box_n(n_atoms: int, sigma: float = 0.2, seed: int = 0) -> dict:
    """Cubic water box of about ``n_atoms`` atoms at the reference density.

    n_mol = max(1, round(n_atoms/3)).  A k^3 site grid (k = ceil(n_mol^(1/3)))
    is laid over a cube whose volume gives the reference molecular density, and
    n_mol of its sites are chosen by a seeded permutation."""
    rng = np.random.default_rng(seed)
    n_mol = max(1, int(round(n_atoms / 3)))
    k = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    L = (n_mol / WATER_MOL_DENSITY) ** (1.0 / 3.0)
    spacing = L / k
    idx = np.stack(np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij"),
                   axis=-1).reshape(-1, 3)
    chosen = np.sort(rng.permutation(idx.shape[0])[:n_mol])
    sites = (idx[chosen] + 0.5) * spacing
    pos = _water_from_sites(rng, sites, sigma)
    species = np.tile(np.array([1, 0, 0], dtype=np.int32), n_mol)
    return dict(pos=pos, species=species, cell=np.diag([L, L, L]).astype(np.float64),
                pbc=np.ones(3, np.int32), elements=["H", "O"])


def fcc_crystal(cells=(30, 30, 28), a: float = FCC_A, sigma: float = 0.1, seed: int = 0) -> dict:
    """Periodic FCC crystal of nx*ny*nz conventional cells (4 atoms each) with
    lattice constant ``a`` and Gaussian displacements N(0, sigma^2) per axis.
    The default is the 100,800-atom Cu-like crystal.  Elements are ("Cu",)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = cells
    basis = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])
    idx = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"),
                   axis=-1).reshape(-1, 1, 3)
    pos = ((idx + basis[None]) * a).reshape(-1, 3)
    pos = pos + rng.normal(scale=sigma, size=pos.shape)
    return dict(pos=pos, species=np.zeros(pos.shape[0], np.int32),
                cell=np.diag([nx * a, ny * a, nz * a]).astype(np.float64),
                pbc=np.ones(3, np.int32), elements=["Cu"])


def fcc_n(n_atoms: int, a: float = FCC_A, sigma: float = 0.1, seed: int = 0) -> dict:
    """Near-cubic FCC crystal with 4*nx*ny*nz close to ``n_atoms`` (at least 4)."""
    ncell = max(1, int(round(n_atoms / 4)))
    best = None
    base = max(1, int(round(ncell ** (1.0 / 3.0))))
    for nx in range(max(1, base - 2), base + 3):
        for ny in range(nx, base + 4):
            nz = max(1, int(round(ncell / (nx * ny))))
            err = abs(nx * ny * nz - ncell) + 0.01 * (max(nx, ny, nz) - min(nx, ny, nz))
            if best is None or err < best[0]:
                best = (err, (nx, ny, nz))
    return fcc_crystal(best[1], a=a, sigma=sigma, seed=seed)


def remap_species(system: dict, elements: list[str]) -> dict:
    """Re-express ``system['species']`` as indices into ``elements``."""
    table = np.array([elements.index(e) for e in system["elements"]], dtype=np.int32)
    out = dict(system)
    out["species"] = table[system["species"]]
    out["elements"] = list(elements)
    return out


def maxwell_boltzmann(species: np.ndarray, elements: list[str], temperature_K: float = 300.0,
                      seed: int = 0) -> np.ndarray:
    """Velocities in A/fs drawn from the Maxwell-Boltzmann distribution."""
    rng = np.random.default_rng(seed)
    kB = 8.617333262e-5  # eV/K
    # 1 eV/amu = 9.648533e-3 A^2/fs^2
    m = np.array([MASS_AMU[elements[s]] for s in species])
    sd = np.sqrt(kB * temperature_K / m * 9.648533212e-3)
    return rng.normal(size=(species.shape[0], 3)) * sd[:, None]


def serving_mix(n_systems: int = 256, n_min: int = 64, n_max: int = 20000, seed: int = 0,
                elements=("H", "O", "Cu")) -> list[dict]:
    """Independent systems for the serving stream: sizes log-uniform in
    [n_min, n_max], even indices water boxes and odd indices FCC crystals, each
    with its own seed, species expressed over ``elements``."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(math.log(n_min), math.log(n_max), size=n_systems))
    out = []
    for k, n in enumerate(sizes):
        s = int(rng.integers(1 << 30))
        sys = water_box_n(int(n), seed=s) if k % 2 == 0 else fcc_n(int(n), seed=s)
        out.append(remap_species(sys, list(elements)))
    return out
