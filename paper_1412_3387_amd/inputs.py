"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module only builds starting configurations (lattices, random
positions, Maxwell velocities, chain topologies, the per-subdomain split of a
box).  It holds none of the method's arithmetic: no forces, no neighbour
search, no integration.  Every generator is a pure function of its seeds and
returns plain numpy arrays (FP64 positions and velocities, int32 tags and
bond partners), so both sides of a parity test can be fed the same bytes.

The paper's own benchmark inputs are not available; these generators stand in
for its Lennard-Jones liquids (Sec. 6, Sec. 8.3), DPD fluid (Sec. 9) and
bead-spring polymers (Sec. 7) at the shapes of the workloads measured here.
Units are LJ reduced units with unit mass.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

LJ_DENSITY = 0.8442
POLYMER_DENSITY = 0.85
DPD_DENSITY = 3.0


@dataclasses.dataclass
class System:
    """One periodic system: positions wrapped into [0, L), velocities, tags."""
    pos: np.ndarray            # (n, 3) float64
    vel: np.ndarray            # (n, 3) float64
    tag: np.ndarray            # (n,) int32, identity of each particle
    L: np.ndarray              # (3,) float64 box lengths
    bonds: Optional[np.ndarray] = None   # (nb, 2) int32 tag pairs
    kind: str = "lj"

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def wrap(pos: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Fold positions into [0, L) (input preparation only)."""
    p = pos - L * np.floor(pos / L)
    p = np.where(p >= L, p - L, p)
    p = np.where(p < 0.0, 0.0, p)
    return p


def maxwell_velocities(n: int, kT: float, seed: int) -> np.ndarray:
    """Gaussian velocities with zero net momentum, rescaled so that the
    kinetic temperature 2 KE / (3n - 3) equals kT exactly (unit mass)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(0.0, math.sqrt(kT), size=(n, 3))
    v -= v.mean(axis=0)
    ke2 = float(np.sum(v * v))           # = 2 KE
    dof = 3 * n - 3
    if ke2 > 0.0 and dof > 0:
        v *= math.sqrt(kT * dof / ke2)
    return v


def fcc_sites(m: int, L: float, offset_frac: float = 0.25) -> np.ndarray:
    """4 m^3 fcc sites in a cube of side L, shifted by offset_frac * a."""
    a = L / m
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0],
                      [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    g = np.arange(m, dtype=np.float64)
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    return (sites + offset_frac) * a


def lj_fluid(n: int, seed_pos: int, seed_vel: int, seed_vac: Optional[int] = None,
             density: float = LJ_DENSITY, T: float = 1.2, noise: float = 0.05) -> System:
    """LJ liquid start: fcc lattice (smallest m with 4 m^3 >= n), seeded
    removal of surplus sites, uniform +-noise displacement, Maxwell
    velocities at T with zero net momentum."""
    L = (n / density) ** (1.0 / 3.0)
    m = 1
    while 4 * m ** 3 < n:
        m += 1
    sites = fcc_sites(m, L)
    surplus = sites.shape[0] - n
    if surplus > 0:
        rv = np.random.Generator(np.random.PCG64(seed_vac if seed_vac is not None else seed_pos + 7919))
        drop = rv.choice(sites.shape[0], size=surplus, replace=False)
        keep = np.ones(sites.shape[0], dtype=bool)
        keep[drop] = False
        sites = sites[keep]
    rp = np.random.Generator(np.random.PCG64(seed_pos))
    pos = sites + rp.uniform(-noise, noise, size=sites.shape)
    Lv = np.array([L, L, L])
    pos = wrap(pos, Lv)
    vel = maxwell_velocities(n, T, seed_vel)
    return System(pos=pos, vel=vel, tag=np.arange(n, dtype=np.int32), L=Lv, kind="lj")


def dpd_fluid(n: int, seed_pos: int, seed_vel: int, density: float = DPD_DENSITY,
              kT: float = 1.0) -> System:
    """DPD fluid start: uniform random positions, Maxwell velocities at kT."""
    L = (n / density) ** (1.0 / 3.0)
    Lv = np.array([L, L, L])
    rp = np.random.Generator(np.random.PCG64(seed_pos))
    pos = wrap(rp.uniform(0.0, L, size=(n, 3)), Lv)
    vel = maxwell_velocities(n, kT, seed_vel)
    return System(pos=pos, vel=vel, tag=np.arange(n, dtype=np.int32), L=Lv, kind="dpd")


def serpentine_sites(k: int) -> np.ndarray:
    """All k^3 sites of a simple-cubic grid in boustrophedon order, so that
    consecutive sites are lattice neighbours."""
    out = []
    row = 0
    for z in range(k):
        ys = range(k) if z % 2 == 0 else range(k - 1, -1, -1)
        for y in ys:
            xs = range(k) if row % 2 == 0 else range(k - 1, -1, -1)
            for x in xs:
                out.append((x, y, z))
            row += 1
    return np.array(out, dtype=np.float64)


def polymer_melt(n_chains: int, seed_vel: int, chain_len: int = 50,
                 density: float = POLYMER_DENSITY, kT: float = 1.0) -> System:
    """Bead-spring melt start: chains laid head to tail along a serpentine
    path through a simple-cubic grid of ceil(n^(1/3)) sites per side, so
    every bond joins grid neighbours; unused sites are left at the path's
    end.  Bonds are (tag, tag + 1) inside each chain."""
    n = n_chains * chain_len
    L = (n / density) ** (1.0 / 3.0)
    k = 1
    while k ** 3 < n:
        k += 1
    h = L / k
    sites = serpentine_sites(k)[:n]
    pos = (sites + 0.5) * h
    Lv = np.array([L, L, L])
    pos = wrap(pos, Lv)
    vel = maxwell_velocities(n, kT, seed_vel)
    b = []
    for c in range(n_chains):
        base = c * chain_len
        for s in range(chain_len - 1):
            b.append((base + s, base + s + 1))
    bonds = np.array(b, dtype=np.int32).reshape(-1, 2)
    return System(pos=pos, vel=vel, tag=np.arange(n, dtype=np.int32), L=Lv,
                  bonds=bonds, kind="polymer")


# ---------------------------------------------------------------------------
# Named workloads (sizes follow the measured configurations)
# ---------------------------------------------------------------------------

def lj_small() -> System:
    """LJ liquid, N = 4,000, density 0.8442, T = 1.2 (50-step FP64 parity run)."""
    return lj_fluid(4000, seed_pos=1, seed_vel=2)


def lj_bulk(n: int = 2_000_000) -> System:
    """LJ bulk liquid, N = 2,000,000 from an fcc 80^3 lattice with 48,000
    seeded vacancies (density 0.8442, T = 1.2)."""
    return lj_fluid(n, seed_pos=21, seed_vel=22, seed_vac=23)


def lj_weak_share(n: int = 32_000) -> System:
    """One GPU's share of the weak-scaling LJ fluid: packing fraction 0.2
    (number density 6 x 0.2 / pi), T = 1.2."""
    return lj_fluid(n, 61, 62, density=6.0 * 0.2 / math.pi)


def dpd_bulk(n: int = 1_000_000) -> System:
    """DPD fluid, N = 1,000,000 at number density 3, kT = 1."""
    return dpd_fluid(n, seed_pos=31, seed_vel=32)


DPD_RNG_SEED = 33


@dataclasses.dataclass
class Subdomains:
    """A periodic box cut into a g x g x g grid of equal cubes."""
    full: System
    grid: int
    side: float
    owner: np.ndarray          # (n,) int32 subdomain index of each particle

    def lo(self, s: int) -> np.ndarray:
        cx, cy, cz = s % self.grid, (s // self.grid) % self.grid, s // (self.grid * self.grid)
        return np.array([cx, cy, cz], dtype=np.float64) * self.side

    def hi(self, s: int) -> np.ndarray:
        return self.lo(s) + self.side

    def local(self, s: int) -> np.ndarray:
        return np.nonzero(self.owner == s)[0]


def stretched_chains(n_side: int = 18, a: float = 1.1, seed_pos: int = 71, seed_vel: int = 72,
                     T: float = 1.0, noise: float = 0.05) -> System:
    """Chains whose bonds are longer than a WCA ghost layer: a simple cubic
    lattice of n_side^3 sites (spacing a); the rows of sites run along x in
    the layers of even z and along y in the others, and each row holds two
    interleaved chains (its even and its odd sites), so consecutive beads of
    a chain are 2a apart.  Seeded +-noise a displacement, Maxwell velocities
    at T."""
    assert n_side % 2 == 0
    L = n_side * a
    idx = np.arange(n_side ** 3)
    ix, iy, iz = idx % n_side, (idx // n_side) % n_side, idx // (n_side * n_side)
    rp = np.random.Generator(np.random.PCG64(seed_pos))
    pos = np.stack([ix, iy, iz], axis=1) * a + rp.uniform(-noise * a, noise * a, (idx.size, 3))
    Lv = np.array([L, L, L])
    pos = wrap(pos, Lv)
    along_x = iz % 2 == 0
    # position of each site along its row, and the row it belongs to
    u = np.where(along_x, ix, iy)
    row = np.where(along_x, iy, ix) + n_side * iz
    order = np.lexsort((u, u % 2, row))  # row, parity, place along the row
    bonds = []
    per_chain = n_side // 2
    for c in range(idx.size // per_chain):
        beads = order[c * per_chain:(c + 1) * per_chain]
        bonds.extend(zip(beads[:-1], beads[1:]))
    vel = maxwell_velocities(idx.size, T, seed_vel)
    return System(pos=pos, vel=vel, tag=idx.astype(np.int32), L=Lv, bonds=np.array(bonds, dtype=np.int32),
                  kind="polymer")


def lj_subdomain_box(grid: int = 3, cells: int = 60, seed_pos: int = 11,
                     seed_vel: int = 12) -> Subdomains:
    """864,000-particle LJ box (fcc 60^3, lattice offset a/4, +-0.05 noise)
    cut into 3 x 3 x 3 cubes of 20^3 fcc cells, i.e. 32,000 particles each."""
    n = 4 * cells ** 3
    full = lj_fluid(n, seed_pos=seed_pos, seed_vel=seed_vel)
    side = float(full.L[0]) / grid
    c = np.floor(full.pos / side).astype(np.int64)
    c = np.clip(c, 0, grid - 1)
    owner = (c[:, 0] + grid * (c[:, 1] + grid * c[:, 2])).astype(np.int32)
    return Subdomains(full=full, grid=grid, side=side, owner=owner)


def batch_ensemble(n_lj: int = 128, n_poly: int = 128, seed_lj: int = 41,
                   seed_poly: int = 42, lj_range=(500, 20000),
                   chain_range=(20, 400)) -> List[System]:
    """Uneven ensemble: n_lj LJ liquids with N ~ U{500..20000} and n_poly
    polymer melts of 50-bead chains with U{20..400} chains each."""
    r1 = np.random.Generator(np.random.PCG64(seed_lj))
    r2 = np.random.Generator(np.random.PCG64(seed_poly))
    sizes = r1.integers(lj_range[0], lj_range[1] + 1, size=n_lj)
    chains = r2.integers(chain_range[0], chain_range[1] + 1, size=n_poly)
    out: List[System] = []
    for k, nk in enumerate(sizes):
        s = 1000 + k
        out.append(lj_fluid(int(nk), seed_pos=s, seed_vel=s + 500_000, seed_vac=s + 900_000))
    for k, ck in enumerate(chains):
        s = 1000 + n_lj + k
        out.append(polymer_melt(int(ck), seed_vel=s))
    return out
