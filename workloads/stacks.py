"""Synthetic layered stacks and power maps (seeded, bit-reproducible).

Grid convention: cell (i, j, l) with i along x, j along y, l the layer from the
bottom; flat index i + nx*(j + ny*l).  Arrays are numpy float64 of shape
(nz, ny, nx) in C order, so ``a.ravel()`` is that flat order.

The paper evaluates on 3D-ICE matrices and public processor floorplans that are
not available here; these generators stand in for them with the same structure
(a 7-point layered stack of silicon dies, metal/bond layers, a TIM and a copper
spreader; block floorplans plus Gaussian hotspots; see the paper's experimental
setup in Section 5).  Every random draw uses
``numpy.random.default_rng(SeedSequence([2606, 17850, cfg, item, die, purpose, ...]))``
with purpose codes 0 = block densities, 1 = hotspots, 2 = lognormal lateral
conductivity, 3 = finite-difference cells, 4 = stack layout, 5 = Lanczos start.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# material: (thermal conductivity W/(m K), volumetric heat capacity J/(m^3 K))
MATERIALS = {
    "Si": (130.0, 1.63e6),
    "BEOL": (2.25, 2.0e6),
    "bond": (1.5, 2.0e6),
    "TIM": (4.0, 2.0e6),
    "Cu": (400.0, 3.45e6),
}
DIE_MATERIALS = ("Si", "BEOL", "bond")

CELL = 50e-6          # m, edge of every cell in every direction
H_TOP = 1.0e4         # W/(m^2 K) convective coefficient on the top face
T_AMB = 300.0         # K
MM2_PER_CELL = (CELL * 1e3) ** 2   # mm^2 of one cell's footprint


def _rng(*key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2606, 17850, *key]))


@dataclass
class Stack:
    """One layered grid: geometry, per-layer materials, boundary data."""

    nx: int
    ny: int
    layers: List[str]                      # material name per z-cell, bottom first
                                           # (names outside the table need explicit
                                           # k_lat, k_vert and heat_cap)
    dx: float = CELL
    dy: float = CELL
    dz: Optional[np.ndarray] = None        # [nz] m
    k_lat_mult: Optional[np.ndarray] = None  # (nz, ny, nx) multiplier, or None
    h_top: float = H_TOP
    h_bottom: float = 0.0
    t_amb: float = T_AMB
    dies: List[List[int]] = field(default_factory=list)  # Si z-cells of each die
    k_lat: Optional[np.ndarray] = None     # [nz] W/(m K); default from the material table
    k_vert: Optional[np.ndarray] = None    # [nz] W/(m K)
    heat_cap: Optional[np.ndarray] = None  # [nz] J/(m^3 K)

    def __post_init__(self):
        if self.dz is None:
            self.dz = np.full(self.nz, CELL)
        if self.k_lat is None:
            self.k_lat = np.array([MATERIALS[m][0] for m in self.layers])
        if self.k_vert is None:
            self.k_vert = np.array([MATERIALS[m][0] for m in self.layers])
        if self.heat_cap is None:
            self.heat_cap = np.array([MATERIALS[m][1] for m in self.layers])
        self.dz = np.asarray(self.dz, float)
        self.k_lat = np.asarray(self.k_lat, float)
        self.k_vert = np.asarray(self.k_vert, float)
        self.heat_cap = np.asarray(self.heat_cap, float)

    @property
    def nz(self) -> int:
        return len(self.layers)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    def si_mask(self) -> np.ndarray:
        """Boolean (nz, ny, nx): cells whose layer is silicon."""
        m = np.array([name == "Si" for name in self.layers])
        return np.broadcast_to(m[:, None, None], self.shape).copy()


# ----------------------------------------------------------------------------
# power-map pieces (densities in W/mm^2 over the (ny, nx) footprint)
# ----------------------------------------------------------------------------

def _gaussian_bumps(nx: int, ny: int, centres: np.ndarray, amps: np.ndarray,
                    sigma: float) -> np.ndarray:
    """Sum of amps[h] * exp(-r_h^2 / (2 sigma^2)) at cell centres, r in cells."""
    xs = np.arange(nx) + 0.5
    ys = np.arange(ny) + 0.5
    out = np.zeros((ny, nx))
    for (cx, cy), a in zip(centres, amps):
        gx = np.exp(-((xs - cx) ** 2) / (2.0 * sigma * sigma))
        gy = np.exp(-((ys - cy) ** 2) / (2.0 * sigma * sigma))
        out += a * gy[:, None] * gx[None, :]
    return out


def _block_floorplan(rng: np.random.Generator, nx: int, ny: int, nblk: int,
                     lo: float = 0.3, hi: float = 1.5) -> np.ndarray:
    """nblk x nblk blocks of uniform density U(lo, hi) W/mm^2."""
    dens = rng.uniform(lo, hi, size=(nblk, nblk))
    bi = (np.arange(nx) * nblk) // nx
    bj = (np.arange(ny) * nblk) // ny
    return dens[bj[:, None], bi[None, :]]


def _hotspots_on(rng: np.random.Generator, base: np.ndarray, count: int,
                 sigma: float = 3.0, gain: float = 4.0) -> np.ndarray:
    """base plus `count` Gaussian hotspots whose peak adds gain x base(centre)."""
    ny, nx = base.shape
    cx = rng.uniform(0.0, nx, size=count)
    cy = rng.uniform(0.0, ny, size=count)
    amps = gain * base[np.minimum(cy.astype(int), ny - 1), np.minimum(cx.astype(int), nx - 1)]
    return base + _gaussian_bumps(nx, ny, np.stack([cx, cy], 1), amps, sigma)


def _place_die_power(stack: Stack, die_density: Sequence[np.ndarray]) -> np.ndarray:
    """W per cell: each die's density split equally over its silicon z-cells."""
    P = np.zeros(stack.shape)
    for cells, dens in zip(stack.dies, die_density):
        w = dens * MM2_PER_CELL / len(cells)
        for l in cells:
            P[l] += w
    return P


def _lognormal_mult(stack: Stack, cfg: int, sigma: float = 0.3) -> np.ndarray:
    """exp(sigma*xi) per cell on die layers (Si, BEOL, bond); 1 elsewhere."""
    m = np.ones(stack.shape)
    for l, name in enumerate(stack.layers):
        if name in DIE_MATERIALS:
            xi = _rng(cfg, 0, l, 2).standard_normal((stack.ny, stack.nx))
            m[l] = np.exp(sigma * xi)
    return m


def _dies_of(layers: Sequence[str], si_per_die: int) -> List[List[int]]:
    si = [l for l, name in enumerate(layers) if name == "Si"]
    return [si[d:d + si_per_die] for d in range(0, len(si), si_per_die)]


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def config0() -> Tuple[Stack, np.ndarray]:
    """64x64x8 uniform stack, 2 dies; 0.5 W/mm^2 + 4 hotspots (5x peak) per die."""
    layers = ["Si", "BEOL", "bond", "Si", "BEOL", "bond", "TIM", "Cu"]
    st = Stack(64, 64, layers)
    st.dies = _dies_of(layers, 1)
    dens = []
    for d in range(len(st.dies)):
        base = np.full((st.ny, st.nx), 0.5)
        dens.append(_hotspots_on(_rng(0, 0, d, 1), base, 4))
    return st, _place_die_power(st, dens)


def uniform_stack(nx: int, ny: int, layers: Sequence[str], h_top: float = H_TOP,
                  h_bottom: float = 0.0) -> Stack:
    """A stack with per-layer uniform conductivity (no multiplier field)."""
    layers = list(layers)
    st = Stack(nx, ny, layers, h_top=h_top, h_bottom=h_bottom)
    st.dies = [[l] for l, name in enumerate(layers) if name == "Si"]
    return st


def _c1_layers() -> List[str]:
    return ["Si", "Si", "BEOL", "bond"] * 3 + ["TIM", "TIM", "Cu", "Cu"]


def config1(nx: int = 512, ny: int = 512) -> Tuple[Stack, np.ndarray]:
    """512x512x16, 3 dies, lognormal(0.3) lateral k on die layers.

    Per die: 16x16 block floorplan U(0.3, 1.5) W/mm^2 plus 32 hotspots.
    """
    layers = _c1_layers()
    st = Stack(nx, ny, layers)
    st.dies = _dies_of(layers, 2)
    st.k_lat_mult = _lognormal_mult(st, 1)
    dens = []
    for d in range(len(st.dies)):
        base = _block_floorplan(_rng(1, 0, d, 0), nx, ny, 16)
        dens.append(_hotspots_on(_rng(1, 0, d, 1), base, 32))
    return st, _place_die_power(st, dens)


def config2_stack(nx: int = 1024, ny: int = 1024) -> Stack:
    """1024x1024x20, 4 dies, per-layer uniform k (transient workload)."""
    layers = ["Si", "Si", "BEOL", "bond"] * 4 + ["TIM", "TIM", "Cu", "Cu"]
    st = Stack(nx, ny, layers)
    st.dies = _dies_of(layers, 2)
    return st


def config2_power(stack: Stack, floorplan: int) -> np.ndarray:
    """Floorplan f in 0..4: per die 16x16 blocks + 32 hotspots, W per cell."""
    dens = []
    for d in range(len(stack.dies)):
        base = _block_floorplan(_rng(2, floorplan, d, 0), stack.nx, stack.ny, 16)
        dens.append(_hotspots_on(_rng(2, floorplan, d, 1), base, 32))
    return _place_die_power(stack, dens)


def config2_floorplan_index(step: int) -> int:
    """Step s (producing T_{s+1}) uses floorplan (s div 20) mod 5."""
    return (step // 20) % 5


def config3(nstacks: int = 64, nrhs: int = 4) -> List[Tuple[Stack, List[np.ndarray]]]:
    """64 stacks of uneven size: edge in {128..384 step 64}, 8-16 layers.

    Layer 0 is Si, the top is Cu, middle layers iid over {Si, BEOL, bond, TIM}.
    Each stack gets nrhs power maps: 8x8 block floorplan + 8 hotspots on
    every Si layer.
    """
    out = []
    edges = np.array([128, 192, 256, 320, 384])
    mids = ["Si", "BEOL", "bond", "TIM"]
    for s in range(nstacks):
        r = _rng(3, s, 0, 4)
        edge = int(edges[r.integers(0, len(edges))])
        nz = int(r.integers(8, 17))
        layers = ["Si"] + [mids[int(q)] for q in r.integers(0, 4, size=nz - 2)] + ["Cu"]
        st = uniform_stack(edge, edge, layers)
        maps = []
        for q in range(nrhs):
            dens = []
            for d in range(len(st.dies)):
                base = _block_floorplan(_rng(3, s, d, 0, q), edge, edge, 8)
                dens.append(_hotspots_on(_rng(3, s, d, 1, q), base, 8))
            maps.append(_place_die_power(st, dens))
        out.append((st, maps))
    return out


def config4() -> Tuple[Stack, np.ndarray]:
    """The adjoint workload uses the 512x512x16 problem of config 1."""
    return config1()


def config4_small() -> Tuple[Stack, np.ndarray]:
    """64x64x8 copy for oracle gradients: config-0 stack, lognormal lateral k,
    16x16 blocks of 4x4 cells, 8 hotspots per die."""
    layers = ["Si", "BEOL", "bond", "Si", "BEOL", "bond", "TIM", "Cu"]
    st = Stack(64, 64, layers)
    st.dies = _dies_of(layers, 1)
    st.k_lat_mult = _lognormal_mult(st, 4)
    dens = []
    for d in range(len(st.dies)):
        base = _block_floorplan(_rng(4, 0, d, 0), 64, 64, 16)
        dens.append(_hotspots_on(_rng(4, 0, d, 1), base, 8))
    return st, _place_die_power(st, dens)


def fd_cells_config4(stack: Stack, count: int = 64) -> np.ndarray:
    """Flat indices of `count` distinct random silicon cells (for FD checks)."""
    si = np.flatnonzero(stack.si_mask().ravel())
    return np.sort(_rng(4, 0, 0, 3).choice(si, size=count, replace=False))


def lanczos_start(n: int, cfg: int = 0) -> np.ndarray:
    """Seeded N(0,1) start vector for spectral estimation."""
    return _rng(cfg, 0, 0, 5).standard_normal(n)
