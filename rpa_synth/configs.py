"""Registry of the synthetic workloads.

Each workload is a periodic cell (lattice rows in Angstrom, fractional atomic
positions, one species per atom), a Gamma-centred k-mesh that doubles as the
Born-von Karman (BvK) supercell, a real-space cutoff for the LRI neighbour sets
and the hoppings, and the number of imaginary time/frequency points.  The
shapes follow the workloads of the paper's performance and case-study sections
(DZP-sized carbon cells, Sec. 5; an adsorbate over a graphene sheet with 16-24
minimax points, Sec. 6) without reproducing any of its data.

Nothing here computes anything of the RPA method; it only lays out geometry.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MASTER_SEED = 20240729

# species name -> (number of NAOs, number of ABFs)
SPECIES_TABLE = {
    "X": (13, 40),    # tiny cell
    "Y": (26, 100),   # diamond-like cell
    "A": (13, 60),    # light species of the two-species cells
    "B": (26, 120),   # heavy species of the two-species cells
    "S": (26, 100),   # sheet atoms
}


def species_shape(name: str):
    """(nao, naux) of a species: a table entry, or 'n<nao>a<naux>' for ad-hoc test species."""
    if name in SPECIES_TABLE:
        return SPECIES_TABLE[name]
    if name.startswith("n") and "a" in name:
        a, b = name[1:].split("a")
        return int(a), int(b)
    raise KeyError(name)


# quantity ids of the seed tree
Q_GEOMETRY, Q_HAMILTONIAN, Q_LRI, Q_COULOMB = 0, 1, 2, 3


@dataclasses.dataclass
class Cell:
    """One periodic cell of a workload."""
    name: str
    lattice: np.ndarray          # (3,3) rows a1,a2,a3 in Angstrom
    frac: np.ndarray             # (natoms,3) fractional positions
    species: list                # natoms species names
    mesh: tuple                  # (N1,N2,N3) k-mesh == BvK supercell
    rcut: float                  # Angstrom, strict d < rcut
    ntau: int                    # number of tau (== omega) points
    seed_key: tuple              # (config id, cell id) in the seed tree
    v_scale: float = 1.0         # scale of the synthetic Coulomb matrix

    @property
    def natoms(self) -> int:
        return len(self.species)

    @property
    def nao(self) -> np.ndarray:
        return np.array([species_shape(s)[0] for s in self.species], dtype=np.int64)

    @property
    def naux(self) -> np.ndarray:
        return np.array([species_shape(s)[1] for s in self.species], dtype=np.int64)

    @property
    def nR(self) -> int:
        return int(np.prod(self.mesh))


def rng_for(seed_key: tuple, quantity: int) -> np.random.Generator:
    """PCG64 stream for one (config, cell, quantity) node of the seed tree."""
    ss = np.random.SeedSequence(MASTER_SEED, spawn_key=tuple(seed_key) + (quantity,))
    return np.random.Generator(np.random.PCG64(ss))


def _cubic(a):
    return np.eye(3) * a


def _random_positions(rng, lattice, n, dmin, max_tries=200000):
    """Uniform fractional positions with periodic minimum distance >= dmin."""
    pos = []
    tries = 0
    while len(pos) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place atoms")
        f = rng.random(3)
        ok = True
        for g in pos:
            d = f - g
            d -= np.round(d)
            if np.linalg.norm(d @ lattice) < dmin:
                ok = False
                break
        if ok:
            pos.append(f)
    return np.array(pos)


def tiny_cell() -> Cell:
    """Two identical atoms in a 5.4 A cubic cell, 2x2x2 mesh, 8 tau points, 8 A cutoff."""
    return Cell("tiny", _cubic(5.4), np.array([[0, 0, 0], [0.25, 0.25, 0.25]], float),
                ["X", "X"], (2, 2, 2), 8.0, 8, (0, 0), v_scale=V_SCALE[0])


def diamond_cell() -> Cell:
    """Eight atoms on diamond-like sites of a 5.4 A cubic cell, 4x4x4 mesh, 16 tau, 10 A cutoff."""
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    frac = np.vstack([fcc, fcc + 0.25])
    return Cell("diamond8", _cubic(5.4), frac, ["Y"] * 8, (4, 4, 4), 10.0, 16, (1, 0),
                v_scale=V_SCALE[1])


def two_species_cell() -> Cell:
    """32 atoms (24 light + 8 heavy) at random sites of an 8.6x8.6x12 A cell, 3x3x1 mesh."""
    lat = np.diag([8.6, 8.6, 12.0])
    rng = rng_for((2, 0), Q_GEOMETRY)
    frac = _random_positions(rng, lat, 32, 1.5)
    return Cell("twospecies32", lat, frac, ["A"] * 24 + ["B"] * 8, (3, 3, 1), 10.0, 16, (2, 0),
                v_scale=V_SCALE[2])


def sheet_cell(mesh=(1, 1, 1)) -> Cell:
    """6x6 hexagonal sheet (a = 2.46 A, 72 atoms) with a bent triatomic 3 A above a hexagon
    centre, 15 A of vacuum, 24 tau points, 12 A cutoff."""
    a = 2.46
    a1 = np.array([a, 0, 0])
    a2 = np.array([a / 2, a * math.sqrt(3) / 2, 0])
    c = 18.0
    lat = np.array([6 * a1, 6 * a2, [0, 0, c]])
    cart = []
    for i in range(6):
        for j in range(6):
            o = i * a1 + j * a2
            cart.append(o + (a1 + a2) / 3)
            cart.append(o + 2 * (a1 + a2) / 3)
    centre = 3 * a1 + 3 * a2           # a hexagon centre (lattice point of the sheet)
    heavy = centre + np.array([0, 0, 3.0])
    cart.append(heavy)
    cart.append(heavy + np.array([0.757, 0, -0.586]))
    cart.append(heavy + np.array([-0.757, 0, -0.586]))
    cart = np.array(cart)
    frac = cart @ np.linalg.inv(lat)
    species = ["S"] * 72 + ["B", "A", "A"]
    cid = 0 if tuple(mesh) == (1, 1, 1) else 1
    return Cell("sheet75_%dx%dx%d" % tuple(mesh), lat, frac, species, tuple(mesh), 12.0, 24,
                (3, cid), v_scale=V_SCALE[3] if cid == 0 else V_SCALE[33])


def serving_cells(ncells=64) -> list:
    """Independent cubic cells of 2..16 atoms (volume 27.7 A^3 per atom), heavy species with
    probability 1/4, meshes from {1,2,3}^3 (isotropic), 8..16 tau points, 8 A cutoff."""
    rng = rng_for((4, 0), Q_GEOMETRY)
    cells = []
    for c in range(ncells):
        n = int(rng.integers(2, 17))
        edge = (n * 27.7) ** (1.0 / 3.0)
        lat = _cubic(edge)
        sp = ["B" if rng.random() < 0.25 else "A" for _ in range(n)]
        m = int(rng.integers(1, 4))
        ntau = int(rng.integers(8, 17))
        frac = _random_positions(rng, lat, n, 1.5)
        cells.append(Cell("serve%02d" % c, lat, frac, sp, (m, m, m), 8.0, ntau, (4, c + 1),
                          v_scale=V_SCALE[4]))
    return cells


# Scale of the synthetic Coulomb matrix v(q) = s * (L L^H + 1e-3 I) / lambda_max(L L^H + 1e-3 I)
# per workload: the largest spectral radius of chi0(q, i omega) v(q) over q and omega (and, for
# the serving workload, over its 64 cells) is 0.9, so || chi0 v || < 1 as the workload
# definition asks.  Output of tests/golden/calibrate_vscale.py (exact oracle radii at s = 1:
# tiny 242.448, diamond-like 744.851, two-species 420.892, sheet (Gamma) 774.277, serving
# 3616.86 on cell serve31); the 2x2x1 sheet reuses the Gamma value.
V_SCALE = {0: 0.00386964, 1: 0.00120261, 2: 0.00213832, 3: 0.00116543, 33: 0.00116577, 4: 0.000277107}


def micro_cell(seed: int, natoms=2, nao=(3, 4), naux=(4, 5), mesh=(2, 1, 1), rcut=4.2,
               edge=3.0, ntau=3) -> Cell:
    """Small random cell for oracle pins and parity edge cases (seeded by `seed`)."""
    rng = rng_for((9, seed), Q_GEOMETRY)
    lat = _cubic(edge)
    frac = rng.random((natoms, 3))
    sp = ["n%da%d" % (nao[i % len(nao)], naux[i % len(naux)]) for i in range(natoms)]
    return Cell("micro%d" % seed, lat, frac, sp, tuple(mesh), rcut, ntau, (9, seed), v_scale=1.0)


def config(i: int):
    """Workload by index: 0 tiny, 1 diamond-like, 2 two-species, 3 sheet (Gamma), 4 serving."""
    if i == 0:
        return tiny_cell()
    if i == 1:
        return diamond_cell()
    if i == 2:
        return two_species_cell()
    if i == 3:
        return sheet_cell((1, 1, 1))
    if i == 33:
        return sheet_cell((2, 2, 1))
    if i == 4:
        return serving_cells()
    raise KeyError(i)
