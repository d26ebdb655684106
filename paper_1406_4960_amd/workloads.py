"""Seeded synthetic slab problems (inputs only).

This module draws the random numbers and lays out the geometry of the test
and benchmark problems: in-plane cell, knot breakpoints along z, Gauss points
per interval, FFT grid, G-set rule, k-points, atoms and their synthetic
potential parameters.  It holds none of the method's arithmetic (no B-spline,
no matrix element, no transform); both the CPU oracle and the HIP library read
the plain dictionary it returns.

Conventions of the dictionary (Hartree atomic units, lengths in bohr):

* ``a1``, ``a2``: in-plane lattice vectors (2-vectors).
* ``breakpoints``: strictly increasing knot breakpoints z_0 < ... < z_Nint; the
  clamped knot sequence of order ``order`` is built from them by each side.
* ``nq``: Gauss-Legendre points per knot interval.
* ``grid``: in-plane FFT grid (N1, N2) along a1, a2.
* ``gset``: ``{"kind": "box", "mmax": [M1, M2]}`` (all |m_i| <= M_i) or
  ``{"kind": "sphere", "ecut": E}`` (1/2 |k+G|^2 <= E, per k-point).
* ``kpts``: k-points in fractional coordinates of the reciprocal vectors.
* ``species``: list of dicts with ``gauss`` = [[A, w], ...] for the local part
  sum_t A_t exp(-r^2 / w_t^2) and, when ``nonlocal`` is true, Kleinman-Bylander
  parameters ``alpha_s``, ``alpha_p`` (Gaussian exponents, bohr^-2) and
  ``E_s``, ``E_p`` (projector energies, Ha) for one s and three p projectors.
* ``atoms``: list of dicts ``{"species": s, "pos": [x, y, z]}`` (Cartesian).
* ``nbands``: number of lowest eigenpairs wanted per k-point.
* Optional species keys ``q_s``, ``q_p`` (ultrasoft form): augmentation charges of the
  s and p projectors, so that the overlap gains sum_p q_p |beta_p><beta_p| (the
  generalized problem of the ultrasoft scheme); absent or zero = norm-conserving.

The seeds follow one rule: problem family index ``idx`` uses
``numpy.random.Generator(PCG64(14064960 + idx))``; member p of the batched
family uses ``14064960 + 1000 * (p + 1)``.
"""
from __future__ import annotations

import copy
import math

import numpy as np

SEED_BASE = 14064960

# FFT grid sizes with only factors 2, 3 and 5 used by the batched family.
SMOOTH_GRIDS = (24, 25, 27, 30, 32, 36, 40, 45, 48, 50, 54, 60, 64, 72, 75, 80)


def _rng(offset: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + offset))


def uniform_breakpoints(z0: float, z1: float, nint: int) -> list:
    return [float(v) for v in np.linspace(z0, z1, nint + 1)]


def graded_breakpoints(z0: float, z1: float, nint: int, gamma: float = 2.0) -> list:
    """Breakpoints dense near the slab centre and sparse towards the walls.

    The paper uses an "exponential-type" sequence without giving a formula; a
    sinh map t -> sinh(gamma t)/sinh(gamma) on a uniform t in [-1, 1] is used,
    which makes the edge spacing cosh(gamma) times the centre spacing.
    """
    t = -1.0 + 2.0 * np.arange(nint + 1) / nint
    half = 0.5 * (z1 - z0)
    zc = 0.5 * (z1 + z0)
    z = zc + half * np.sinh(gamma * t) / math.sinh(gamma)
    z[0], z[-1] = z0, z1
    return [float(v) for v in z]


def mp_grid(n1: int, n2: int) -> list:
    """Monkhorst-Pack fractional k-points (no symmetry reduction)."""
    f1 = [(2 * r - n1 - 1) / (2.0 * n1) for r in range(1, n1 + 1)]
    f2 = [(2 * r - n2 - 1) / (2.0 * n2) for r in range(1, n2 + 1)]
    return [[a, b] for a in f1 for b in f2]


def _hex(a: float):
    return [a, 0.0], [0.5 * a, 0.5 * math.sqrt(3.0) * a]


def _kb_species(rng: np.random.Generator, gauss) -> dict:
    return {
        "gauss": gauss,
        "nonlocal": True,
        "alpha_s": float(rng.uniform(1.0, 3.0)),
        "alpha_p": float(rng.uniform(1.0, 3.0)),
        "E_s": float(rng.uniform(-1.0, 1.0)),
        "E_p": float(rng.uniform(-1.0, 1.0)),
    }


def tiny() -> dict:
    """Square cell a = 5, Gamma only, 7x7 G box, 40 cubic B-splines on
    [-15, 15], four seeded Gaussian wells, no nonlocal part (n = 1960)."""
    rng = _rng(0)
    a = 5.0
    species, atoms = [], []
    for _ in range(4):
        depth = float(rng.uniform(0.5, 2.0))
        width = float(rng.uniform(0.8, 1.5))
        f1, f2 = rng.uniform(0.0, 1.0, size=2)
        rz = float(rng.uniform(-3.0, 3.0))
        species.append({"gauss": [[-depth, width]], "nonlocal": False})
        atoms.append({"species": len(species) - 1, "pos": [float(f1 * a), float(f2 * a), rz]})
    return {
        "name": "tiny-square-a5-gamma",
        "a1": [a, 0.0], "a2": [0.0, a],
        "order": 4,
        "breakpoints": uniform_breakpoints(-15.0, 15.0, 39),
        "nq": 5,
        "grid": [16, 16],
        "gset": {"kind": "box", "mmax": [3, 3]},
        "kpts": [[0.0, 0.0]],
        "species": species,
        "atoms": atoms,
        "nbands": 8,
    }


def _graphene_species(rng):
    gauss = [[-float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.8, 1.5))],
             [float(rng.uniform(0.1, 0.5)), float(rng.uniform(0.8, 1.0))]]
    return _kb_species(rng, gauss)


def graphene() -> dict:
    """Hexagonal a = 4.65 slab, 36x36 grid, ~491 G, 80 graded cubic B-splines
    on [-20, 20], two atoms with Gaussian local parts and 4 KB projectors each,
    2x2 Monkhorst-Pack k-points, 32 bands (n ~ 39,280 per k)."""
    rng = _rng(1)
    a = 4.65
    a1, a2 = _hex(a)
    sp = _graphene_species(rng)
    atoms = []
    for f in ((1.0 / 3.0, 1.0 / 3.0), (2.0 / 3.0, 2.0 / 3.0)):
        x = f[0] * a1[0] + f[1] * a2[0]
        y = f[0] * a1[1] + f[1] * a2[1]
        atoms.append({"species": 0, "pos": [x, y, 0.0]})
    return {
        "name": "graphene-like-hex-a4.65",
        "a1": a1, "a2": a2,
        "order": 4,
        "breakpoints": graded_breakpoints(-20.0, 20.0, 79),
        "nq": 5,
        "grid": [36, 36],
        "gset": {"kind": "sphere", "ecut": 161.9},
        "kpts": mp_grid(2, 2),
        "species": [sp],
        "atoms": atoms,
        "nbands": 32,
    }


def graphene_2x2() -> dict:
    """2x2 supercell of the graphene-like slab: 8 atoms, 72x72 grid,
    ~1,903 G, 96 graded B-splines, 2x2 MP k-points, 64 bands."""
    base = graphene()
    rng = _rng(2)
    del rng  # the physics is the graphene family's; no new draws
    a = 2 * 4.65
    a1, a2 = _hex(a)
    b1, b2 = _hex(4.65)
    atoms = []
    for i in range(2):
        for j in range(2):
            for at in base["atoms"]:
                x = at["pos"][0] + i * b1[0] + j * b2[0]
                y = at["pos"][1] + i * b1[1] + j * b2[1]
                atoms.append({"species": 0, "pos": [x, y, 0.0]})
    return {
        "name": "graphene-like-2x2-hex-a9.30",
        "a1": a1, "a2": a2,
        "order": 4,
        "breakpoints": graded_breakpoints(-20.0, 20.0, 95),
        "nq": 5,
        "grid": [72, 72],
        "gset": {"kind": "sphere", "ecut": 159.1},
        "kpts": mp_grid(2, 2),
        "species": base["species"],
        "atoms": atoms,
        "nbands": 64,
    }


def batched_member(p: int) -> dict:
    """Member p of the uneven batch: seeded cell, grid, knots, atoms, k, bands."""
    rng = _rng(1000 * (p + 1))
    a = float(rng.uniform(4.0, 10.0))
    if rng.uniform() < 0.5:
        a1, a2 = _hex(a)
    else:
        a1, a2 = [a, 0.0], [0.0, a]
    n = int(SMOOTH_GRIDS[int(rng.integers(0, len(SMOOTH_GRIDS)))])
    f = float(rng.uniform(0.70, 0.80))
    radius = f * math.pi * (n - 1) / a
    nb = int(rng.integers(48, 129))
    nat = int(rng.integers(2, 17))
    sp = _graphene_species(rng)
    atoms = []
    for _ in range(nat):
        u, v = rng.uniform(0.0, 1.0, size=2)
        atoms.append({"species": 0,
                      "pos": [float(u * a1[0] + v * a2[0]), float(u * a1[1] + v * a2[1]),
                              float(rng.uniform(-3.0, 3.0))]})
    nk = int(rng.integers(1, 9))
    nbands = int(rng.integers(16, 97))
    return {
        "name": f"batched-{p:02d}",
        "a1": a1, "a2": a2,
        "order": 4,
        "breakpoints": graded_breakpoints(-20.0, 20.0, nb - 1),
        "nq": 5,
        "grid": [n, n],
        "gset": {"kind": "sphere", "ecut": 0.5 * radius * radius},
        "kpts": mp_grid(4, 2)[:nk],
        "species": [sp],
        "atoms": atoms,
        "nbands": nbands,
    }


def batched(count: int = 48) -> list:
    return [batched_member(p) for p in range(count)]


def surface() -> dict:
    """4x2 surface cell of a square a_s = 4.767 lattice (19.07 x 9.534), 128x64
    grid, ~4,003 G, 64 atoms in 8 layers with seeded +-0.2 bohr displacements,
    192 graded B-splines on [-30, 30] with 6 Gauss points per interval,
    4 projectors per atom, 4x2 MP k-points, 320 bands."""
    rng = _rng(4)
    asq = 4.767
    a1, a2 = [4 * asq, 0.0], [0.0, 2 * asq]
    sp = _graphene_species(rng)
    offsets = ((0.0, 0.0), (0.5, 0.0), (0.5, 0.5), (0.0, 0.5))
    atoms = []
    spacing = 1.685
    for layer in range(8):
        z = (layer - 3.5) * spacing
        ox, oy = offsets[layer % 4]
        for cx in range(4):
            for cy in range(2):
                d = rng.uniform(-0.2, 0.2, size=3)
                atoms.append({"species": 0,
                              "pos": [float((cx + ox) * asq + d[0]), float((cy + oy) * asq + d[1]),
                                      float(z + d[2])]})
    return {
        "name": "surface-4x2-128x64",
        "a1": a1, "a2": a2,
        "order": 4,
        "breakpoints": graded_breakpoints(-30.0, 30.0, 191),
        "nq": 6,
        "grid": [128, 64],
        "gset": {"kind": "sphere", "ecut": 138.1},
        "kpts": mp_grid(4, 2),
        "species": [sp],
        "atoms": atoms,
        "nbands": 320,
    }


def with_augmentation(desc: dict, offset: int = 7, lo: float = 0.1, hi: float = 0.5) -> dict:
    """The same description with seeded augmentation charges q_s, q_p ~ U[lo, hi] on
    every nonlocal species (the ultrasoft overlap; positive charges keep S positive
    definite)."""
    rng = _rng(offset)
    species = []
    for sp in desc["species"]:
        sp = dict(sp)
        if sp.get("nonlocal", False):
            sp["q_s"] = float(rng.uniform(lo, hi))
            sp["q_p"] = float(rng.uniform(lo, hi))
        species.append(sp)
    return dict(desc, species=species, name=desc["name"] + "-uspp")


def graphene_uspp() -> dict:
    """The graphene-like slab in the ultrasoft form: the same cell, grid, splines,
    atoms and projectors, plus augmentation charges q_s, q_p ~ U[0.1, 0.5]."""
    return with_augmentation(graphene(), offset=11)


def micro(seed: int = 7, nonlocal_: bool = True, nint: int = 7, mmax: int = 1,
          kfrac=(0.1, 0.2), natoms: int = 1, grid: int = 8) -> dict:
    """A very small cell (3x3 G box, 8 B-splines by default) for brute-force
    checks of the matrix elements."""
    rng = _rng(100 + seed)
    a = 4.0
    a1, a2 = [a, 0.0], [0.3 * a, 0.9 * a]
    species = []
    atoms = []
    for _ in range(natoms):
        gauss = [[-float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.8, 1.5))]]
        if nonlocal_:
            species.append(_kb_species(rng, gauss))
        else:
            species.append({"gauss": gauss, "nonlocal": False})
        u, v = rng.uniform(0.0, 1.0, size=2)
        atoms.append({"species": len(species) - 1,
                      "pos": [float(u * a1[0] + v * a2[0]), float(u * a1[1] + v * a2[1]),
                              float(rng.uniform(-1.0, 1.0))]})
    return {
        "name": f"micro-{seed}",
        "a1": a1, "a2": a2,
        "order": 4,
        "breakpoints": uniform_breakpoints(-6.0, 6.0, nint),
        "nq": 5,
        "grid": [grid, grid],
        "gset": {"kind": "box", "mmax": [mmax, mmax]},
        "kpts": [list(kfrac)],
        "species": species,
        "atoms": atoms,
        "nbands": 4,
    }


def mp_line(n: int) -> list:
    """Monkhorst-Pack fractions of 2 pi / L along the periodic axis."""
    return [(2 * r - n - 1) / (2.0 * n) for r in range(1, n + 1)]


def armchair_ribbon_atoms(na: int, a: float = 4.65) -> tuple:
    """Carbon-like sites of an armchair ribbon with na dimer lines across x, periodic
    along y with period sqrt(3) a (bond length d = a / sqrt(3)): line n sits at
    x = (n - (na - 1)/2) a/2 and holds the two atoms y = 0, d (n even) or 1.5 d, 2.5 d
    (n odd), so neighbouring lines bond at distance d.  Returns (period, [(x, y)])."""
    d = a / math.sqrt(3.0)
    out = []
    for n in range(na):
        x = (n - 0.5 * (na - 1)) * 0.5 * a
        ys = (0.0, d) if n % 2 == 0 else (1.5 * d, 2.5 * d)
        out += [(float(x), float(y)) for y in ys]
    return 3.0 * d, out


def _wire(name, na, x_half, nint_x, z_half, nint_z, ecut, ny, nk, nbands, offset):
    rng = _rng(offset)
    sp = _graphene_species(rng)
    period, sites = armchair_ribbon_atoms(na)
    return {
        "kind": "wire",
        "name": name,
        "period": period,
        "order": 4,
        "breakpoints_x": uniform_breakpoints(-x_half, x_half, nint_x),
        "breakpoints_z": graded_breakpoints(-z_half, z_half, nint_z),
        "nq": 5,
        "ny": ny,
        "ecut": ecut,
        "kpts": mp_line(nk),
        "species": [sp],
        "atoms": [{"species": 0, "pos": [x, y, 0.0]} for x, y in sites],
        "nbands": nbands,
    }


def ribbon() -> dict:
    """1D-periodic armchair ribbon (19 dimer lines, 38 atoms per period 8.05 bohr)
    in the basis of two B-spline directions x 1D plane waves: 112 uniform intervals
    on x in [-28, 28] (113 splines), 48 graded intervals on z in [-16, 16] (49
    splines), the graphene-like cutoff 1/2 (k+G)^2 <= 161.9 (47 plane waves), a
    64-point y grid, 4 k-points, 96 bands (n ~ 260,000 per k)."""
    return _wire("armchair-ribbon-19", 19, 28.0, 112, 16.0, 48, 161.9, 64, 4, 96, 30)


def ribbon_narrow() -> dict:
    """A 3-line ribbon small enough for dense eigenvalues: 16 x 16 intervals on
    [-8, 8]^2, 1/2 (k+G)^2 <= 15 (15 plane waves), 16-point y grid, 2 k-points,
    16 bands (n ~ 4,300)."""
    return _wire("armchair-ribbon-3", 3, 8.0, 16, 8.0, 16, 15.0, 16, 2, 16, 31)


def wire_micro(seed: int = 0, nint: int = 6, ecut: float = 6.0, ny: int = 8, kfrac: float = 0.17,
               natoms: int = 2, nonlocal_: bool = True, period: float = 4.0) -> dict:
    """A very small 1D-periodic cell for brute-force checks: seeded wells on
    [-5, 5]^2 with nint intervals per direction."""
    rng = _rng(200 + seed)
    species, atoms = [], []
    for _ in range(natoms):
        gauss = [[-float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.8, 1.5))]]
        species.append(_kb_species(rng, gauss) if nonlocal_ else {"gauss": gauss, "nonlocal": False})
        atoms.append({"species": len(species) - 1,
                      "pos": [float(rng.uniform(-1.5, 1.5)), float(rng.uniform(0.0, period)),
                              float(rng.uniform(-1.0, 1.0))]})
    return {
        "kind": "wire",
        "name": f"wire-micro-{seed}",
        "period": period,
        "order": 4,
        "breakpoints_x": uniform_breakpoints(-5.0, 5.0, nint),
        "breakpoints_z": graded_breakpoints(-5.0, 5.0, nint),
        "nq": 5,
        "ny": ny,
        "ecut": ecut,
        "kpts": [kfrac],
        "species": species,
        "atoms": atoms,
        "nbands": 4,
    }


def at_gamma(desc: dict) -> dict:
    """The same cell with the single k-point Gamma (k = 0), where the eigenvectors can
    be taken real in space."""
    d = copy.deepcopy(desc)
    d["name"] = desc["name"] + "-gamma"
    d["kpts"] = [[0.0, 0.0]]
    return d


CONFIGS = {
    "tiny": tiny,
    "graphene": graphene,
    "graphene_uspp": graphene_uspp,
    "graphene_2x2": graphene_2x2,
    "surface": surface,
    "ribbon": ribbon,
    "ribbon_narrow": ribbon_narrow,
}


def random_block(seed: int, nbands: int, nb: int, ng: int) -> np.ndarray:
    """Seeded complex block [band][i][G] with entries uniform in the unit square."""
    rng = _rng(5000 + seed)
    re = rng.uniform(-1.0, 1.0, size=(nbands, nb, ng))
    im = rng.uniform(-1.0, 1.0, size=(nbands, nb, ng))
    return re + 1j * im
