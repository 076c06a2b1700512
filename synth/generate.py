"""Seeded input draws for the five workloads (gas phase, no periodic box).

Units throughout: Angstrom, femtosecond, atomic mass unit, electronvolt.

Recipe (shared by every workload, restated in the design notes):

* species counts: largest-remainder rounding of H:C:N:O = 50:30:10:10
  (ties go to the earlier element), laid out as an H block, then C, N, O;
* positions: random sequential addition (RSA) with numpy's PCG64.  A
  candidate drawn uniformly in the region is rejected when it lies closer
  than 0.9 A to any atom already placed; candidates are taken strictly in
  draw order, so the batched implementation below accepts exactly the atoms
  a one-at-a-time loop would;
* the region is a cube (the 22-atom molecule) or a ball whose radius gives a
  number density of 0.1 atoms per cubic Angstrom;
* velocities: Maxwell-Boltzmann at 300 K, v = sqrt(kB T kappa / m) * xi with
  xi ~ N(0, 1), centre-of-mass velocity removed per molecule, no rescaling;
* network weights: Xavier-normal in float32, std = sqrt(2 / (fan_in +
  fan_out)), drawn layer by layer in blob order; biases are zero.

The weight blob layout (float32, per element H, C, N, O in that order):
W1[160][384], b1[160], W2[128][160], b2[128], W3[96][128], b3[96],
W4[1][96], b4[1] -- weights stored [out][in], row-major.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
from scipy.spatial import cKDTree

ELEMENTS = ("H", "C", "N", "O")
#: IUPAC abridged standard atomic weights, amu.
MASSES_AMU = np.array([1.008, 12.011, 14.007, 15.999], dtype=np.float64)
COMPOSITION = (50, 30, 10, 10)

#: Boltzmann constant in eV/K.
KB_EV = 8.617333262e-5
#: Conversion eV / (Angstrom amu) -> Angstrom / fs^2.
KAPPA = 9.64853321e-3

MIN_SEP = 0.9
DENSITY = 0.1

#: (out, in) of every linear layer of the per-element network.
WEIGHT_SHAPES = ((160, 384), (128, 160), (96, 128), (1, 96))
N_WEIGHTS_PER_ELEMENT = sum(o * i + o for (o, i) in WEIGHT_SHAPES)
N_WEIGHTS = 4 * N_WEIGHTS_PER_ELEMENT


@dataclasses.dataclass
class System:
    """One workload instance in the caller's atom order."""

    name: str
    pos: np.ndarray          # (N, 3) float64, Angstrom
    species: np.ndarray      # (N,) int32 in {0: H, 1: C, 2: N, 3: O}
    masses: np.ndarray       # (N,) float64, amu
    vel: np.ndarray          # (N, 3) float64, Angstrom / fs
    mol_offsets: np.ndarray  # (M + 1,) int32; molecule m is [off[m], off[m+1])
    weights: np.ndarray      # (N_WEIGHTS,) float32
    meta: dict
    box: Optional[np.ndarray] = None  # (3,) orthorhombic box edges (Angstrom); None = gas phase

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_molecules(self) -> int:
        return int(self.mol_offsets.shape[0] - 1)

    def molecule(self, m: int) -> slice:
        return slice(int(self.mol_offsets[m]), int(self.mol_offsets[m + 1]))


def composition_counts(n: int, ratio=COMPOSITION) -> List[int]:
    """Largest-remainder split of ``n`` atoms over the element ratio."""
    total = float(sum(ratio))
    exact = [n * r / total for r in ratio]
    counts = [int(math.floor(e)) for e in exact]
    rem = n - sum(counts)
    order = sorted(range(len(ratio)), key=lambda k: (-(exact[k] - counts[k]), k))
    for k in order[:rem]:
        counts[k] += 1
    return counts


def species_block(counts) -> np.ndarray:
    return np.concatenate([np.full(c, e, dtype=np.int32) for e, c in enumerate(counts)])


def ball_radius(n: int, density: float = DENSITY) -> float:
    return (3.0 * n / (4.0 * math.pi * density)) ** (1.0 / 3.0)


def _rsa(n: int, draw, rng, d_min: float, batch: int, boxsize=None) -> np.ndarray:
    """Random sequential addition; ``draw(rng, k)`` returns k candidates.
    With ``boxsize`` distances are taken between nearest periodic images."""
    placed = np.empty((0, 3), dtype=np.float64)
    while placed.shape[0] < n:
        cand = draw(rng, batch)
        if placed.shape[0]:
            tree = cKDTree(placed, boxsize=boxsize)
            near = tree.query_ball_point(cand, r=d_min, return_length=True)
            cand = cand[near == 0]
        # resolve conflicts inside the batch in draw order
        if cand.shape[0] > 1:
            pairs = cKDTree(cand, boxsize=boxsize).query_pairs(d_min, output_type="ndarray")
            if pairs.shape[0]:
                later = {}
                for a, b in pairs:
                    a, b = (int(a), int(b)) if a < b else (int(b), int(a))
                    later.setdefault(b, []).append(a)
                keep = np.ones(cand.shape[0], dtype=bool)
                for b in sorted(later):
                    if any(keep[a] for a in later[b]):
                        keep[b] = False
                cand = cand[keep]
        placed = np.concatenate([placed, cand], axis=0)
    return placed[:n].copy()


def rsa_cube(n: int, edge: float, seed: int, d_min: float = MIN_SEP) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))

    def draw(r, k):
        return r.uniform(0.0, edge, size=(k, 3))

    return _rsa(n, draw, rng, d_min, batch=max(64, n))


def box_edge(n: int, density: float = DENSITY) -> float:
    return (n / density) ** (1.0 / 3.0)


def rsa_periodic(n: int, edge: float, seed: int, d_min: float = MIN_SEP) -> np.ndarray:
    """RSA of ``n`` atoms in [0, edge)^3 with periodic minimum separation."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def draw(r, k):
        return r.uniform(0.0, edge, size=(k, 3))

    return _rsa(n, draw, rng, d_min, batch=max(256, min(n, 32768)), boxsize=edge)


def rsa_ball(n: int, seed: int, density: float = DENSITY, d_min: float = MIN_SEP) -> np.ndarray:
    """RSA of ``n`` atoms in a ball centred on the origin at the given density."""
    rng = np.random.Generator(np.random.PCG64(seed))
    radius = ball_radius(n, density)

    def draw(r, k):
        # uniform in the ball: rejection from the enclosing cube
        out = []
        got = 0
        while got < k:
            c = r.uniform(-radius, radius, size=(2 * k, 3))
            c = c[np.einsum("ij,ij->i", c, c) < radius * radius]
            out.append(c)
            got += c.shape[0]
        return np.concatenate(out, axis=0)[:k]

    return _rsa(n, draw, rng, d_min, batch=max(256, min(n, 32768)))


def maxwell_boltzmann(masses: np.ndarray, mol_offsets: np.ndarray, seed: int,
                      temperature: float = 300.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    n = masses.shape[0]
    xi = rng.standard_normal(size=(n, 3))
    vel = np.sqrt(KB_EV * temperature * KAPPA / masses)[:, None] * xi
    for m in range(mol_offsets.shape[0] - 1):
        s = slice(int(mol_offsets[m]), int(mol_offsets[m + 1]))
        mm = masses[s]
        vcom = (mm[:, None] * vel[s]).sum(axis=0) / mm.sum()
        vel[s] -= vcom
    return vel


def xavier_weights(seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _e in range(4):
        for (fo, fi) in WEIGHT_SHAPES:
            std = np.float32(math.sqrt(2.0 / (fi + fo)))
            parts.append(rng.standard_normal(size=fo * fi, dtype=np.float32) * std)
            parts.append(np.zeros(fo, dtype=np.float32))
    blob = np.concatenate(parts).astype(np.float32)
    assert blob.shape[0] == N_WEIGHTS
    return blob


def molecule_sizes(n_mol: int, seed: int, lo: int = 10, hi: int = 300) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(math.log(lo), math.log(hi), size=n_mol)
    return np.clip(np.rint(np.exp(u)), lo, hi).astype(np.int64)


def _single(name: str, n: int, pos_seed: int, vel_seed: int, w_seed: int,
            cube: Optional[float] = None, counts=None) -> System:
    counts = counts if counts is not None else composition_counts(n)
    species = species_block(counts)
    pos = rsa_cube(n, cube, pos_seed) if cube is not None else rsa_ball(n, pos_seed)
    masses = MASSES_AMU[species]
    off = np.array([0, n], dtype=np.int32)
    vel = maxwell_boltzmann(masses, off, vel_seed)
    meta = {"pos_seed": pos_seed, "vel_seed": vel_seed, "weight_seed": w_seed,
            "region": ("cube %.1f A" % cube) if cube is not None else
            ("ball R=%.3f A" % ball_radius(n))}
    return System(name, pos, species, masses, vel, off, xavier_weights(w_seed), meta)


def _periodic(name: str, n: int, pos_seed: int, vel_seed: int, w_seed: int) -> System:
    species = species_block(composition_counts(n))
    L = box_edge(n)
    pos = rsa_periodic(n, L, pos_seed)
    masses = MASSES_AMU[species]
    off = np.array([0, n], dtype=np.int32)
    vel = maxwell_boltzmann(masses, off, vel_seed)
    meta = {"pos_seed": pos_seed, "vel_seed": vel_seed, "weight_seed": w_seed,
            "region": "periodic cube L=%.3f A" % L}
    return System(name, pos, species, masses, vel, off, xavier_weights(w_seed), meta,
                  box=np.array([L, L, L]))


def _batch(name: str, n_mol: int, size_seed: int, pos_seed0: int, vel_seed: int,
           w_seed: int) -> System:
    sizes = molecule_sizes(n_mol, size_seed)
    pos, spec = [], []
    for m, n in enumerate(sizes):
        spec.append(species_block(composition_counts(int(n))))
        pos.append(rsa_ball(int(n), pos_seed0 + m))
    species = np.concatenate(spec)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    masses = MASSES_AMU[species]
    vel = maxwell_boltzmann(masses, off, vel_seed)
    meta = {"size_seed": size_seed, "pos_seed0": pos_seed0, "vel_seed": vel_seed,
            "weight_seed": w_seed, "sizes": sizes.tolist()}
    return System(name, np.concatenate(pos), species, masses, vel, off,
                  xavier_weights(w_seed), meta)


#: The workloads: name -> builder arguments.
CONFIGS: Dict[str, dict] = {
    # 22-atom molecule (12 H, 6 C, 2 N, 2 O) in a 10 A cube
    "mol22": dict(kind="single", n=22, pos_seed=1, vel_seed=2, w_seed=0, cube=10.0,
                  counts=(12, 6, 2, 2)),
    # 2,500-atom cluster, ball R = 18.14 A
    "cluster2500": dict(kind="single", n=2500, pos_seed=11, vel_seed=12, w_seed=0),
    # precision study clusters
    "cluster2500b": dict(kind="single", n=2500, pos_seed=21, vel_seed=22, w_seed=0),
    "cluster23k": dict(kind="single", n=23000, pos_seed=23, vel_seed=24, w_seed=0),
    # 256 molecules of 10..300 atoms
    "batch256": dict(kind="batch", n_mol=256, size_seed=31, pos_seed0=32, vel_seed=33,
                     w_seed=0),
    # 100,000-atom droplet, ball R = 62.04 A
    "droplet100k": dict(kind="single", n=100000, pos_seed=41, vel_seed=42, w_seed=0),
    # periodic cubes at the same density (condensed phase): L = 13.57, 29.24, 61.27 A
    "box250": dict(kind="periodic", n=250, pos_seed=55, vel_seed=56, w_seed=0),
    "box2500": dict(kind="periodic", n=2500, pos_seed=51, vel_seed=52, w_seed=0),
    "box23k": dict(kind="periodic", n=23000, pos_seed=53, vel_seed=54, w_seed=0),
}


def make_config(name: str, **override) -> System:
    """Build a named workload; keyword overrides change seeds or sizes."""
    args = dict(CONFIGS[name])
    args.update(override)
    kind = args.pop("kind")
    if kind == "periodic":
        return _periodic(name, args["n"], args["pos_seed"], args["vel_seed"], args["w_seed"])
    if kind == "single":
        return _single(name, args["n"], args["pos_seed"], args["vel_seed"], args["w_seed"],
                       cube=args.get("cube"), counts=args.get("counts"))
    return _batch(name, args["n_mol"], args["size_seed"], args["pos_seed0"],
                  args["vel_seed"], args["w_seed"])
