"""Seeded synthetic workloads: parameter sets and initial inputs.

This module holds no arithmetic of the method itself.  It only describes the
simulated systems (box, species, spheres, field) and draws their seeded inputs:
the initial solute densities (uniform mean plus bounded noise, from the
counter-based generator splitmix64) and the sphere positions (random sequential
addition without overlap).  The same arrays are handed to the GPU library and
to the CPU oracle.

The systems follow the shape of the paper's validation workloads (Sec. IV and
Table I: a cubic periodic box, charged spheres, monovalent salt, a uniform
field), restated directly in lattice units (a = tau = kT = fluid density = 1).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field

import numpy as np

# Stability bound of the explicit diffusive flux at the normalisation used by
# the library: D must stay below 2 / max_k sum_i (1 - cos k.c_i)/(A0 |c_i|)
# ~= 0.3964; the 3-species workload therefore runs its fastest species at 0.39.
D_FAST_SPECIES = 0.39

MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea, Flood 2014), vectorised on uint64."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & MASK64
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & MASK64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & MASK64
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, stream: int, n: int) -> np.ndarray:
    """U in [0, 1) for counters 0..n-1 of one stream: (splitmix64(seed ^ stream<<40 ^ i) >> 11) * 2^-53."""
    key = np.uint64(seed) ^ (np.uint64(stream) << np.uint64(40))
    x = splitmix64(np.arange(n, dtype=np.uint64) ^ key)
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclass
class Species:
    D: float          # diffusion coefficient
    z: int            # valency
    mean: float       # mean number density per cell


@dataclass
class Sphere:
    x: tuple
    R: float
    Z: float
    M: float
    v: tuple = (0.0, 0.0, 0.0)
    mode: int = 0     # 0 free, 1 prescribed velocity, 2 fixed


@dataclass
class Workload:
    name: str
    shape: tuple                     # (nx, ny, nz)
    precision: str                   # "fp64" or "fp32"
    species: list
    spheres: list
    lambda_B: float
    E: tuple
    steps: int
    nu: float = 1.0 / 6.0
    kT: float = 1.0
    fluid_density: float = 1.0
    agrid: float = 1.0
    tau: float = 1.0
    seed: int = 1607
    noise: float = 0.01
    scheme: str = "pv"               # "pv" (partial volume) or "simple"
    charge: str = "psi"              # "psi" (Z Psi / V_p) or "uniform" (Z / N_b)
    integrator: str = "vv"           # "vv" or "se"
    extra: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return int(self.shape[0] * self.shape[1] * self.shape[2])

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def initial_densities(w: Workload) -> np.ndarray:
    """rho_k(cell) = mean_k * (1 + noise * (2U - 1)), shape (n_species, N), x fastest."""
    out = np.empty((len(w.species), w.cells))
    for k, s in enumerate(w.species):
        u = uniform01(w.seed, k, w.cells)
        out[k] = s.mean * (1.0 + w.noise * (2.0 * u - 1.0))
    return out


def sphere_volume(R: float) -> float:
    return 4.0 / 3.0 * math.pi * R ** 3


def place_spheres(n: int, R: float, shape: tuple, seed: int, gap: float = 2.0,
                  max_tries: int = 100000) -> list:
    """Random sequential addition: uniform centres in the box, a candidate is
    rejected if its minimum-image distance to any accepted centre is below
    2R + gap."""
    rng = np.random.default_rng(seed)
    L = np.array(shape, dtype=np.float64)
    out = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place spheres without overlap")
        c = rng.uniform(0.0, 1.0, 3) * L
        ok = True
        for o in out:
            dd = c - o
            dd -= L * np.round(dd / L)
            if float(np.sqrt((dd * dd).sum())) < 2 * R + gap:
                ok = False
                break
        if ok:
            out.append(c)
    return [tuple(float(v) for v in c) for c in out]


def salt(D: float = 0.3, mean: float = 0.01) -> list:
    return [Species(D, +1, mean), Species(D, -1, mean)]


def c0() -> Workload:
    """32^3 FP64, one sphere (R=4, Z=+20 spread uniformly over its boundary
    cells) moving at a prescribed velocity 0.01 along x; 500 steps."""
    return Workload(
        name="c0_32cube_fp64_prescribed_sphere", shape=(32, 32, 32), precision="fp64",
        species=salt(), lambda_B=0.7, E=(0.01, 0.0, 0.0), steps=500,
        spheres=[Sphere(x=(16.0, 16.0, 16.0), R=4.0, Z=20.0, M=2 * sphere_volume(4.0),
                        v=(0.01, 0.0, 0.0), mode=1)],
        charge="uniform")


def c1(precision: str = "fp32") -> Workload:
    """64^3, one free sphere (R=6, Z=+40, M=1000), velocity Verlet; 5000 steps."""
    return Workload(
        name=f"c1_64cube_{precision}_free_sphere", shape=(64, 64, 64), precision=precision,
        species=salt(), lambda_B=0.7, E=(0.01, 0.0, 0.0), steps=5000,
        spheres=[Sphere(x=(32.0, 32.0, 32.0), R=6.0, Z=40.0, M=1000.0)])


def c2(precision: str = "fp32") -> Workload:
    """128^3, 8 free spheres (R=5, Z=+30), 3 species; 2000 steps.  Species as
    stated: a +1 counterion (D 0.2, 0.005), +1/-1 salt (D 0.3 and 0.39, 0.0125
    and 0.02)."""
    R = 5.0
    pos = place_spheres(8, R, (128, 128, 128), seed=1609)
    return Workload(
        name=f"c2_128cube_{precision}_8spheres_3species", shape=(128, 128, 128), precision=precision,
        species=[Species(0.2, +1, 0.005), Species(0.3, +1, 0.0125), Species(D_FAST_SPECIES, -1, 0.02)],
        lambda_B=0.7, E=(0.02, 0.0, 0.0), steps=2000,
        spheres=[Sphere(x=c, R=R, Z=30.0, M=2 * sphere_volume(R)) for c in pos])


def c3(precision: str = "fp32") -> Workload:
    """256^3 (16.8 M cells), 64 free spheres (R=6, Z=+40), 2 monovalent
    species at 0.01; 1000 steps."""
    R = 6.0
    pos = place_spheres(64, R, (256, 256, 256), seed=1610)
    return Workload(
        name=f"c3_256cube_{precision}_64spheres", shape=(256, 256, 256), precision=precision,
        species=salt(), lambda_B=0.7, E=(0.01, 0.0, 0.0), steps=1000,
        spheres=[Sphere(x=c, R=R, Z=40.0, M=2 * sphere_volume(R)) for c in pos])


EDGES = (32, 48, 64, 96, 128)


def serve_requests(n: int = 200, seed: int = 1611, rate: float = 1.0, steps: int = 1000) -> list:
    """Seeded request stream for the serving loop: Poisson arrivals (rate in
    requests per second), box edge uniform over EDGES, 1-16 spheres (volume
    fraction at most 10 %), radius U[3, 6], valency U{10..50}, mass 2 V_p,
    field U[0.005, 0.03] along x, salt density U[0.002, 0.02]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        L = int(rng.choice(EDGES))
        R = float(rng.uniform(3.0, 6.0))
        nsp = int(rng.integers(1, 17))
        nsp = max(1, min(nsp, int(0.10 * L ** 3 / sphere_volume(R))))
        Z = float(rng.integers(10, 51))
        E = float(rng.uniform(0.005, 0.03))
        c = float(rng.uniform(0.002, 0.02))
        pos = place_spheres(nsp, R, (L, L, L), seed=seed * 1000 + i)
        w = Workload(
            name=f"req{i}", shape=(L, L, L), precision="fp32", species=salt(0.3, c),
            lambda_B=0.7, E=(E, 0.0, 0.0), steps=steps, seed=seed * 1000 + i,
            spheres=[Sphere(x=p, R=R, Z=Z, M=2 * sphere_volume(R)) for p in pos])
        out.append((t, w))
    return out


CONFIGS = {"c0": c0, "c1": c1, "c2": c2, "c3": c3}
