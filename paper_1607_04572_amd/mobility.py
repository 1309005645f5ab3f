"""Electrophoretic mobility workloads of the paper's validation (Sec. IV):
a charged sphere in salt in a uniform field, free (electrophoresis) or held
fixed (electro-osmosis, the co-moving frame), and several free spheres at
constant volume fraction.  Everything runs through the C ABI.

Table I restated in lattice units (grid spacing a = 1 nm, time step
tau = 0.2 of the unit t0 = sqrt(m0 a^2 / kT) with m0 = rho a^3):
  kT = (tau / t0)^2 = 0.04, lambda_B = 0.7136 (298.15 K, eps_r = 78.54),
  nu = eta / rho * tau / a^2 = 2.79, E = e E a / kT = 0.01,
  c = 1 mM = 6.022e-4 ions per cell and species (Debye length 9.6 cells),
  D = 2e-9 m^2/s * tau / a^2 = 6.22e-3 (the table prints "2 m^2/s"; read as
  a typical ion's 2e-9 m^2/s -- 2 in the table's own units would exceed the
  explicit scheme's stability bound), Z = 30, rho_p = 2 rho, box 64^3.
The reduced mobility (Sec. IV.A) is mu = 6 pi eta lambda_B v / (e E), v the
sphere's speed relative to the bulk fluid; in lattice units e E = kT E.
The systems are neutral: the salt's anions carry the sphere's counter-charge,
spread uniformly over the fluid cells."""
from __future__ import annotations

import math
import time

import numpy as np

from . import workloads as W

TABLE1 = dict(kT=0.04, lambda_B=0.7136, nu=2.79, E=0.01, c=6.022e-4, D=6.22e-3, Z=30.0, L=64)


def reduced_mobility(v_rel, p=TABLE1):
    return 6.0 * math.pi * p["nu"] * p["lambda_B"] * np.asarray(v_rel) / (p["kT"] * p["E"])


def colloid_workload(spheres, shape, scheme="pv", precision="fp32", p=TABLE1, name="colloid"):
    """spheres: list of (centre, R, mode); neutral salt plus counter-anions."""
    N = shape[0] * shape[1] * shape[2]
    vol = sum(4.0 / 3.0 * math.pi * R ** 3 for _, R, _ in spheres)
    counter = p["Z"] * len(spheres) / (N - vol)
    sph = [W.Sphere(x=tuple(c), R=R, Z=p["Z"], M=2.0 * W.sphere_volume(R), mode=mode) for c, R, mode in spheres]
    return W.Workload(name=name, shape=tuple(shape), precision=precision,
                      species=[W.Species(p["D"], +1, p["c"]), W.Species(p["D"], -1, p["c"] + counter)],
                      lambda_B=p["lambda_B"], E=(p["E"], 0.0, 0.0), steps=0, nu=p["nu"], kT=p["kT"], noise=0.0,
                      scheme=scheme, charge="psi" if scheme == "pv" else "uniform", integrator="se",
                      spheres=sph)


def run(w, steps: int, every: int, count_inside: bool = False, say=None) -> dict:
    """Step w for `steps` steps; every `every` steps record each sphere's
    velocity along the field, the bulk fluid velocity (fluid momentum / fluid
    mass), the boundary-cell count and, with count_inside, the number of cells
    completely inside a sphere (Psi = 1)."""
    from .ek import EkSim
    g = EkSim(w)
    g.prepare()
    rec = {"step": [], "v": [], "u_bulk": [], "n_boundary": [], "n_inside": []}
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        g.step(every)
        done += every
        d = g.diagnostics()
        rec["step"].append(done)
        rec["v"].append([q["v"][0] for q in g.particles()])
        rec["u_bulk"].append(d["fluid_momentum"][0] / d["fluid_mass"])
        rec["n_boundary"].append(d["boundary_cells"])
        if count_inside:
            rec["n_inside"].append(int(np.count_nonzero(g.field("psi") == 1.0)))
        if say and done % (every * 20) == 0:
            say(f"  {w.name} step {done} v {np.mean(rec['v'][-1]):.4e} u_bulk {rec['u_bulk'][-1]:.3e} "
                f"{time.perf_counter() - t0:.1f}s")
    g.sync()
    rec["seconds"] = time.perf_counter() - t0
    g.close()
    out = {k: np.asarray(v) for k, v in rec.items()}
    out["v_rel"] = out["v"] - out["u_bulk"][:, None]
    return out


def _claimed_cells(R: float, c, pv: bool) -> int:
    """Cells a sphere of radius R at c claims: completely inside (partial
    volumes; Psi = 1, i.e. all 16^3 leaf centres of the depth-4 subdivision
    within R, the farthest of them 1/32 in from the cell's corner) or centre
    inside (simple scheme)."""
    lo = np.floor(np.asarray(c) - R - 1).astype(int)
    hi = np.ceil(np.asarray(c) + R + 1).astype(int)
    ax = [np.arange(lo[d], hi[d]) for d in range(3)]
    if pv:
        s2 = [np.maximum(np.abs(a + 1 / 32 - c[d]), np.abs(a + 31 / 32 - c[d])) ** 2 for d, a in enumerate(ax)]
    else:
        s2 = [(a + 0.5 - c[d]) ** 2 for d, a in enumerate(ax)]
    return int(np.sum(s2[0][:, None, None] + s2[1][None, :, None] + s2[2][None, None, :] <= R * R))


def nominal_radius(R_eff: float, pv: bool, centre=(32.0, 32.0, 32.0), samples: int = 100) -> float:
    """Radius of a sphere moving along x whose claimed-cell count, averaged over
    one cell of travel, equals the volume (4/3) pi R_eff^3 (Sec. IV.A's
    effective radius, inverted)."""
    target = 4.0 / 3.0 * math.pi * R_eff ** 3

    def mean_count(R):
        return np.mean([_claimed_cells(R, (centre[0] + k / samples, centre[1], centre[2]), pv)
                        for k in range(samples)])

    lo, hi = 0.5 * R_eff, 2.0 * R_eff
    for _ in range(30):
        mid = 0.5 * (lo + hi)
        if mean_count(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def effective_radius(counts) -> float:
    """Radius of the sphere whose volume (4/3) pi R^3 equals the mean count."""
    return float((3.0 * np.mean(counts) / (4.0 * math.pi)) ** (1.0 / 3.0))


def oscillation(mu_t, period_steps: float, every: int) -> tuple:
    """Mean and relative oscillation amplitude (half the peak-to-peak range
    over the mean) of a mobility series over its last whole periods."""
    mu_t = np.asarray(mu_t)
    n = int(round(period_steps / every))
    k = max(1, len(mu_t) // max(n, 1))
    tail = mu_t[-k * n:] if n > 0 and k * n <= len(mu_t) else mu_t
    m = float(np.mean(tail))
    return m, float((tail.max() - tail.min()) / 2.0 / m)
