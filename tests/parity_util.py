"""Helpers shared by the GPU parity tests: build the same seeded system in the
oracle and in the GPU library, and the error norms used to compare them.

Norms: densities max over fluid cells |d rho_k| / mean_k; fields
max |d| / max |ref|; populations max over fluid cells |d f_i| / w_i; particle
velocities |d v| / max(|v_ref|, 1e-3)."""
from __future__ import annotations

import sys

import numpy as np

from oracle import oracle as O
from paper_1607_04572_amd import workloads as W

W19 = O.D3Q19_W


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_params(w: W.Workload) -> O.OrParams:
    # the workloads are stated in lattice units (a = tau = kT = fluid density = 1)
    assert w.agrid == 1 and w.tau == 1 and w.fluid_density == 1
    return O.make_params(*w.shape, w.nu, w.kT, w.lambda_B, w.E, [(s.D, s.z) for s in w.species],
                         partial_volume=w.scheme == "pv", charge_mode=1 if w.charge == "uniform" else 0,
                         integrator=0 if w.integrator == "vv" else 1)


def oracle_spheres(w: W.Workload) -> list:
    return [dict(x=s.x, R=s.R, Z=s.Z, M=s.M, v=s.v, mode=s.mode) for s in w.spheres]


def make_oracle(w: W.Workload, rho0=None, **kw) -> O.OracleSim:
    rho0 = W.initial_densities(w) if rho0 is None else rho0
    return O.OracleSim(oracle_params(w), oracle_spheres(w), rho0, **kw)


def make_gpu(w: W.Workload, rho0=None, **kw):
    from paper_1607_04572_amd.ek import EkSim
    rho0 = W.initial_densities(w) if rho0 is None else rho0
    kw = {k: v for k, v in kw.items() if k in ("static_mask", "static_charge")}
    return EkSim(w, initial_density=rho0, **kw)


def density_err(w, g_rho, o_rho, fluid):
    ns = len(w.species)
    g = g_rho.reshape(ns, -1)
    o = o_rho.reshape(ns, -1)
    return max(np.max(np.abs(g[k][fluid] - o[k][fluid])) / w.species[k].mean for k in range(ns))


def field_err(g, o):
    m = np.max(np.abs(o))
    return np.max(np.abs(g - o)) / (m if m > 0 else 1.0)


def pop_err(g_f, o_f, fluid):
    g = g_f.reshape(19, -1)[:, fluid]
    o = o_f.reshape(19, -1)[:, fluid]
    return np.max(np.abs(g - o) / W19[:, None])


def compare(w, g, o, label=""):
    """Return a dict of errors between the GPU simulation g and the oracle o."""
    N = w.cells
    flag_g = g.field("flag")
    owner_g = g.field("owner")
    fluid = (flag_g == 0) & (o.flag == 0)
    out = {
        "flag_mismatch": int(np.sum(flag_g != o.flag)),
        "owner_mismatch": int(np.sum(owner_g != o.owner)),
        "psi": float(np.max(np.abs(g.field("psi") - o.psi))),
        "density": density_err(w, g.field("density"), o.rho, fluid),
        "phi": field_err(g.field("phi"), o.phi),
        "velocity": field_err(g.field("velocity").reshape(3, N)[:, fluid], o.u.reshape(3, N)[:, fluid]),
        "force": field_err(g.field("force").reshape(3, N)[:, fluid], o.fext.reshape(3, N)[:, fluid]),
        "populations": pop_err(g.field("populations"), o.f, fluid),
        "rhob": field_err(g.field("particle_charge"), o.rhob),
    }
    gp = g.particles()
    op = o.particles()
    dv, dx, dF = 0.0, 0.0, 0.0
    for a, b in zip(gp, op):
        dx = max(dx, float(np.max(np.abs(a["x"] - b["x"]))))
        dv = max(dv, float(np.linalg.norm(a["v"] - b["v"]) / max(np.linalg.norm(b["v"]), 1e-3)))
        dF = max(dF, float(np.linalg.norm(a["F"] - b["F"]) / max(np.linalg.norm(b["F"]), 1e-12)))
    out.update({"particle_x": dx, "particle_v": dv, "particle_F": dF})
    say(label, {k: (f"{v:.3e}" if isinstance(v, float) else v) for k, v in out.items()})
    return out


def snapshot(g, w: W.Workload) -> O.OracleSim:
    """The GPU state at a step boundary, as the oracle takes it (populations,
    densities, velocity, flags, owners, particles)."""
    parts = g.particles()
    spheres = [dict(x=p["x"], v=p["v"], w=p["omega"], F=p["F"], T=p["T"], R=s.R, Z=s.Z, M=s.M, mode=s.mode)
               for p, s in zip(parts, w.spheres)]
    return O.OracleSim.from_state(oracle_params(w), spheres, g.field("populations"), g.field("density"),
                                  g.field("velocity"), g.field("flag"), g.field("owner"))
