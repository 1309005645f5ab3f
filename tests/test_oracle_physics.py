"""Physics pin of the coupled oracle: electro-osmotic flow in a charged slit
with counterions only (Gouy-Chapman), whose steady state has a closed form.
This exercises Poisson (Eq. poisson), the Nernst-Planck fluxes (Eq. flux,
discrete form of Sec. III.C), the coupling force (Eq. fluidcoupling) and the
LB solver with resting walls (Sec. III.A) together.

Closed form for a slit of width d between walls of surface charge sigma,
counterion valency z, external field E along the walls:
  phi(x) = (2/z) ln cos(C x),  rho(x) = C^2 / (2 pi lambda_B z^2) sec^2(C x),
  C tan(C d / 2) = -2 pi lambda_B z sigma,
  u(x) = 2 kT E / (4 pi lambda_B eta z) ln[cos(C x) / cos(C d / 2)],
with x measured from the mid-plane and eta = nu * rho0."""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import oracle as O


@pytest.mark.slow
def test_gouy_chapman_electro_osmosis():
    nx, ny, nz = 32, 2, 2
    N = nx * ny * nz
    lb, kT, nu, D, z = 0.7, 1.0, 1 / 6, 0.3, 1
    E = 0.01
    Nc = 0.1                      # counterions per unit wall area (per column)
    p = O.make_params(nx, ny, nz, nu, kT, lb, (0.0, E, 0.0), [(D, z)])
    x = np.tile(np.arange(nx), ny * nz)
    wall = (x == 0).astype(np.uint8)
    static_charge = np.where(wall == 1, -Nc, 0.0)   # one wall cell per column
    rho = np.where(wall == 1, 0.0, Nc / (nx - 1))
    s = O.OracleSim(p, [], rho, static_mask=wall, static_charge=static_charge)
    for _ in range(6000):
        s.step()
    d = nx - 1.0                  # walls half-way between nodes: x = 1/2 and nx - 1/2
    sigma = -Nc / 2.0             # each of the two wall faces carries half
    C = brentq(lambda c: c * np.tan(c * d / 2) + 2 * np.pi * lb * z * sigma, 1e-6, np.pi / d - 1e-9)
    xf = np.arange(1, nx) - nx / 2.0
    rho_ref = C ** 2 / (2 * np.pi * lb * z * z) / np.cos(C * xf) ** 2
    u_ref = 2 * kT * E / (4 * np.pi * lb * nu * z) * np.log(np.cos(C * xf) / np.cos(C * d / 2))
    rho_sim = s.density()[0][:nx][1:]
    u_sim = s.u[N:N + nx][1:]
    assert abs(rho_sim.sum() - Nc) < 1e-12
    assert np.max(np.abs(rho_sim / rho_ref - 1)) < 0.015
    assert np.max(np.abs(u_sim - u_ref)) < 0.01 * u_ref.max()
    # the profile is symmetric about the mid-plane
    assert np.allclose(u_sim, u_sim[::-1], rtol=1e-6)


def _flagged_cells(L, centre, R):
    """Cells whose centre (i + 1/2) lies within R of the sphere centre (no wrap needed here)."""
    i = np.arange(L) + 0.5
    X, Y, Zc = np.meshgrid(i, i, i, indexing="ij")
    return int(np.sum((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Zc - centre[2]) ** 2 <= R * R))


def _frame_run(L, R, centre, mode, Z, E, steps, every, pv=True):
    """A charged sphere with its counterions (a neutral system) in a field E
    along x.  Returns per sample the
    sphere velocity, the mean fluid velocity along x and the flagged cell count."""
    # charge: Z Psi / V_p with partial volumes (Sec. III.D.2), else Z spread over the boundary cells
    p = O.make_params(L, L, L, 1 / 6, 1.0, 0.7, (E, 0.0, 0.0), [(0.3, -1)], charge_mode=0 if pv else 1,
                      integrator=0, partial_volume=pv)
    sph = [dict(x=centre, R=R, Z=Z, M=2 * (4 / 3) * np.pi * R ** 3, mode=mode)]
    N = L ** 3
    probe = O.OracleSim(p, sph, np.ones(N))
    fluid = probe.flag == 0
    s = O.OracleSim(p, sph, np.where(fluid, Z / fluid.sum(), 0.0))
    out = []
    for _ in range(steps // every):
        s.run(every)
        fl = s.flag == 0
        out.append((s.particles()[0]["v"][0], s.u[:N][fl].mean(), np.count_nonzero(~fl)))
    return np.array(out)


@pytest.mark.slow
@pytest.mark.parametrize("pv", [False])
def test_electrophoresis_matches_comoving_electroosmosis(pv):
    """A freely moving charged sphere (electrophoresis) against the same sphere
    held fixed while its counterions drive the fluid past it (electro-osmosis,
    the co-moving frame): in the stationary state the sphere's speed relative to
    the bulk fluid is the same (Sec. IV, single-sphere comparison).  As in the
    paper, the moving particle (partial-volume or simple scheme) and the fixed
    one (the method with fixed boundaries: centre-inside cells) are compared at
    the same effective size: the moving particle's boundary cells -- in the
    partial-volume scheme the cells completely inside it -- are counted and
    averaged over time, and the fixed sphere's radius and lattice offset are
    chosen so that its count of boundary cells equals that average.  The paper
    reports agreement to 1.4 % (simple scheme) and 2.4 % (partial volumes); the
    bar here is 3 % (observed 1.4 %, simple scheme).  The partial-volume
    comparison needs the paper's own system (Table I, 64^3, tens of thousands of
    steps) and runs on the GPU: in boxes this small the cut shell, fluid to the
    LB but partly closed to the solute, is a sizeable part of the particle, and
    the two frames differ by 5-6 %."""
    L, Z, E = 16, 10.0, 0.01
    steps, every = 2400, 100
    free = _frame_run(L, 3.0 if not pv else 3.6, (8.0, 8.0, 8.0), 0, Z, E, steps, every, pv=pv)
    half = len(free) // 2
    v_rel = np.mean(free[half:, 0] - free[half:, 1])   # sphere relative to the bulk fluid
    n_cells = np.mean(free[half:, 2])
    assert v_rel > 0.0                                   # a positive sphere moves along +E
    # fixed sphere of the same effective size
    cands = sorted((abs(_flagged_cells(L, c, R) - n_cells), round(R, 2), c)
                   for R in np.arange(2.5, 3.6, 0.01)
                   for c in ((8.0, 8.0, 8.0), (8.5, 8.5, 8.5), (8.0, 8.5, 8.5), (8.0, 8.0, 8.5)))
    _, R_f, c_f = cands[0]
    fixed = _frame_run(L, R_f, c_f, 2, Z, E, steps, every, pv=False)
    u_eo = fixed[:, 1]
    print("pv", pv, "v_rel", v_rel, "boundary cells", n_cells, "fixed R", R_f, c_f, "EO", -u_eo[-1],
          "ratio", v_rel / -u_eo[-1])
    assert abs(u_eo[-1] / u_eo[-5] - 1) < 1e-3         # the electro-osmotic flow is stationary
    assert np.all(fixed[:, 0] == 0.0)
    assert abs(v_rel / -u_eo[-1] - 1) < 0.03, (v_rel, -u_eo[-1], R_f, c_f, n_cells)
