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
