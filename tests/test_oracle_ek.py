"""Pins of the oracle's EK solute update (Sec. III.C, III.D.2) against closed
forms and invariants that the paper and the continuum equations fix."""
import math

import numpy as np
import pytest

from oracle import oracle as O

A0 = 1.0 + 2.0 * math.sqrt(2.0)
C19 = O.D3Q19_C


def grid(shape):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.reshape(-1).astype(float), y.reshape(-1).astype(float), z.reshape(-1).astype(float)


def params(shape, D=0.2, z=0, E=(0, 0, 0), pv=True, kT=1.0):
    return O.make_params(*shape, 1 / 6, kT, 0.0, E, [(D, z)], partial_volume=pv)


def zeros(shape, k=1):
    return np.zeros(k * int(np.prod(shape)))


def test_msd_grows_by_6D_per_step():
    """Sec. III.C: A0 = 1 + 2 sqrt 2 recovers the mean-square displacement 6 D t."""
    shape = (16, 16, 16)
    D = 0.23
    p = params(shape, D=D)
    N = int(np.prod(shape))
    x, y, z = grid(shape)
    rho = np.zeros(N)
    rng = np.random.default_rng(3)
    blob = (abs(x - 8) <= 1) & (abs(y - 8) <= 1) & (abs(z - 8) <= 1)
    rho[blob] = rng.uniform(0.5, 1.5, blob.sum())
    out, _ = O.ek_update(p, rho, zeros(shape), zeros(shape), np.zeros(N, np.uint8), zeros(shape, 3))

    def moments(r):
        m = r.sum()
        c = np.array([(r * x).sum(), (r * y).sum(), (r * z).sum()]) / m
        s2 = (r * ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)).sum() / m
        return m, c, s2

    m0, c0, s0 = moments(rho)
    m1, c1, s1 = moments(out)
    assert abs(m1 - m0) < 1e-13 * m0
    assert np.allclose(c1, c0, atol=1e-13)
    assert abs((s1 - s0) - 6 * D) < 1e-12


def test_fourier_mode_decay_factor():
    """A single Fourier mode is an eigenvector of the diffusive update with the
    factor 1 - (D/A0) sum_i (1 - cos k.c_i)/|c_i| (the discrete Laplacian of the
    flux of Sec. III.C)."""
    shape = (12, 16, 8)
    D = 0.31
    p = params(shape, D=D)
    N = int(np.prod(shape))
    x, y, z = grid(shape)
    k = 2 * np.pi * np.array([2 / 12, 3 / 16, 1 / 8])
    mode = np.cos(k[0] * x + k[1] * y + k[2] * z + 0.3)
    rho = 1.0 + 0.01 * mode
    out, _ = O.ek_update(p, rho, zeros(shape), zeros(shape), np.zeros(N, np.uint8), zeros(shape, 3))
    lam = 1 - D / A0 * sum((1 - np.cos(k @ c)) / np.linalg.norm(c) for c in C19[1:])
    assert np.allclose(out - 1.0, lam * 0.01 * mode, atol=1e-15, rtol=0)


def test_uniform_field_drift_is_DzE():
    """Einstein relation of Eq. flux: mobility D/kT, so the centre of mass of a
    species of valency z moves by D z E per step in a uniform field."""
    shape = (16, 16, 16)
    D, zval = 0.27, -2
    E = (0.013, -0.021, 0.017)
    p = params(shape, D=D, z=zval, E=E)
    N = int(np.prod(shape))
    x, y, zc = grid(shape)
    rng = np.random.default_rng(5)
    rho = np.where((abs(x - 8) <= 2) & (abs(y - 8) <= 2) & (abs(zc - 8) <= 2), rng.uniform(0.5, 1.5, N), 0.0)
    out, _ = O.ek_update(p, rho, zeros(shape), zeros(shape), np.zeros(N, np.uint8), zeros(shape, 3))
    m0, m1 = rho.sum(), out.sum()
    c0 = np.array([(rho * g).sum() for g in (x, y, zc)]) / m0
    c1 = np.array([(out * g).sum() for g in (x, y, zc)]) / m1
    assert np.allclose(c1 - c0, D * zval * np.array(E), atol=1e-14, rtol=0)


def overlap_fraction(u, s):
    """Volume of the unit cube displaced by u that lies in the neighbour cube at
    offset s: per axis max(0, min(u+1, s+1) - max(u, s))."""
    f = 1.0
    for d in range(3):
        f *= max(0.0, min(u[d] + 1.0, s[d] + 1.0) - max(u[d], s[d]))
    return f


def test_vof_advection_is_cube_intersection():
    """Sec. III.C: the solute of a cell displaced by u is split over the 26
    neighbours by the intersection volumes of the displaced cube."""
    shape = (8, 8, 8)
    p = params(shape, D=0.0)
    N = 512
    u = np.array([0.31, -0.17, 0.06])
    c = 4 + 8 * (4 + 8 * 4)
    rho = np.zeros(N)
    rho[c] = 1.0
    uf = np.zeros(3 * N)
    for d in range(3):
        uf[d * N + c] = u[d]
    out, _ = O.ek_update(p, rho, zeros(shape), zeros(shape), np.zeros(N, np.uint8), uf)
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                n = (4 + sx) + 8 * ((4 + sy) + 8 * (4 + sz))
                assert abs(out[n] - overlap_fraction(u, (sx, sy, sz))) < 1e-15
    assert abs(out.sum() - 1.0) < 1e-15


def test_uniform_velocity_moves_centre_by_u():
    shape = (16, 16, 16)
    p = params(shape, D=0.1)
    N = int(np.prod(shape))
    x, y, z = grid(shape)
    rng = np.random.default_rng(7)
    rho = np.where((abs(x - 8) <= 2) & (abs(y - 8) <= 2) & (abs(z - 8) <= 2), rng.uniform(0.5, 1.5, N), 0.0)
    u = np.array([0.12, -0.33, 0.05])
    uf = np.repeat(u, N)
    out, _ = O.ek_update(p, rho, zeros(shape), zeros(shape), np.zeros(N, np.uint8), uf)
    c0 = np.array([(rho * g).sum() for g in (x, y, z)]) / rho.sum()
    c1 = np.array([(out * g).sum() for g in (x, y, z)]) / out.sum()
    assert np.allclose(c1 - c0, u, atol=1e-14, rtol=0)


def boltzmann_ring(phi_x, zval, nx):
    """rho(x+1)/rho(x) = (1 + z dphi/2)/(1 - z dphi/2), dphi = phi(x) - phi(x+1)."""
    r = np.empty(nx)
    r[0] = 1.0
    for i in range(nx - 1):
        dphi = phi_x[i] - phi_x[i + 1]
        r[i + 1] = r[i] * (1 + zval * dphi / 2) / (1 - zval * dphi / 2)
    return r


@pytest.mark.parametrize("with_psi", [False, True])
def test_even_potential_zero_flux_equilibrium(with_psi):
    """Zero field, an imposed even 1-D potential: the concentration with
    link ratios (1 + z dphi/2)/(1 - z dphi/2) closes on the ring and carries
    zero flux on every link, so nothing changes and the coupling force vanishes.
    With partial volumes the solute amount is concentration * (1 - Psi)
    (Eq. flux-pv), for any Psi.  This pins the sign of the migrative term and
    the equal prefactor of both terms; exp(-z phi) is recovered to O(dphi^3)."""
    shape = (24, 6, 4)
    nx = shape[0]
    zval = 1
    p = params(shape, D=0.25, z=zval, pv=True)
    N = int(np.prod(shape))
    x, y, z = grid(shape)
    xs = np.arange(nx)
    phi_x = 0.3 * np.cos(2 * np.pi * xs / nx)
    c_x = boltzmann_ring(phi_x, zval, nx)
    # the ring closes exactly because the potential differences pair up
    last = phi_x[-1] - phi_x[0]
    closure = c_x[-1] * (1 + zval * last / 2) / (1 - zval * last / 2)
    assert abs(closure - 1.0) < 1e-14
    conc = 0.01 * c_x[x.astype(int)]
    phi = phi_x[x.astype(int)]
    psi = np.random.default_rng(1).uniform(0.0, 0.9, N) if with_psi else np.zeros(N)
    rho = conc * (1 - psi)
    out, fext = O.ek_update(p, rho, phi, psi, np.zeros(N, np.uint8), zeros(shape, 3))
    assert np.max(np.abs(out - rho)) < 1e-17
    assert np.max(np.abs(fext)) < 1e-15
    # Boltzmann to third order in the potential step
    boltz = np.exp(-zval * (phi_x - phi_x[0]))
    assert np.max(np.abs(c_x / boltz - 1)) < 2e-3


def test_random_potential_does_not_close():
    """A non-even potential gives a product of link ratios != 1 on the ring, so
    the even-potential closure above is not automatic."""
    rng = np.random.default_rng(2)
    phi_x = rng.uniform(-0.3, 0.3, 24)
    c = boltzmann_ring(phi_x, 1, 24)
    last = phi_x[-1] - phi_x[0]
    assert abs(c[-1] * (1 + last / 2) / (1 - last / 2) - 1.0) > 1e-4


def test_coupling_force_uniform_field():
    """Eq. fluidcoupling: for a uniform solute in a uniform field the force
    density on the fluid is kT sum_k z_k rho_k E."""
    shape = (8, 8, 8)
    E = (0.011, -0.007, 0.003)
    p = O.make_params(*shape, 1 / 6, 1.7, 0.0, E, [(0.3, 1), (0.2, -2), (0.1, 3)])
    N = 512
    rho = np.concatenate([np.full(N, 0.01), np.full(N, 0.02), np.full(N, 0.005)])
    out, fext = O.ek_update(p, rho, zeros(shape), zeros(shape), np.zeros(N, np.uint8), zeros(shape, 3))
    q = 1 * 0.01 - 2 * 0.02 + 3 * 0.005
    for d in range(3):
        assert np.allclose(fext[d * N:(d + 1) * N], 1.7 * q * E[d], rtol=1e-13, atol=1e-18)
    assert np.allclose(out, rho, rtol=0, atol=1e-17)


def test_coupling_force_gradient():
    """For z = 0 and a linear profile the force density is -kT grad rho."""
    shape = (16, 8, 8)
    p = O.make_params(*shape, 1 / 6, 1.3, 0.0, (0, 0, 0), [(0.2, 0)])
    N = int(np.prod(shape))
    x, y, z = grid(shape)
    b = (0.002, -0.001, 0.0005)
    rho = 0.5 + b[0] * x + b[1] * y + b[2] * z
    _, fext = O.ek_update(p, rho, zeros(shape), zeros(shape), np.zeros(N, np.uint8), zeros(shape, 3))
    interior = (x > 1) & (x < 14) & (y > 1) & (y < 6) & (z > 1) & (z < 6)
    for d in range(3):
        assert np.allclose(fext[d * N:(d + 1) * N][interior], -1.3 * b[d], rtol=1e-12, atol=0)


def test_mass_conserved_and_boundary_cells_closed():
    """Sec. III.C: no flux into or out of boundary cells; the update is a flux
    divergence, so the total of every species is conserved."""
    shape = (12, 10, 8)
    N = int(np.prod(shape))
    rng = np.random.default_rng(11)
    p = O.make_params(*shape, 1 / 6, 1.0, 0.0, (0.01, 0.02, -0.01), [(0.3, 1), (0.15, -1)])
    rho = rng.uniform(0.005, 0.02, 2 * N)
    flag = (rng.uniform(size=N) < 0.15).astype(np.uint8)
    rho[:N][flag == 1] = 0.0
    rho[N:][flag == 1] = 0.0
    psi = np.where(flag == 1, 1.0, rng.uniform(0, 0.8, N) * (rng.uniform(size=N) < 0.3))
    phi = rng.normal(scale=0.2, size=N)
    u = rng.uniform(-0.3, 0.3, 3 * N)
    out, fext = O.ek_update(p, rho, phi, psi, flag, u)
    for k in range(2):
        assert abs(out[k * N:(k + 1) * N].sum() - rho[k * N:(k + 1) * N].sum()) < 1e-15 * N
        assert np.all(out[k * N:(k + 1) * N][flag == 1] == 0.0)
    for d in range(3):
        assert np.all(fext[d * N:(d + 1) * N][flag == 1] == 0.0)


def test_isolated_fluid_cell_keeps_its_solute():
    """A fluid cell whose 26 neighbours are all boundary exchanges nothing."""
    shape = (8, 8, 8)
    N = 512
    p = O.make_params(*shape, 1 / 6, 1.0, 0.0, (0.05, 0, 0), [(0.3, 1)])
    flag = np.zeros((8, 8, 8), np.uint8)
    flag[3:6, 3:6, 3:6] = 1
    flag[4, 4, 4] = 0
    rho = np.full(N, 0.01)
    rho[flag.reshape(-1) == 1] = 0
    u = np.full(3 * N, 0.2)
    out, _ = O.ek_update(p, rho, np.random.default_rng(0).normal(size=N), np.zeros(N), flag, u)
    assert out[4 + 8 * (4 + 8 * 4)] == 0.01
