"""Pins of the oracle's LB stream/collide (Sec. III.A: TRT collision, Guo force
term, velocity bounce-back)."""
import numpy as np
import pytest

from oracle import oracle as O

C19 = O.D3Q19_C
W19 = O.D3Q19_W


def run_lb(p, f, flag, owner, fext, steps, parts=None, tol=None):
    u = None
    for s in range(steps):
        f_new, u = O.lb_update(p, f, flag, owner, fext, parts)
        if tol is not None and np.max(np.abs(f_new - f)) < tol:
            f = f_new
            break
        f = f_new
    return f, u


@pytest.mark.parametrize("nu", [1 / 6, 0.5, 0.05])
def test_poiseuille_exact_with_magic_parameter(nu):
    """Force-driven flow between resting walls.  With the TRT magic parameter
    3/16 the bounce-back wall sits exactly half-way between nodes, so the
    discrete steady profile equals the parabola u = g/(2 nu) (x - 1/2)(L - 1/2 - x)
    for any viscosity.  This pins the reading of "lambda_o = 3/16", the Guo
    force term (Eq. guo) and the half-force velocity."""
    nx, ny, nz = 12, 2, 2
    p = O.make_params(nx, ny, nz, nu, 1.0, 0.0, (0, 0, 0), [(0.1, 0)])
    N = nx * ny * nz
    x = np.tile(np.arange(nx), ny * nz)
    flag = (x == 0).astype(np.uint8)
    owner = np.full(N, -1, np.int32)
    g = 1e-5
    fext = np.zeros(3 * N)
    fext[N:2 * N][flag == 0] = g
    f = np.tile(W19[:, None], (1, N)).reshape(-1)
    f, u = run_lb(p, f, flag, owner, fext, 60000, tol=1e-18)
    uy = u[N:2 * N]
    xf = x[flag == 0].astype(float)
    ref = g / (2 * nu) * (xf - 0.5) * (nx - 0.5 - xf)
    assert np.max(np.abs(uy[flag == 0] - ref)) < 1e-10 * ref.max()
    assert np.max(np.abs(u[:N])) < 1e-10 * ref.max() and np.max(np.abs(u[2 * N:])) < 1e-10 * ref.max()


@pytest.mark.parametrize("nu", [1 / 6, 0.05])
def test_couette_exact_with_a_moving_wall(nu):
    """Velocity bounce-back (Sec. III.A): a plane of boundary cells at x = m
    owned by a particle moving at (0, U, 0), a resting plane at x = 0, periodic
    in x.  The steady profile of each channel is linear between the walls, which
    sit half-way between nodes: u_y = U (x - 1/2) / (m - 1) between the resting
    and the moving wall, U (nx - 1/2 - x) / (nx - m - 1) beyond.  A wrong sign
    or factor of the wall term 6 w_i c_i.u_b, or the wall velocity of another
    cell, moves the profile off the lines."""
    nx, ny, nz, m = 14, 2, 2, 6
    p = O.make_params(nx, ny, nz, nu, 1.0, 0.0, (0, 0, 0), [(0.1, 0)])
    N = nx * ny * nz
    x = np.tile(np.arange(nx), ny * nz)
    flag = ((x == 0) | (x == m)).astype(np.uint8)
    owner = np.where(x == m, 0, -1).astype(np.int32)
    U = 1e-3
    parts = [dict(x=(m + 0.5, 1.0, 1.0), R=0.5, Z=0.0, M=1.0, v=(0.0, U, 0.0), mode=1)]
    f = np.tile(W19[:, None], (1, N)).reshape(-1)
    f, u = run_lb(p, f, flag, owner, np.zeros(3 * N), 200000, parts=parts, tol=1e-19)
    uy = u[N:2 * N]
    a = (x > 0) & (x < m)
    b = x > m
    assert np.max(np.abs(uy[a] - U * (x[a] - 0.5) / (m - 1))) < 1e-9 * U
    assert np.max(np.abs(uy[b] - U * (nx - 0.5 - x[b]) / (nx - m - 1))) < 1e-9 * U
    fl = flag == 0
    assert np.max(np.abs(u[:N][fl])) < 1e-9 * U and np.max(np.abs(u[2 * N:][fl])) < 1e-9 * U


def test_rest_state_is_stationary():
    nx, ny, nz = 6, 5, 4
    N = nx * ny * nz
    p = O.make_params(nx, ny, nz, 1 / 6, 1.0, 0.0, (0, 0, 0), [(0.1, 0)])
    flag = np.zeros(N, np.uint8)
    flag[7] = flag[40] = 1
    f = np.tile(W19[:, None], (1, N)).reshape(-1)
    out, u = O.lb_update(p, f, flag, np.full(N, -1, np.int32), np.zeros(3 * N))
    assert np.max(np.abs(out - f)) < 1e-16
    assert np.max(np.abs(u)) < 1e-16


def streamed(f, shape):
    """Plain periodic streaming f_i(r) <- f_i(r - c_i) on the (19, nz, ny, nx) grid."""
    nx, ny, nz = shape
    f4 = f.reshape(19, nz, ny, nx)
    out = np.empty_like(f4)
    for i, c in enumerate(C19):
        out[i] = np.roll(f4[i], shift=(c[2], c[1], c[0]), axis=(0, 1, 2))
    return out.reshape(19, -1)


def test_collision_conserves_mass_and_adds_force():
    """Eq. lb with Omega + Delta: the collision keeps the density and raises
    the momentum by exactly the force density (sum_i Delta_i = 0,
    sum_i Delta_i c_i = f)."""
    shape = (7, 6, 5)
    N = 210
    rng = np.random.default_rng(4)
    rho = 1 + 0.01 * rng.normal(size=N)
    u = 0.02 * rng.normal(size=(3, N))
    f = (O.equilibrium(rho, u) + 1e-4 * rng.normal(size=(19, N))).reshape(-1)
    fext = 1e-3 * rng.normal(size=3 * N)
    out, uo = O.lb_update(O.make_params(*shape, 0.11, 1.0, 0.0, (0, 0, 0), [(0.1, 0)]),
                          f, np.zeros(N, np.uint8), np.full(N, -1, np.int32), fext)
    fs = streamed(f, shape)
    fo = out.reshape(19, N)
    Cf = C19.T.astype(float)
    assert np.allclose(fo.sum(0), fs.sum(0), rtol=0, atol=1e-15)
    j_in, j_out = Cf @ fs, Cf @ fo
    assert np.allclose(j_out, j_in + fext.reshape(3, N), rtol=0, atol=1e-16)
    # the reported velocity is the half-force velocity
    assert np.allclose(uo.reshape(3, N), j_in + 0.5 * fext.reshape(3, N), rtol=0, atol=1e-16)


def test_resting_walls_conserve_mass():
    shape = (10, 8, 6)
    N = 480
    rng = np.random.default_rng(8)
    flag = (rng.uniform(size=N) < 0.2).astype(np.uint8)
    f = (O.equilibrium(1 + 0.01 * rng.normal(size=N), 0.03 * rng.normal(size=(3, N)))).reshape(-1)
    p = O.make_params(*shape, 1 / 6, 1.0, 0.0, (0, 0, 0), [(0.1, 0)])
    out, _ = O.lb_update(p, f, flag, np.full(N, -1, np.int32), np.zeros(3 * N))
    fl = flag == 0
    assert abs(out.reshape(19, N)[:, fl].sum() - f.reshape(19, N)[:, fl].sum()) < 1e-12


def test_shear_wave_decay():
    """A transverse shear wave decays at the rate nu k^2 (Stokes, Eq. stokes),
    up to the O(k^2) lattice correction."""
    nx, ny, nz = 32, 2, 2
    N = nx * ny * nz
    nu = 0.1
    p = O.make_params(nx, ny, nz, nu, 1.0, 0.0, (0, 0, 0), [(0.1, 0)])
    x = np.tile(np.arange(nx), ny * nz)
    k = 2 * np.pi / nx
    u = np.zeros((3, N))
    u[1] = 1e-3 * np.sin(k * x)
    f = O.equilibrium(np.ones(N), u).reshape(-1)
    flag = np.zeros(N, np.uint8)
    owner = np.full(N, -1, np.int32)
    amps = []
    for t in range(301):
        f, uo = O.lb_update(p, f, flag, owner, np.zeros(3 * N))
        if t in (100, 300):
            amps.append((uo[N:2 * N] * np.sin(k * x)).sum() * 2 / N)
    rate = np.log(amps[0] / amps[1]) / 200
    assert abs(rate / (nu * k * k) - 1) < 0.01
