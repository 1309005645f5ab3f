"""Pins of the oracle's periodic Poisson solve (Eq. poisson, FFT solver of
Sec. III.C)."""
import numpy as np

from oracle import oracle as O


def laplacian7(phi3):
    out = -6 * phi3
    for ax in range(3):
        out = out + np.roll(phi3, 1, axis=ax) + np.roll(phi3, -1, axis=ax)
    return out


def test_single_mode_closed_form():
    nx, ny, nz = 16, 12, 8
    lb = 0.7
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    m = (3, 2, 1)
    arg = 2 * np.pi * (m[0] * x / nx + m[1] * y / ny + m[2] * z / nz)
    q = 0.05 * np.cos(arg) + 0.3  # the constant is removed (neutralising background)
    phi = O.poisson(q.reshape(-1), nx, ny, nz, lb).reshape(nz, ny, nx)
    K2 = sum(2 - 2 * np.cos(2 * np.pi * mm / n) for mm, n in zip(m, (nx, ny, nz)))
    assert np.allclose(phi, 4 * np.pi * lb * 0.05 * np.cos(arg) / K2, rtol=0, atol=1e-14)


def test_dense_direct_solve_8cube():
    """Brute force: assemble the periodic 7-point Laplacian as a dense matrix and
    solve it (with the zero-mean condition) directly."""
    n = 8
    N = n ** 3
    rng = np.random.default_rng(0)
    q = rng.normal(size=N)
    A = np.zeros((N, N))
    for zz in range(n):
        for yy in range(n):
            for xx in range(n):
                i = xx + n * (yy + n * zz)
                A[i, i] = -6
                for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    j = (xx + dx) % n + n * ((yy + dy) % n + n * ((zz + dz) % n))
                    A[i, j] += 1
    lb = 0.9
    rhs = -4 * np.pi * lb * (q - q.mean())
    Aug = np.vstack([A, np.ones((1, N))])
    sol = np.linalg.lstsq(Aug, np.concatenate([rhs, [0.0]]), rcond=None)[0]
    phi = O.poisson(q, n, n, n, lb)
    assert np.max(np.abs(phi - sol)) < 1e-12 * np.max(np.abs(sol))


def test_laplacian_property_any_size():
    nx, ny, nz = 18, 12, 10
    rng = np.random.default_rng(1)
    q = rng.normal(size=nx * ny * nz) + 2.0
    lb = 0.7
    phi = O.poisson(q, nx, ny, nz, lb).reshape(nz, ny, nx)
    lap = laplacian7(phi)
    q3 = q.reshape(nz, ny, nx)
    assert np.allclose(lap, -4 * np.pi * lb * (q3 - q3.mean()), rtol=0, atol=1e-12)
    assert abs(phi.mean()) < 1e-14


# -- inhomogeneous permittivity (iterative-solver path of Sec. III.C) ----------
def test_dielectric_uniform_equals_fft():
    """eps = const: the solution is the FFT one divided by the constant."""
    nx, ny, nz = 12, 10, 8
    rng = np.random.default_rng(3)
    q = rng.normal(size=nx * ny * nz)
    phi = O.poisson_dielectric(q, np.full(q.size, 2.5), nx, ny, nz, 0.7)
    ref = O.poisson(q, nx, ny, nz, 0.7) / 2.5
    assert np.max(np.abs(phi - ref)) < 1e-12 * np.max(np.abs(ref))


def layered_exact(q1, eps1, lb):
    """Exact discrete solution of a 1-D periodic problem (charge and
    permittivity varying along x only): the face flux F_i = e_(i+1/2)
    (phi_i - phi_(i+1)) obeys F_i - F_(i-1) = 4 pi lb (q_i - mean q), so F is
    a cumulative sum plus a constant C, and the constant makes the potential
    steps F_i / e_(i+1/2) sum to zero around the ring."""
    n = q1.size
    b = 4 * np.pi * lb * (q1 - q1.mean())
    ef = 2 * eps1 * np.roll(eps1, -1) / (eps1 + np.roll(eps1, -1))
    S = np.cumsum(b)  # F_i - C
    C = -np.sum(S / ef) / np.sum(1 / ef)
    steps = (S + C) / ef  # phi_i - phi_(i+1)
    phi = np.concatenate([[0.0], -np.cumsum(steps[:-1])])
    return phi - phi.mean()


def test_dielectric_layered_closed_form():
    """A slab of permittivity 8 between slabs of 1 (x-layered), with charge
    sheets: the 3-D solve equals the exact 1-D series-capacitor solution on
    every y-z column."""
    nx, ny, nz = 24, 6, 4
    x = np.arange(nx)
    eps1 = np.where((x >= 8) & (x < 16), 8.0, 1.0)
    q1 = np.zeros(nx)
    q1[3], q1[11], q1[20] = 1.0, -0.4, -0.6  # neutral: the flux is constant between sheets
    eps = np.tile(eps1, ny * nz)
    q = np.tile(q1, ny * nz)
    phi = O.poisson_dielectric(q, eps, nx, ny, nz, 0.7).reshape(nz, ny, nx)
    ref = layered_exact(q1, eps1, 0.7)
    assert np.max(np.abs(phi - ref[None, None, :])) < 1e-12 * np.max(np.abs(ref))
    # the field jumps by the permittivity ratio across an uncharged interface
    e_left = phi[0, 0, 6] - phi[0, 0, 7]
    e_right = phi[0, 0, 8] - phi[0, 0, 9]
    assert abs(e_left / e_right - 8.0) < 1e-9


def test_dielectric_reciprocity():
    """Green's reciprocity for any symmetric discretisation: the potential at
    cell b due to a unit charge at a equals that at a due to the same charge at
    b (random permittivity field)."""
    nx, ny, nz = 10, 8, 6
    N = nx * ny * nz
    rng = np.random.default_rng(5)
    eps = rng.uniform(0.5, 4.0, N)
    a, b = 17, 301
    qa = np.zeros(N)
    qa[a] = 1.0
    qb = np.zeros(N)
    qb[b] = 1.0
    pa = O.poisson_dielectric(qa, eps, nx, ny, nz, 0.7)
    pb = O.poisson_dielectric(qb, eps, nx, ny, nz, 0.7)
    assert abs(pa[b] - pb[a]) < 1e-12 * abs(pa[a])
    assert abs(pa[b] - pb[a]) < 1e-12 * abs(pa[b]) + 1e-15
