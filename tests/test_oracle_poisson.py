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
