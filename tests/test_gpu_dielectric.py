"""Poisson's equation with an inhomogeneous permittivity on the GPU
(ek_set_permittivity: Jacobi-preconditioned conjugate gradients in FP64;
Sec. III.C names iterative solvers for a varying dielectric) through the C ABI.

- Permittivity 1 everywhere: the iterative path gives the FFT path's step.
- A layered dielectric (a slab of permittivity 8) with charge sheets: the
  potential equals the exact solution of the 1-D problem.
- A random permittivity with a slab, moving charged spheres and salt: the
  full step against the oracle (whose Poisson solve is a sparse direct solve
  of the same equation), FP64 and FP32."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_04572_amd import ek as E
from paper_1607_04572_amd import workloads as W
from parity_util import compare, make_gpu, make_oracle, ok_fp32, ok_fp64, say

pytestmark = pytest.mark.gpu

SHAPE = (24, 16, 12)


def eps_field(seed=7):
    nx, ny, nz = SHAPE
    rng = np.random.default_rng(seed)
    x = np.tile(np.arange(nx), ny * nz)
    eps = rng.uniform(1.0, 3.0, nx * ny * nz)
    eps[(x >= 14) & (x < 19)] = 8.0
    return eps


def workload(precision, spheres=True):
    sph = [W.Sphere(x=(6.3, 8.2, 6.1), R=3.2, Z=25.0, M=300.0, v=(0.05, 0.01, 0.0), mode=1),
           W.Sphere(x=(17.6, 7.7, 5.8), R=2.8, Z=-15.0, M=200.0)] if spheres else []
    return W.Workload(name=f"dielectric_{precision}", shape=SHAPE, precision=precision, species=W.salt(0.3, 0.01),
                      lambda_B=0.7, E=(0.01, 0.004, 0.0), steps=10, spheres=sph)


def test_unit_permittivity_equals_fft():
    w = workload("fp64")
    a, b = make_gpu(w), make_gpu(w)
    a.prepare()
    b.prepare()
    E.ek_set_permittivity(b.ctx, np.ones(w.cells), tol=1e-14, max_iter=5000)
    a.step(3)
    b.step(3)
    it, res = E.ek_get_poisson_stats(b.ctx)
    say("unit permittivity: iterations", it, "residual", res)
    for f in ("phi", "density", "populations", "velocity"):
        ga, gb = a.field(f), b.field(f)
        err = np.max(np.abs(ga - gb)) / max(np.max(np.abs(ga)), 1e-300)
        say(f, f"{err:.3e}")
        assert err < 1e-11, (f, err)
    a.close()
    b.close()


def test_layered_dielectric_exact():
    """Charge sheets between slabs of permittivity 1 and 8 (x-layered): the
    potential of the first step is the exact 1-D series solution."""
    nx, ny, nz = SHAPE
    x = np.arange(nx)
    eps1 = np.where((x >= 8) & (x < 16), 8.0, 1.0)
    sheets = np.zeros(nx)
    sheets[3], sheets[11], sheets[20] = 0.02, -0.008, -0.012
    w = W.Workload(name="layered", shape=SHAPE, precision="fp64", species=[W.Species(0.1, 1, 0.01)],
                   lambda_B=0.7, E=(0.0, 0.0, 0.0), steps=1, spheres=[], noise=0.0)
    rho = np.tile(0.01 + sheets, ny * nz)[None, :]
    g = make_gpu(w, rho0=rho)
    E.ek_set_permittivity(g.ctx, np.tile(eps1, ny * nz), tol=1e-14, max_iter=5000)
    g.step(1)
    phi = g.field("phi").reshape(nz, ny, nx)
    q1 = 0.01 + sheets
    b = 4 * np.pi * 0.7 * (q1 - q1.mean())
    ef = 2 * eps1 * np.roll(eps1, -1) / (eps1 + np.roll(eps1, -1))
    S = np.cumsum(b)
    C = -np.sum(S / ef) / np.sum(1 / ef)
    steps = (S + C) / ef
    ref = np.concatenate([[0.0], -np.cumsum(steps[:-1])])
    ref -= ref.mean()
    err = np.max(np.abs(phi - ref[None, None, :])) / np.max(np.abs(ref))
    say("layered: iterations", E.ek_get_poisson_stats(g.ctx), "error", f"{err:.3e}")
    assert err < 1e-12
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_dielectric_steps_against_oracle(precision):
    w = workload(precision)
    eps = eps_field()
    o = make_oracle(w, permittivity=eps)
    g = make_gpu(w)
    g.prepare()
    E.ek_set_permittivity(g.ctx, eps, tol=1e-14, max_iter=5000)
    done = 0
    for cp in (1, 4, 10):
        g.step(cp - done)
        o.run(cp - done)
        done = cp
        e = compare(w, g, o, f"{w.name} step {cp}")
        say("  poisson iterations, residual", E.ek_get_poisson_stats(g.ctx))
        ok_fp64(e) if precision == "fp64" else ok_fp32(e)
    g.close()
