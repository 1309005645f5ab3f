"""Error paths of the C ABI, each forced from the host (include/ek.h).

- EK_ERR_OVERLAP: spheres that intersect (directly or through the periodic
  boundary) are refused by ek_add_sphere.
- EK_ERR_UNSTABLE: the volume-of-fluid advection (Sec. III.C) displaces a
  cell by u tau and intersects it with its neighbours only, so every velocity
  component must stay below one cell per step.  A fluid cell given momentum
  1.5 through ek_set_fields, or a free sphere kicked past one cell per step
  by a large force, latches the error on the device; the next synchronising
  call reports it, and so does the next ek_step once the stream has passed
  the step that latched it; every later call on the context returns it.
- EK_ERR_NONFINITE: populations at the largest finite value overflow to
  infinity and NaN in the next collision.
- Serving form: a request that fails is stopped, reported by the poll and
  retired with its error; the other requests of the batch are unaffected.
All of these run to completion on the device (no data-dependent indexing)."""
import numpy as np
import pytest

from paper_1607_04572_amd import ek as E
from paper_1607_04572_amd import workloads as W
from parity_util import make_gpu, say

pytestmark = pytest.mark.gpu

W19 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def box(precision, spheres=(), E_ext=(0.01, 0.0, 0.0), n=16):
    return W.Workload(name=f"err_{precision}", shape=(n, n, n), precision=precision, species=W.salt(0.3, 0.01),
                      lambda_B=0.7, E=E_ext, steps=4, spheres=list(spheres))


def expect(code, fn, *a):
    with pytest.raises(E.EkError) as ex:
        fn(*a)
    assert ex.value.code == code, (ex.value.code, code)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_overlapping_spheres_refused(precision):
    w = box(precision)
    g = E.EkSim(w, max_particles=4)
    E.ek_add_sphere(g.ctx, (5.0, 8.0, 8.0), 3.0, 10.0, 100.0)
    say("overlap", precision)
    expect(-4, E.ek_add_sphere, g.ctx, (10.5, 8.0, 8.0), 2.6, 10.0, 100.0)  # centres 5.5 apart, radii 5.6
    expect(-4, E.ek_add_sphere, g.ctx, (15.5, 8.0, 8.0), 2.8, 10.0, 100.0)  # 5.5 apart through the periodic face, radii 5.8
    assert E.ek_add_sphere(g.ctx, (11.0, 8.0, 8.0), 2.9, 10.0, 100.0) == 1  # 6 apart, radii 5.9
    g.close()


def populations_with(w, cell, values):
    N = w.cells
    f = np.tile(W19[:, None], (1, N))
    for i, v in values.items():
        f[i, cell] = v
    return f.reshape(-1)


def torch_sync():
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fluid_faster_than_one_cell_per_step(precision):
    w = box(precision)
    g = make_gpu(w)
    g.prepare()
    c = 8 + 16 * (8 + 16 * 8)
    g.set_field("populations", populations_with(w, c, {1: W19[1] + 1.5}))
    say("unstable fluid", precision)
    g.step(2)
    torch_sync()
    expect(-3, E.ek_step, g.ctx, 1)       # the next ek_step sees the latched status
    expect(-3, E.ek_synchronize, g.ctx)   # and every later call
    expect(-3, E.ek_get_diagnostics, g.ctx)
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_free_sphere_faster_than_one_cell_per_step(precision):
    # a light, strongly charged sphere in a strong field: F_el ~ Z E = 5 on a
    # mass of 1 kicks it far past one cell per step after the first step
    w = box(precision, [W.Sphere(x=(8.0, 8.0, 8.0), R=3.0, Z=50.0, M=1.0)], E_ext=(0.1, 0.0, 0.0))
    g = make_gpu(w)
    g.prepare()
    say("unstable sphere", precision)
    g.step(3)
    expect(-3, E.ek_synchronize, g.ctx)
    expect(-3, E.ek_get_particles, g.ctx, 1)
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_nonfinite_state(precision):
    w = box(precision)
    g = make_gpu(w)
    g.prepare()
    c = 5 + 16 * (9 + 16 * 7)
    big = 1.7e308 if precision == "fp64" else 3.0e38
    g.set_field("populations", populations_with(w, c, {1: big, 2: big, 3: big, 4: big}))
    say("non-finite", precision)
    g.step(3)
    expect(-7, E.ek_get_fields, g.ctx, "density", w.cells, 2)
    expect(-7, E.ek_step, g.ctx, 1)
    g.close()


def test_batch_retires_a_failed_request():
    ok = W.Workload(name="ok", shape=(32, 32, 32), precision="fp32", species=W.salt(0.3, 0.01), lambda_B=0.7,
                    E=(0.01, 0.0, 0.0), steps=20,
                    spheres=[W.Sphere(x=(16.0, 16.0, 16.0), R=4.0, Z=20.0, M=2 * W.sphere_volume(4.0))])
    bad = W.Workload(name="bad", shape=(32, 32, 32), precision="fp32", species=W.salt(0.3, 0.01), lambda_B=0.7,
                     E=(0.1, 0.0, 0.0), steps=20,
                     spheres=[W.Sphere(x=(10.0, 12.0, 16.0), R=3.0, Z=50.0, M=1.0)])
    b = E.EkBatch(1 << 30)
    s_ok = b.admit(ok, seeded=True)
    s_bad = b.admit(bad, seeded=True)
    say("batch with a failing request")
    done = set()
    for _ in range(10):
        b.step(4)
        done |= set(b.poll(wait=True))
        if s_ok in done:
            break
    assert s_bad in done and s_ok in done
    with pytest.raises(E.EkError) as ex:
        b.collect(s_bad)
    assert ex.value.code == -3
    parts, diag = b.collect(s_ok)
    assert diag["step"] == 20 and np.all(np.isfinite(parts[0]["v"]))
    assert b.active() == (0, 0)
    b.close()
