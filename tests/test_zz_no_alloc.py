"""The allocation-free step (ek_step_noalloc, include/ek.h) against ek_step
through the C ABI: the same kernels with the particle partial sums in the
library's fixed per-GPU array instead of the context's arena, so the results
must agree bit for bit.  Two calls in a row, the second on a smaller system
(fewer spheres and workgroups, so the array still holds the first call's
larger contents beyond what the second writes); and a system whose partial
sums exceed the array is refused with EK_ERR_NO_SPACE."""
import numpy as np
import pytest

from paper_1607_04572_amd import ek as E
from paper_1607_04572_amd import workloads as W
from parity_util import make_gpu, say

pytestmark = pytest.mark.gpu

FIELDS = ("density", "populations", "phi", "velocity", "force", "psi", "flag", "owner", "particle_charge")


def spheres_case(edge, n, R, precision, seed):
    pos = W.place_spheres(n, R, (edge,) * 3, seed=seed)
    return W.Workload(name=f"noalloc_{edge}_{n}_{precision}", shape=(edge,) * 3, precision=precision,
                      species=W.salt(0.3, 0.01), lambda_B=0.7, E=(0.01, 0.005, 0.0), steps=12,
                      spheres=[W.Sphere(x=c, R=R, Z=30.0, M=2 * W.sphere_volume(R)) for c in pos])


def run_pair(w, steps):
    say(f"case {w.name}: {steps} steps by ek_step and by ek_step_noalloc")
    a = make_gpu(w)
    b = make_gpu(w)
    a.prepare()
    b.prepare()
    a.step(steps)
    E.ek_step_noalloc(b.ctx, steps)
    b.sync()
    for f in FIELDS:
        assert np.array_equal(a.field(f), b.field(f)), f
    for pa, pb in zip(a.particles(), b.particles()):
        for k in ("x", "v", "omega", "F", "T", "F_hyd", "F_el", "F_cov"):
            assert np.array_equal(pa[k], pb[k]), k
    da, db = a.diagnostics(), b.diagnostics()
    assert da["step"] == db["step"] == steps
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_step_equals_step_two_calls(precision):
    run_pair(spheres_case(48, 8, 6.0, precision, seed=31), 13)  # odd: ends on the other ping-pong half
    run_pair(spheres_case(24, 2, 3.5, precision, seed=32), 6)


def test_noalloc_step_refuses_oversized_partials():
    # 128 spheres of radius 6: 12 workgroups per box, 3 x 128 x 12 x 128 B = 576 KiB > 512 KiB
    w = spheres_case(128, 128, 6.0, "fp32", seed=33)
    g = make_gpu(w)
    g.prepare()
    with pytest.raises(E.EkError) as ex:
        E.ek_step_noalloc(g.ctx, 1)
    assert ex.value.code == -6
    g.step(1)  # the arena path still runs it
    g.close()
