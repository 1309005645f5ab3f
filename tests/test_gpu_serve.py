"""Serving form on the GPU: batched steps of several simulations in one arena.

- A request gives the same bits alone and in a mix of other requests admitted
  at different times (every simulation's arithmetic is independent of the
  batch).
- A batched request gives the same bits as the single-simulation path.
- Admission is by footprint: a request that does not fit is refused with
  EK_ERR_NO_SPACE and fits once memory is freed.
- The serve loop completes a small seeded request stream."""
import numpy as np
import pytest

from paper_1607_04572_amd import workloads as W
from paper_1607_04572_amd.ek import EkBatch, EkError, EkSim
from parity_util import say

pytestmark = pytest.mark.gpu


def req(name, L, R, Z, n, E, c, seed, steps):
    pos = W.place_spheres(n, R, (L, L, L), seed=seed)
    return W.Workload(name=name, shape=(L, L, L), precision="fp32", species=W.salt(0.3, c), lambda_B=0.7,
                      E=(E, 0.0, 0.0), steps=steps, seed=seed,
                      spheres=[W.Sphere(x=p, R=R, Z=Z, M=2 * W.sphere_volume(R)) for p in pos])


A = req("A", 48, 4.0, 30.0, 3, 0.02, 0.01, 11, 60)
B = req("B", 32, 3.5, 20.0, 1, 0.01, 0.005, 12, 90)
C = req("C", 64, 5.0, 40.0, 4, 0.03, 0.015, 13, 40)


def final_state_batch(order, steps_between, target="A"):
    """Admit the requests of `order` one after another with `steps_between`
    batched steps in between; run until everything is done; return the final
    fields and particles of `target`."""
    b = EkBatch(4 << 30)
    slots = {}
    out = None
    for k, w in enumerate(order):
        slots[w.name] = b.admit(w, initial_density=W.initial_densities(w))
        if k < len(order) - 1:
            b.step(steps_between)
    finished = set()
    while len(finished) < len(order):
        b.step(7)
        for s in b.poll():
            name = [n for n, v in slots.items() if v == s][0]
            finished.add(name)
            if name == target:
                out = {f: b.field(s, f) for f in ("density", "populations", "phi", "velocity", "psi", "flag")}
                out["particles"], _ = b.collect(s)
            else:
                b.collect(s)
    b.close()
    return out


def assert_same(a, b):
    for k in ("density", "populations", "phi", "velocity", "psi", "flag"):
        assert np.array_equal(a[k], b[k]), k
    for pa, pb in zip(a["particles"], b["particles"]):
        for f in ("x", "v", "omega", "F", "T"):
            assert np.array_equal(pa[f], pb[f]), f


def test_alone_equals_mix_bitwise():
    say("case alone vs mix")
    alone = final_state_batch([A], 0)
    mix1 = final_state_batch([B, A, C], 13)
    mix2 = final_state_batch([C, B, A], 5)
    assert_same(alone, mix1)
    assert_same(alone, mix2)


def test_batch_equals_single_path():
    say("case batch vs single")
    batch = final_state_batch([A], 0)
    g = EkSim(A, initial_density=W.initial_densities(A))
    g.step(A.steps)
    single = {f: g.field(f) for f in ("density", "populations", "phi", "velocity", "psi", "flag")}
    single["particles"] = g.particles()
    g.close()
    assert_same(batch, single)


def test_simple_scheme_in_a_mix_equals_single_path():
    """A simple-scheme request batched beside partial-volume ones (the batched
    step then includes the refill kernels, which it leaves out while no live
    request uses that scheme) gives the same bits as the single-simulation
    path, and so does a partial-volume request of the same mix."""
    say("case simple scheme in a mix")
    S = A.replace(name="S", scheme="simple")
    for target, w in (("S", S), ("B", B)):
        batch = final_state_batch([B, S, C], 9, target=target)
        g = EkSim(w, initial_density=W.initial_densities(w))
        g.step(w.steps)
        single = {f: g.field(f) for f in ("density", "populations", "phi", "velocity", "psi", "flag")}
        single["particles"] = g.particles()
        g.close()
        assert_same(batch, single)


def test_admission_by_footprint():
    say("case admission")
    from paper_1607_04572_amd.ek import ek_query_footprint, params_from_workload
    need = ek_query_footprint(params_from_workload(C, max_particles=len(C.spheres)))
    b = EkBatch(need + need // 2 + (1 << 20))
    s1 = b.admit(C, n_steps=3)
    with pytest.raises(EkError) as e:
        b.admit(C, n_steps=3)
    assert e.value.code == -6
    b.step(3)
    assert b.poll(wait=True) == [s1]
    b.collect(s1)
    s2 = b.admit(C, n_steps=2)
    b.step(2)
    assert b.poll(wait=True) == [s2]
    b.collect(s2)
    b.close()


def test_serve_loop_small_stream():
    from paper_1607_04572_amd import serve
    say("case serve loop")
    reqs = W.serve_requests(12, seed=5, rate=50.0, steps=30)
    res = serve.run(reqs, arena_bytes=8 << 30, chunk=10)
    say(res)
    assert res["requests"] == 12 and res["p99_s"] >= res["p50_s"] > 0 and res["mlups"] > 0


def test_seeded_density_equals_host_recipe():
    """Seeded initial densities built on the device (ek_seed_density) are the
    values of the host recipe workloads.initial_densities, stored bit for bit
    as the host-array path stores them: FP32 deviations and FP64 plain, a cell
    count that is not a multiple of the 256-cell launch blocks, two seeds;
    and the two states stay equal through steps."""
    import dataclasses
    sph = [W.Sphere(x=(9.0, 6.0, 6.0), R=3.0, Z=10.0, M=2 * W.sphere_volume(3.0))]
    for prec, seed, shape in (("fp32", 5, (24, 18, 12)), ("fp64", 2 ** 40 + 3, (18, 12, 24))):
        w = dataclasses.replace(W.c0(), shape=shape, precision=prec, spheres=sph, seed=seed, charge="psi")
        say(f"case seeded density {prec} seed={seed} shape={w.shape}")
        a = EkSim(w, initial_density=W.initial_densities(w))
        b = EkSim(w, seeded=True)
        assert np.array_equal(a.field("density"), b.field("density"))
        a.step(4)
        b.step(4)
        for f in ("density", "populations", "phi", "velocity"):
            assert np.array_equal(a.field(f), b.field(f)), f
        a.close()
        b.close()


def test_seeded_admission_equals_host_array():
    say("case seeded admission")
    out = []
    for seeded in (False, True):
        b = EkBatch(2 << 30)
        s = b.admit(C, seeded=True) if seeded else b.admit(C, initial_density=W.initial_densities(C))
        b.step(9)
        out.append({f: b.field(s, f) for f in ("density", "populations", "phi", "velocity", "flag")})
        b.close()
    for f in out[0]:
        assert np.array_equal(out[0][f], out[1][f]), f
