"""GPU parity on the stated workload configurations, through the C ABI.

- 64^3 FP32, one free sphere: trajectory against the oracle.
- 128^3 FP32, 8 free spheres, 3 species: trajectory for a few steps, and one
  oracle step resumed from the GPU state after 100 steps.
- 256^3 FP32 and FP64, 64 free spheres (the configuration bench.py times, with
  the same graph-replayed launches): one oracle step resumed from the GPU
  state, and conservation over the run.

A resumed comparison starts both sides from the same state (populations,
densities, velocity, flags, owners, particles), so it isolates one step's
arithmetic at full size; flags, owners and Psi must agree exactly."""
import numpy as np
import pytest

from paper_1607_04572_amd import workloads as W
from parity_util import compare, make_gpu, make_oracle, ok_fp32, ok_fp64, say, snapshot

pytestmark = pytest.mark.gpu


def fp32_ok(e):
    ok_fp32(e)
    assert e["rhob"] < 1e-6


def fp64_ok(e):
    ok_fp64(e)


def resume_one_step(w, warm, ok):
    say(f"case {w.name}: {warm} GPU steps, then one step on both sides")
    g = make_gpu(w)
    g.prepare()
    t0 = g.diagnostics()["species_total"][:len(w.species)]
    g.step(warm)
    g.sync()
    o = snapshot(g, w)
    g.step(1)
    g.sync()
    o.step()
    e = compare(w, g, o, f"{w.name} resumed +1")
    ok(e)
    t1 = np.asarray(g.diagnostics()["species_total"][:len(w.species)])
    g.close()
    return np.asarray(t0), t1


@pytest.mark.timeout(600)
def test_c1_64cube_fp32_free_sphere_trajectory():
    """Fields agree to FP32 rounding while the two trajectories stay within
    rounding of each other; later, the sphere positions (FP64 on both sides,
    driven by forces summed from FP32 fields on the GPU) drift apart by
    ~1e-6 cells, enough for a depth-4 leaf centre to sit on different sides of
    the surface, so only the trajectory is compared there; the resumed step
    checks the arithmetic again at that time."""
    w = W.c1("fp32")
    say(f"case {w.name}")
    g = make_gpu(w)
    o = make_oracle(w)
    g.prepare()
    done = 0
    for n in (1, 50, 200):
        g.step(n - done)
        o.run(n - done)
        done = n
        e = compare(w, g, o, f"{w.name} step {n}")
        ok_fp32(e, fields=n <= 50)
        assert e["particle_x"] < 1e-5
    g.close()
    resume_one_step(w, 200, fp32_ok)


@pytest.mark.timeout(600)
def test_c2_128cube_fp32_three_species():
    w = W.c2("fp32")
    say(f"case {w.name} trajectory")
    g = make_gpu(w)
    o = make_oracle(w)
    g.prepare()
    done = 0
    for n in (1, 5):
        g.step(n - done)
        o.run(n - done)
        done = n
        e = compare(w, g, o, f"{w.name} step {n}")
        fp32_ok(e)
    g.close()
    resume_one_step(w, 100, fp32_ok)


@pytest.mark.timeout(900)
def test_c3_256cube_fp32_resumed_step_and_conservation():
    w = W.c3("fp32")
    t0, t1 = resume_one_step(w, 40, fp32_ok)
    # solute is conserved link by link; the FP32 deviations round each update
    assert np.all(np.abs(t1 / t0 - 1) < 1e-9), (t0, t1)
    say("species totals", t0, t1)


@pytest.mark.timeout(900)
def test_c3_256cube_fp64_resumed_step():
    w = W.c3("fp64")
    t0, t1 = resume_one_step(w, 10, fp64_ok)
    assert np.all(np.abs(t1 / t0 - 1) < 1e-12), (t0, t1)
