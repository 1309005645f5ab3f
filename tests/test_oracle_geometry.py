"""Pins of the oracle's geometry (Sec. III.D.2 partial volume, Fig. 1 boundary
cells) against brute force and closed forms."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def brute_psi_count(dx, dy, dz, R):
    """Depth-4 sub-cell centres (a 16^3 grid inside the cell) that lie in the
    sphere.  Whole sub-boxes decided inside/outside contain only centres on the
    same side, so the recursive count equals this count away from exact ties."""
    t = (np.arange(16) + 0.5) / 16.0 - 0.5
    X, Y, Z = np.meshgrid(dx + t, dy + t, dz + t, indexing="ij")
    return int(((X * X + Y * Y + Z * Z) <= R * R).sum())


def test_psi_extremes():
    L = O.lib()
    assert L.or_psi_count(0.0, 0.0, 0.0, 4.0) == 4096
    assert L.or_psi_count(1.0, 1.0, 1.0, 4.0) == 4096
    assert L.or_psi_count(5.0, 0.0, 0.0, 4.0) == 0
    assert L.or_psi_count(4.6, 0.0, 0.0, 4.0) == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_psi_matches_subcell_centre_count(seed):
    rng = np.random.default_rng(seed)
    L = O.lib()
    for _ in range(300):
        R = rng.uniform(0.7, 7.0)
        d = rng.normal(size=3)
        d *= (R + rng.uniform(-1.0, 1.0)) / np.linalg.norm(d)
        assert L.or_psi_count(*d, R) == brute_psi_count(*d, R)


@pytest.mark.parametrize("R", [3.0, 4.0, 5.3, 6.0])
def test_psi_total_volume(R):
    """sum_cells Psi approximates 4/3 pi R^3 (midpoint rule on a 1/16 grid)."""
    p = O.make_params(24, 24, 24, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.3, 1)])
    x = (12.31, 11.87, 12.05)
    flag, owner, psi, rhob = O.geometry(p, [dict(x=x, R=R, Z=10.0, M=1.0)])
    V = 4 / 3 * math.pi * R ** 3
    assert abs(psi.sum() - V) / V < 2e-3
    # Psi is dyadic (multiples of 1/4096) and within [0, 1]
    assert np.all(psi * 4096 == np.round(psi * 4096))
    assert psi.min() >= 0.0 and psi.max() <= 1.0
    # Psi-distributed charge: sum rho_b = Z sum Psi / V_p
    assert abs(rhob.sum() - 10.0 * psi.sum() / V) < 1e-12


def _disp(shape, s):
    nx, ny, nz = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    out = []
    for ax, (g, L) in enumerate(zip((xx, yy, zz), (nx, ny, nz))):
        dd = g + 0.5 - s["x"][ax]
        out.append(np.where(dd > L / 2, dd - L, np.where(dd < -L / 2, dd + L, dd)))
    return out


def brute_flags(shape, parts, pv):
    """Owner of each cell by brute force: the lowest-index particle that claims
    it -- simple scheme: the cell centre is inside (Fig. 1 caption);
    partial-volume scheme: the cell is completely inside, i.e. all 16^3 leaf
    centres of its depth-4 subdivision are (Psi_p = 1)."""
    nx, ny, nz = shape
    owner = np.full((nz, ny, nx), -1)
    for k, s in enumerate(parts):
        dx, dy, dz = _disp(shape, s)
        if not pv:
            claim = dx * dx + dy * dy + dz * dz <= s["R"] ** 2
        else:
            claim = np.zeros_like(owner, dtype=bool)
            near = np.argwhere((np.abs(dx) < s["R"]) & (np.abs(dy) < s["R"]) & (np.abs(dz) < s["R"]))
            for z, y, x in near:
                claim[z, y, x] = brute_psi_count(dx[z, y, x], dy[z, y, x], dz[z, y, x], s["R"]) == 4096
        owner[claim & (owner < 0)] = k
    return owner.reshape(-1)


@pytest.mark.parametrize("pv", [False, True])
def test_flags_owner_bruteforce_periodic(pv):
    """Three spheres, one wrapping across the periodic boundary, two
    overlapping: the boundary flag and the owner (lowest index) against brute
    force, for each scheme's rule of when a particle claims a cell."""
    shape = (16, 12, 20)
    parts = [dict(x=(0.7, 11.2, 19.4), R=3.3, Z=5.0, M=1.0),
             dict(x=(3.1, 1.0, 1.5), R=2.6, Z=7.0, M=1.0),
             dict(x=(9.5, 6.5, 10.5), R=4.0, Z=1.0, M=1.0)]
    p = O.make_params(*shape, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.3, 1)], charge_mode=1, partial_volume=pv)
    flag, owner, psi, rhob = O.geometry(p, parts)
    ref = brute_flags(shape, parts, pv)
    assert np.array_equal(owner, ref)
    assert np.array_equal(flag, (ref >= 0).astype(np.uint8))
    assert (ref >= 0).sum() > 100
    if pv:
        # every claimed cell is full, and every cell some particle covers fully is claimed
        assert np.all(psi[flag == 1] == 1.0)
    # uniform charge mode: each particle's charge is spread exactly over its cells
    for k, s in enumerate(parts):
        assert abs(rhob[owner == k].sum() - s["Z"]) < 1e-12
    assert np.all(rhob[owner < 0] == 0)


def test_partial_volume_claims_fewer_cells_than_centre_rule():
    """A cell whose centre is inside but which is cut by the surface is a
    boundary cell in the simple scheme and a fluid cell (0 < Psi < 1) in the
    partial-volume scheme."""
    shape = (16, 16, 16)
    parts = [dict(x=(8.3, 7.9, 8.1), R=4.2, Z=5.0, M=1.0)]
    f_pv = O.geometry(O.make_params(*shape, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.3, 1)], partial_volume=True), parts)
    f_si = O.geometry(O.make_params(*shape, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.3, 1)], partial_volume=False), parts)
    pv_flag, si_flag, psi = f_pv[0], f_si[0], f_pv[2]
    assert np.all(si_flag[pv_flag == 1] == 1)
    cut = (si_flag == 1) & (pv_flag == 0)
    assert cut.sum() > 50 and np.all((psi[cut] > 0) & (psi[cut] < 1))


def test_psi_sum_capped_at_one():
    p = O.make_params(16, 16, 16, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.3, 1)])
    parts = [dict(x=(8.0, 8.0, 8.0), R=3.0, Z=1, M=1), dict(x=(10.0, 8.0, 8.0), R=3.0, Z=1, M=1)]
    flag, owner, psi, rhob = O.geometry(p, parts)
    p1 = O.geometry(p, parts[:1])[2]
    p2 = O.geometry(p, parts[1:])[2]
    assert np.array_equal(psi, np.minimum(1.0, p1 + p2))


def test_psi_recursion_equals_leaf_count_at_ties():
    """Near ties: radii chosen so that one depth-4 leaf centre lies (in FP64)
    exactly on the sphere.  The recursive subdivision and the plain count of
    leaf centres with fl(fl(cx^2 + cy^2) + cz^2) <= R^2 must still agree (the
    GPU counts leaf centres directly)."""
    rng = np.random.default_rng(11)
    L = O.lib()
    t = (2 * np.arange(16) + 1) / 32.0
    hits = 0
    for _ in range(400):
        d = rng.uniform(-6, 6, 3)
        lo = d - 0.5
        i, j, k = rng.integers(0, 16, 3)
        cx, cy, cz = lo[0] + t[i], lo[1] + t[j], lo[2] + t[k]
        R = float(np.sqrt((cx * cx + cy * cy) + cz * cz))
        X, Y, Z = np.meshgrid(lo[0] + t, lo[1] + t, lo[2] + t, indexing="ij")
        direct = int((((X * X + Y * Y) + Z * Z) <= R * R).sum())
        assert L.or_psi_count(*d, R) == direct
        hits += direct not in (0, 4096)
    assert hits > 100
