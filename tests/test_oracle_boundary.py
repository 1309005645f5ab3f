"""Pins of the oracle's moving-boundary update (Sec. III.B Aidun destroy/create,
Sec. III.D solute expel/refill), forces (Eq. force, electrostatic force) and the
particle integrator, against hand-built cases and exact conservation laws."""
import numpy as np
import pytest

from oracle import oracle as O

C19 = O.D3Q19_C
W19 = O.D3Q19_W


def idx(x, y, z, n):
    return (x % n) + n * ((y % n) + n * (z % n))


def base(n=8, ns=1, pv=True):
    p = O.make_params(n, n, n, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.3, 1)] * ns, partial_volume=pv)
    N = n ** 3
    f = np.tile(W19[:, None], (1, N)).reshape(-1)
    return p, N, f


def test_expel_equal_shares_to_d3q19_neighbours():
    p, N, f = base()
    n = 8
    c = idx(3, 4, 5, n)
    flag_old = np.zeros(N, np.uint8)
    flag_new = flag_old.copy()
    flag_new[c] = 1
    owner = np.full(N, -1, np.int32)
    owner_new = owner.copy()
    owner_new[c] = 0
    rho = np.full(N, 0.1)
    rho[c] = 1.0
    part = [dict(x=(3.5, 4.5, 5.5), R=0.4, Z=0, M=1)]
    _, out, _, _, counts = O.boundary_update(p, part, flag_old, owner, flag_new, owner_new, f, rho)
    assert out[c] == 0.0
    for cv in C19[1:]:
        assert abs(out[idx(3 + cv[0], 4 + cv[1], 5 + cv[2], n)] - (0.1 + 1 / 18)) < 1e-15
    assert abs(out.sum() - rho.sum()) < 1e-13
    assert tuple(counts) == (1, 0, 0)


def test_expel_falls_back_to_d3q27_then_pool():
    p, N, f = base()
    n = 8
    flag_old = np.zeros((n, n, n), np.uint8)
    # a 3x3x3 block of boundary cells without its 8 corners, so the centre's 18
    # D3Q19 neighbours are boundary but its 8 corner neighbours are fluid
    flag_old[2:5, 2:5, 2:5] = 1
    for a in (2, 4):
        for b in (2, 4):
            for e in (2, 4):
                flag_old[a, b, e] = 0
    flag_old[3, 3, 3] = 0
    flag_new = flag_old.copy()
    flag_new[3, 3, 3] = 1
    flag_old, flag_new = flag_old.reshape(-1), flag_new.reshape(-1)
    own_old = np.where(flag_old == 1, 0, -1).astype(np.int32)
    own_new = np.where(flag_new == 1, 0, -1).astype(np.int32)
    c = idx(3, 3, 3, n)
    rho = np.where(flag_old == 1, 0.0, 0.2)
    rho[c] = 0.8
    part = [dict(x=(3.5, 3.5, 3.5), R=0.5, Z=0, M=1)]
    _, out, _, _, counts = O.boundary_update(p, part, flag_old, own_old, flag_new, own_new, f, rho)
    corners = [idx(3 + a, 3 + b, 3 + e, n) for a in (-1, 1) for b in (-1, 1) for e in (-1, 1)]
    for q in corners:
        assert abs(out[q] - (0.2 + 0.8 / 8)) < 1e-15
    assert out[c] == 0.0 and abs(out.sum() - rho.sum()) < 1e-13
    # now close the corners too: the solute goes to the global pool
    flag_old2 = flag_old.copy()
    flag_old2[corners] = 1
    flag_new2 = flag_new.copy()
    flag_new2[corners] = 1
    own_old2 = np.where(flag_old2 == 1, 0, -1).astype(np.int32)
    own_new2 = np.where(flag_new2 == 1, 0, -1).astype(np.int32)
    rho2 = np.where(flag_old2 == 1, 0.0, 0.2)
    rho2[c] = 0.8
    _, out2, _, _, counts2 = O.boundary_update(p, part, flag_old2, own_old2, flag_new2, own_new2, f, rho2)
    stable = (flag_old2 == 0) & (flag_new2 == 0)
    assert np.allclose(out2[stable], 0.2 + 0.8 / stable.sum(), rtol=0, atol=1e-15)
    assert counts2[2] == 1 and abs(out2.sum() - rho2.sum()) < 1e-13


def test_aidun_destroy_and_create():
    """Covered cell: its fluid momentum goes to the particle.  Vacated cell:
    equilibrium at the surface velocity and the mean density of its stable
    fluid neighbours; its momentum is taken from the particle."""
    p, N, f = base()
    n = 8
    rng = np.random.default_rng(3)
    f = (f.reshape(19, N) * (1 + 0.05 * rng.normal(size=(19, N)))).reshape(-1)
    c = idx(2, 2, 2, n)
    v = idx(5, 5, 5, n)
    flag_old = np.zeros(N, np.uint8)
    flag_old[v] = 1
    flag_new = np.zeros(N, np.uint8)
    flag_new[c] = 1
    own_old = np.where(flag_old == 1, 0, -1).astype(np.int32)
    own_new = np.where(flag_new == 1, 0, -1).astype(np.int32)
    part = [dict(x=(4.0, 4.0, 4.0), R=1.0, Z=0, M=1, v=(0.01, -0.02, 0.005), w=(0.001, 0.002, -0.003))]
    rho = np.full(N, 0.01)
    f_out, _, Fc, Tc, counts = O.boundary_update(p, part, flag_old, own_old, flag_new, own_new, f, rho)
    F = f.reshape(19, N)
    p_destroy = C19.T @ F[:, c]
    r_v = np.array([5.5, 5.5, 5.5]) - 4.0
    vb = np.array(part[0]["v"]) + np.cross(part[0]["w"], r_v)
    dens = [F[:, idx(5 + cv[0], 5 + cv[1], 5 + cv[2], n)].sum() for cv in C19[1:]]
    rbar = np.mean(dens)
    feq = O.equilibrium(np.array([rbar]), vb.reshape(3, 1))[:, 0]
    assert np.allclose(f_out.reshape(19, N)[:, v], feq, rtol=0, atol=1e-16)
    assert np.allclose(Fc[0], p_destroy - vb, rtol=0, atol=1e-15)
    r_c = np.array([2.5, 2.5, 2.5]) - 4.0
    assert np.allclose(Tc[0], np.cross(r_c, p_destroy) - np.cross(r_v, vb), rtol=0, atol=1e-15)
    assert tuple(counts) == (1, 1, 0)


def test_simple_scheme_refill():
    """Eqs. refill and refill-neighbours: the vacated cell receives
    sum rho_n/(N_f+1) from its N_f stable neighbours, each of which keeps
    N_f/(N_f+1) of its solute."""
    p, N, f = base(pv=False)
    n = 8
    v = idx(4, 4, 4, n)
    flag_old = np.zeros(N, np.uint8)
    flag_old[v] = 1
    flag_old[idx(5, 4, 4, n)] = 1  # one neighbour stays boundary
    flag_new = np.zeros(N, np.uint8)
    flag_new[idx(5, 4, 4, n)] = 1
    own_old = np.where(flag_old == 1, 0, -1).astype(np.int32)
    own_new = np.where(flag_new == 1, 0, -1).astype(np.int32)
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.01, 0.02, N)
    rho[flag_old == 1] = 0.0
    part = [dict(x=(5.0, 4.5, 4.5), R=1.0, Z=0, M=1)]
    _, out, _, _, _ = O.boundary_update(p, part, flag_old, own_old, flag_new, own_new, f, rho)
    nbrs = [idx(4 + cv[0], 4 + cv[1], 4 + cv[2], n) for cv in C19[1:] if not (cv[0] == 1 and cv[1] == 0 and cv[2] == 0)]
    Nf = len(nbrs)
    assert Nf == 17
    assert abs(out[v] - sum(rho[m] for m in nbrs) / (Nf + 1)) < 1e-16
    for m in nbrs:
        assert abs(out[m] - rho[m] * Nf / (Nf + 1)) < 1e-16
    assert abs(out.sum() - rho.sum()) < 1e-15


def test_integrators_constant_force():
    """Velocity Verlet: x_n = x0 + n v0 + a n^2 / 2; symplectic Euler:
    x_n = x0 + n v0 + a n (n+1) / 2 (Sec. III.B)."""
    for integ, ref in ((0, lambda n, a: n * n / 2 * a), (1, lambda n, a: n * (n + 1) / 2 * a)):
        p = O.make_params(1000, 1000, 1000, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.1, 0)], integrator=integ)
        pt = O.make_particles([dict(x=(100.0, 200.0, 300.0), v=(0.01, 0.0, -0.02), R=2.0, Z=0, M=4.0)])
        F = np.array([0.004, -0.002, 0.001])
        T = np.array([0.0, 0.0, 0.0])
        pt[0].F[:] = F  # force of the (fictitious) previous step
        nsteps = 50
        for _ in range(nsteps):
            O.move(p, pt)
            O.finish(p, pt, F, T)
        a = F / 4.0
        x = np.array(pt[0].x[:])
        expect = np.array([100.0, 200.0, 300.0]) + nsteps * np.array([0.01, 0.0, -0.02]) + ref(nsteps, a)
        assert np.allclose(x, expect, rtol=0, atol=1e-10)


def sim(n, parts, species=((0.3, 1, 0.01), (0.3, -1, 0.01)), E=(0.01, 0, 0), lb=0.7, charge_mode=0,
        pv=True, integ=0, seed=5):
    p = O.make_params(n, n, n, 1 / 6, 1.0, lb, E, [(D, z) for D, z, _ in species],
                      partial_volume=pv, charge_mode=charge_mode, integrator=integ)
    N = n ** 3
    rng = np.random.default_rng(seed)
    rho = np.concatenate([m * (1 + 0.01 * (2 * rng.uniform(size=N) - 1)) for _, _, m in species])
    return O.OracleSim(p, parts, rho)


@pytest.mark.parametrize("pv", [True, False])
def test_solute_conserved_through_moving_boundaries(pv):
    """Sec. III.D: expel (and refill) conserve every species to rounding while
    a sphere crosses cells; densities stay non-negative."""
    s = sim(16, [dict(x=(8.2, 8.1, 7.9), R=3.2, Z=10, M=100, v=(0.23, 0.11, -0.07), mode=1)], pv=pv)
    tot0 = s.species_totals()
    covered = 0
    for _ in range(25):
        s.step()
        covered += s.last["covered"] + s.last["vacated"]
        assert np.allclose(s.species_totals(), tot0, rtol=1e-14, atol=0)
        assert s.rho.min() >= 0.0
        assert np.all(s.density()[:, s.flag == 1] == 0.0)
    assert covered > 50


def test_momentum_budget_exact():
    """Fluid momentum changes by the force density minus what the particles
    received (bounce-back momentum exchange, Eq. force, and the Aidun
    destroy/create impulses): P(n) - P(n-1) = sum f_ext - sum_p (F_hyd + F_cov)."""
    s = sim(16, [dict(x=(8.0, 8.0, 8.0), R=3.5, Z=30, M=200, v=(0.05, -0.03, 0.02))], E=(0.02, 0.01, 0))
    for _ in range(20):
        P0 = s.fluid_momentum()
        s.step()
        P1 = s.fluid_momentum()
        fsum = s.fext.reshape(3, -1).sum(axis=1)
        Fp = (s.last["F_hyd"] + s.last["F_cov"]).sum(axis=0)
        assert np.allclose(P1 - P0, fsum - Fp, rtol=0, atol=1e-13)


def test_drag_opposes_motion():
    s = sim(16, [dict(x=(8.0, 8.0, 8.0), R=3.0, Z=0, M=100, v=(0.02, 0.0, 0.0), mode=1)],
            species=((0.3, 1, 0.0),), E=(0, 0, 0), lb=0.0)
    for _ in range(15):
        s.step()
    F = s.last["F_hyd"][0] + s.last["F_cov"][0]
    assert F[0] < 0 and abs(F[1]) < 1e-3 * abs(F[0]) and abs(F[2]) < 1e-3 * abs(F[0])


@pytest.mark.parametrize("charge_mode", [0, 1])
def test_isolated_charged_sphere_feels_only_external_field(charge_mode):
    """No solute: the particle's own potential exerts no net force (the
    Green's function is symmetric and the gradient antisymmetric), so
    F_el = kT (sum_r rho_b) E."""
    E = (0.013, -0.004, 0.007)
    s = sim(16, [dict(x=(7.3, 8.6, 8.1), R=3.4, Z=25, M=100, mode=2)], species=((0.3, 1, 0.0),),
            E=E, charge_mode=charge_mode)
    s.step()
    Q = s.rhob.sum()
    if charge_mode == 1:
        assert abs(Q - 25) < 1e-12
    assert np.allclose(s.last["F_el"][0], Q * np.array(E), rtol=1e-11, atol=0)


def test_fixed_uncharged_sphere_in_fluid_at_rest_stays_at_rest():
    s = sim(12, [dict(x=(6.0, 6.0, 6.0), R=3.0, Z=0, M=100, mode=2)], species=((0.3, 1, 0.0),),
            E=(0, 0, 0), lb=0.0)
    f0 = s.f.copy()
    for _ in range(3):
        s.step()
    fl = np.tile(s.flag == 0, 19)
    assert np.max(np.abs(s.f[fl] - f0[fl])) < 1e-16
    assert np.max(np.abs(s.last["F_hyd"])) < 1e-14


def test_electrostatic_torque_is_dipole_cross_field():
    """With lambda_B = 0 (no self-field) the electrostatic torque on a charged
    sphere is kT sum_r rho_b(r) (r - r_p) x E: computed here independently from
    the particle's charge density and minimum-image arms."""
    n = 16
    E = np.array([0.013, -0.004, 0.007])
    x = np.array([7.3, 8.6, 8.1])
    s = sim(n, [dict(x=tuple(x), R=3.4, Z=25, M=100, mode=2)], species=((0.3, 1, 0.0),), E=tuple(E), lb=0.0)
    s.step()
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    arm = np.stack([g.reshape(-1) + 0.5 - c for g, c in zip((xx, yy, zz), x)])
    arm = np.where(arm > n / 2, arm - n, np.where(arm < -n / 2, arm + n, arm))
    dip = (s.rhob[None, :] * arm).sum(axis=1)
    assert np.allclose(s.last["T_el"][0], np.cross(dip, E), rtol=1e-12, atol=1e-15)
    assert np.allclose(s.last["F_el"][0], s.rhob.sum() * E, rtol=1e-12, atol=0)


def test_hydrodynamic_torque_opposes_rotation_and_vanishes_for_symmetric_translation():
    """A sphere spinning in fluid at rest feels a torque against its spin (and
    no force); a sphere translating along x with mirror-symmetric geometry
    feels no torque."""
    spin = sim(20, [dict(x=(10.0, 10.0, 10.0), R=3.5, Z=0, M=100, w=(0.0, 0.0, 0.004), mode=1)],
               species=((0.3, 1, 0.0),), E=(0, 0, 0), lb=0.0)
    for _ in range(30):
        spin.step()
    T = spin.last["T_hyd"][0]
    assert T[2] < 0 and abs(T[0]) < 1e-10 * abs(T[2]) and abs(T[1]) < 1e-10 * abs(T[2])
    assert np.max(np.abs(spin.last["F_hyd"][0])) < 1e-10 * abs(T[2])
    move = sim(20, [dict(x=(10.0, 10.0, 10.0), R=3.5, Z=0, M=100, v=(0.02, 0.0, 0.0), mode=1)],
               species=((0.3, 1, 0.0),), E=(0, 0, 0), lb=0.0)
    for _ in range(10):
        move.step()
    F = move.last["F_hyd"][0] + move.last["F_cov"][0]
    T = move.last["T_hyd"][0] + move.last["T_cov"][0]
    assert np.max(np.abs(T)) < 1e-12 * abs(F[0])


@pytest.mark.parametrize("pv", [True, False])
def test_initial_state_rule(pv):
    """Fluid at rest with f_i = w_i; no solute in boundary cells; with partial
    volumes a fluid cell holds (1 - Psi) of the given concentration."""
    n = 12
    p = O.make_params(n, n, n, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.3, 1), (0.2, -1)], partial_volume=pv)
    rng = np.random.default_rng(2)
    rho0 = rng.uniform(0.005, 0.015, 2 * n ** 3)
    s = O.OracleSim(p, [dict(x=(6.2, 5.9, 6.4), R=3.1, Z=5, M=10)], rho0)
    assert np.array_equal(s.f.reshape(19, -1), np.tile(W19[:, None], (1, n ** 3)))
    r = s.rho.reshape(2, -1)
    r0 = rho0.reshape(2, -1)
    fl = s.flag == 1
    assert np.all(r[:, fl] == 0.0)
    expect = r0[:, ~fl] * ((1.0 - s.psi[~fl]) if pv else 1.0)
    assert np.array_equal(r[:, ~fl], expect)


# -- angular momentum ----------------------------------------------------------
def _arms(s):
    """Cell-centre arms about the box centre o = L/2 per axis, without wrapping
    (cell centres sit at i + 1/2, so every arm lies in (-L/2, L/2))."""
    zz, yy, xx = np.meshgrid(np.arange(s.nz), np.arange(s.ny), np.arange(s.nx), indexing="ij")
    return np.stack([xx.reshape(-1) + 0.5 - s.nx / 2, yy.reshape(-1) + 0.5 - s.ny / 2,
                     zz.reshape(-1) + 0.5 - s.nz / 2])


def _fluid_angular_momentum(s, arms):
    mom = C19.T.astype(np.float64) @ s.f.reshape(19, -1)
    fl = s.flag == 0
    return np.cross(arms[:, fl].T, mom[:, fl].T).sum(axis=0)


def _seam_term(s, f_prev, flag_prev):
    """Streaming carries a population from x to x + c_i, so its arm changes by
    c_i, parallel to its momentum, and its angular momentum is unchanged --
    except where x + c_i crosses the periodic seam: there the arm jumps by
    -+L_d e_d as well.  Sum of those jumps x momentum over the populations that
    cross (all of them land in fluid cells here: the spheres stay clear of the
    seam)."""
    dims = (s.nx, s.ny, s.nz)
    N = s.N
    idx3 = np.stack(np.unravel_index(np.arange(N), (s.nz, s.ny, s.nx))[::-1])  # x, y, z
    f = f_prev.reshape(19, N)
    W = np.zeros(3)
    for i in range(1, 19):
        c = C19[i]
        shift = np.zeros((3, N))
        for d in range(3):
            t = idx3[d] + c[d]
            shift[d] = np.where(t >= dims[d], -dims[d], np.where(t < 0, dims[d], 0))
        cross = np.any(shift != 0, axis=0) & (flag_prev == 0)
        if not cross.any():
            continue
        dest = [(idx3[d][cross] + c[d]) % dims[d] for d in range(3)]
        assert np.all(s.flag[dest[0] + s.nx * (dest[1] + s.ny * dest[2])] == 0)
        W += np.cross(shift[:, cross].T, c.astype(np.float64)).T @ f[i, cross]
    return W


def _angular_budget(s, steps):
    """Check, step by step, that the fluid's angular momentum about the box
    centre o changes by exactly what the coupling force density puts in, minus
    what the particles receive through bounce-back (Eq. force) and the Aidun
    destroy/create impulses, each about o:
      L(n) - L(n-1) = sum_x (x - o) x f_ext(x)
                      - sum_p [T_p + (x_p - o) x F_p]_(hyd + cov) + W_seam.
    The momentum exchanged on a link from fluid cell x_f into boundary cell
    r_b = x_f + c_i is parallel to c_i, so its arm may be taken at r_b (as the
    particle's torque does) or at x_f (where the fluid loses it): the budget
    closes exactly, and any error in the torque's arm, sign or cross product
    opens it."""
    arms = _arms(s)
    o = np.array([s.nx / 2, s.ny / 2, s.nz / 2])
    worst, scale = 0.0, 0.0
    for _ in range(steps):
        L0 = _fluid_angular_momentum(s, arms)
        f_prev, flag_prev = s.f.copy(), s.flag.copy()
        s.step()
        L1 = _fluid_angular_momentum(s, arms)
        fl = s.flag == 0
        ext = np.cross(arms[:, fl].T, s.fext.reshape(3, -1)[:, fl].T).sum(axis=0)
        Tp = np.zeros(3)
        for k, q in enumerate(s.particles()):
            F = s.last["F_hyd"][k] + s.last["F_cov"][k]
            T = s.last["T_hyd"][k] + s.last["T_cov"][k]
            Tp += T + np.cross(q["x"] - o, F)
            scale = max(scale, np.abs(s.last["T_hyd"][k]).max(), np.abs(s.last["T_cov"][k]).max())
        W = _seam_term(s, f_prev, flag_prev)
        res = (L1 - L0) - (ext - Tp + W)
        worst = max(worst, float(np.abs(res).max()))
        scale = max(scale, float(np.abs(L1 - L0).max()), float(np.abs(ext).max()))
    return worst, scale


def test_angular_momentum_budget_spinning_translating_sphere():
    """A prescribed sphere that spins and translates (cells covered and
    vacated every few steps), charged, in salt with a field: the torque of
    Eq. force and of the Aidun impulses against the fluid's angular momentum."""
    s = sim(24, [dict(x=(12.3, 11.8, 12.1), R=3.6, Z=20, M=200, v=(0.11, 0.07, -0.05),
                      w=(0.004, -0.003, 0.005), mode=1)], E=(0.01, 0.005, 0.0))
    events = 0
    worst, scale = 0.0, 0.0
    for _ in range(4):
        w_, sc = _angular_budget(s, 5)
        events += s.last["covered"] + s.last["vacated"]
        worst, scale = max(worst, w_), max(scale, sc)
    assert scale > 1e-2 and events > 20
    assert worst < 1e-12 * scale, (worst, scale)


def test_angular_momentum_budget_free_spheres():
    """Two free spheres (velocity Verlet) with forces on: charged, in salt and
    a field, one of them given a spin; the torque they receive turns them."""
    s = sim(24, [dict(x=(8.2, 12.3, 11.7), R=3.2, Z=25, M=150, v=(0.03, 0.0, 0.01), w=(0.0, 0.0, 0.01)),
                 dict(x=(16.4, 11.6, 12.4), R=3.0, Z=-15, M=120, v=(-0.02, 0.01, 0.0))],
            E=(0.02, 0.0, 0.01))
    worst, scale = _angular_budget(s, 20)
    assert scale > 1e-3
    assert worst < 1e-12 * scale, (worst, scale)
    assert all(np.abs(q["w"]).max() > 0 for q in s.particles())


def test_angular_momentum_budget_fails_for_a_planted_arm_error():
    """The budget is sensitive to the torque: adding a tenth of (x_p - o) x F
    to the reported torque (an arm about the wrong point) opens it by far more
    than the bar."""
    s = sim(24, [dict(x=(13.3, 11.8, 12.1), R=3.6, Z=20, M=200, v=(0.11, 0.07, -0.05),
                      w=(0.004, -0.003, 0.005), mode=1)], E=(0.01, 0.005, 0.0))
    arms = _arms(s)
    o = np.array([12.0, 12.0, 12.0])
    s.run(3)
    L0 = _fluid_angular_momentum(s, arms)
    f_prev, flag_prev = s.f.copy(), s.flag.copy()
    s.step()
    L1 = _fluid_angular_momentum(s, arms)
    fl = s.flag == 0
    ext = np.cross(arms[:, fl].T, s.fext.reshape(3, -1)[:, fl].T).sum(axis=0)
    q = s.particles()[0]
    F = s.last["F_hyd"][0] + s.last["F_cov"][0]
    T = s.last["T_hyd"][0] + s.last["T_cov"][0]
    W = _seam_term(s, f_prev, flag_prev)
    good = (L1 - L0) - (ext - (T + np.cross(q["x"] - o, F)) + W)
    bad = (L1 - L0) - (ext - (T + 1.1 * np.cross(q["x"] - o, F)) + W)
    assert np.abs(good).max() < 1e-12 * np.abs(T).max()
    assert np.abs(bad).max() > 1e-6 * np.abs(T).max()


def test_integrators_constant_torque():
    """The angular velocity under a constant torque grows by T/I per step with
    I = 2/5 M R^2 (both integrators), and the stored torque is the one given."""
    for integ in (0, 1):
        p = O.make_params(1000, 1000, 1000, 1 / 6, 1.0, 0.7, (0, 0, 0), [(0.1, 0)], integrator=integ)
        pt = O.make_particles([dict(x=(100.0, 200.0, 300.0), w=(0.001, 0.0, -0.002), R=2.0, Z=0, M=4.0)])
        T = np.array([0.003, -0.001, 0.002])
        pt[0].T[:] = T
        for _ in range(40):
            O.move(p, pt)
            O.finish(p, pt, np.zeros(3), T)
        I = 0.4 * 4.0 * 2.0 ** 2
        assert np.allclose(np.array(pt[0].w[:]), np.array([0.001, 0.0, -0.002]) + 40 * T / I, rtol=0, atol=1e-14)
        assert np.array_equal(np.array(pt[0].T[:]), T)
