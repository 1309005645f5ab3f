"""Plain FP64 CPU oracle for one time step of lattice electrokinetics with moving
charged particles (Kuron et al., "Moving Charged Particles in Lattice
Boltzmann-Based Electrokinetics").

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library: the per-cell phases live in ``ek_oracle.c`` (plain loops),
the Poisson solve below uses numpy's FFT as a library primitive, and the step
order is the one stated in ``OracleSim.step``.

Units are lattice units (a = tau = 1, fluid reference density 1); the potential
is e*Phi/kT.  Flat arrays use cell index x + nx*(y + ny*z).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libek_oracle.so")
MAX_SPECIES = 8

# Populations carry the standard D3Q19 weights; these are only used by the
# Python side to build initial states in tests (the C side has its own copy).
D3Q19_C = np.array(
    [[0, 0, 0],
     [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
     [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
     [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
     [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]], dtype=np.int64)
D3Q19_W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


class OrParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("nu", C.c_double), ("kT", C.c_double), ("lambda_B", C.c_double),
                ("E", C.c_double * 3), ("n_species", C.c_int),
                ("D", C.c_double * MAX_SPECIES), ("z", C.c_double * MAX_SPECIES),
                ("partial_volume", C.c_int), ("charge_mode", C.c_int),
                ("integrator", C.c_int)]


class OrParticle(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("v", C.c_double * 3), ("w", C.c_double * 3),
                ("R", C.c_double), ("Z", C.c_double), ("M", C.c_double),
                ("mode", C.c_int), ("pad", C.c_int),
                ("F", C.c_double * 3), ("T", C.c_double * 3)]


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, os.path.join(HERE, "ek_oracle.c"), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        dp, u8p, i32p, i64p = P(C.c_double), P(C.c_uint8), P(C.c_int32), P(C.c_int64)
        pp, ptp = P(OrParams), P(OrParticle)
        L.or_psi_count.argtypes = [C.c_double] * 4
        L.or_psi_count.restype = C.c_int
        L.or_geometry.argtypes = [pp, ptp, C.c_int, u8p, dp, u8p, i32p, dp, dp]
        L.or_init_fields.argtypes = [pp, u8p, dp, dp, dp]
        L.or_boundary_update.argtypes = [pp, ptp, C.c_int, u8p, i32p, u8p, i32p, dp, dp, dp, dp, i64p]
        L.or_charge.argtypes = [pp, dp, dp, dp]
        L.or_ek_update.argtypes = [pp, dp, dp, dp, dp, u8p, dp, dp]
        L.or_lb_update.argtypes = [pp, ptp, dp, dp, u8p, i32p, dp, dp]
        L.or_hydro_force.argtypes = [pp, ptp, C.c_int, dp, u8p, i32p, dp, dp]
        L.or_el_force.argtypes = [pp, ptp, C.c_int, dp, u8p, i32p, dp, dp]
        L.or_move.argtypes = [pp, ptp, C.c_int]
        L.or_finish.argtypes = [pp, ptp, C.c_int, dp, dp]
        for fn in ("or_geometry", "or_init_fields", "or_boundary_update", "or_charge",
                   "or_ek_update", "or_lb_update", "or_hydro_force", "or_el_force",
                   "or_move", "or_finish"):
            getattr(L, fn).restype = None
        _LIB = L
    return _LIB


def _p(a, ctype):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(ctype))


def d(a):
    assert a is None or a.dtype == np.float64
    return _p(a, C.c_double)


def u8(a):
    assert a is None or a.dtype == np.uint8
    return _p(a, C.c_uint8)


def i32(a):
    assert a is None or a.dtype == np.int32
    return _p(a, C.c_int32)


def make_params(nx, ny, nz, nu, kT, lambda_B, E, species, partial_volume=True,
                charge_mode=0, integrator=0) -> OrParams:
    """species: list of (D, z) in lattice units."""
    p = OrParams()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.nu, p.kT, p.lambda_B = nu, kT, lambda_B
    for i in range(3):
        p.E[i] = E[i]
    p.n_species = len(species)
    assert 1 <= len(species) <= MAX_SPECIES
    for k, (D, z) in enumerate(species):
        p.D[k], p.z[k] = D, z
    p.partial_volume = int(bool(partial_volume))
    p.charge_mode = int(charge_mode)
    p.integrator = int(integrator)
    return p


def make_particles(specs) -> C.Array:
    """specs: list of dicts with x, R, Z, M and optional v, w, mode, and the
    force F and torque T of the last completed step (0 by default)."""
    arr = (OrParticle * max(1, len(specs)))()
    for k, s in enumerate(specs):
        q = arr[k]
        for dd in range(3):
            q.x[dd] = s["x"][dd]
            q.v[dd] = s.get("v", (0, 0, 0))[dd]
            q.w[dd] = s.get("w", (0, 0, 0))[dd]
            q.F[dd] = s.get("F", (0, 0, 0))[dd]
            q.T[dd] = s.get("T", (0, 0, 0))[dd]
        q.R, q.Z, q.M = s["R"], s["Z"], s["M"]
        q.mode = int(s.get("mode", 0))
    return arr


def poisson(q: np.ndarray, nx: int, ny: int, nz: int, lambda_B: float) -> np.ndarray:
    """Periodic Poisson solve (Eq. poisson) on the lattice: the 7-point discrete
    Laplacian of phi equals -4 pi lambda_B (q - mean q).  In Fourier space
    phi_k = 4 pi lambda_B q_k / K^2, K^2 = sum_d (2 - 2 cos(2 pi k_d / n_d)), and
    the k = 0 mode is zero (uniform neutralising background).  Reading: the
    paper names an FFT solver but not its discrete Green's function."""
    q3 = q.reshape(nz, ny, nx).astype(np.float64)
    q3 = q3 - q3.mean()
    qh = np.fft.rfftn(q3)
    kz = 2 * np.pi * np.arange(nz) / nz
    ky = 2 * np.pi * np.arange(ny) / ny
    kx = 2 * np.pi * np.arange(nx // 2 + 1) / nx
    K2 = ((2 - 2 * np.cos(kz))[:, None, None] + (2 - 2 * np.cos(ky))[None, :, None]
          + (2 - 2 * np.cos(kx))[None, None, :])
    K2[0, 0, 0] = 1.0
    G = 4 * np.pi * lambda_B / K2
    G[0, 0, 0] = 0.0
    phi = np.fft.irfftn(qh * G, s=(nz, ny, nx), axes=(0, 1, 2))
    return np.ascontiguousarray(phi.reshape(-1))


def face_permittivity(eps3: np.ndarray, axis: int) -> np.ndarray:
    """Permittivity on the face between each cell and its + neighbour along
    `axis`: the harmonic mean 2 e_a e_b / (e_a + e_b) of the two cells.
    Reading: the paper names iterative solvers for an inhomogeneous dielectric
    without a discretisation; the harmonic mean is the face value for which a
    layered dielectric (charge sheets between slabs of different permittivity)
    has the exact series-capacitor solution."""
    e2 = np.roll(eps3, -1, axis=axis)
    return 2.0 * eps3 * e2 / (eps3 + e2)


def poisson_dielectric(q: np.ndarray, eps: np.ndarray, nx: int, ny: int, nz: int,
                       lambda_B: float) -> np.ndarray:
    """Periodic Poisson solve with a relative permittivity eps (N values > 0)
    per cell (Sec. III.C, non-FFT solvers for an inhomogeneous dielectric):
      sum over the 6 faces of e_f (phi_c - phi_n) = 4 pi lambda_B (q_c - mean q),
    i.e. -div(eps grad phi) = 4 pi lambda_B (q - mean q) with the 7-point
    stencil; for eps = 1 this is the FFT solve above.  The periodic operator
    is singular (constants): phi is fixed to 0 in cell 0, the system solved by
    a sparse direct solver (a library primitive), and the mean of phi then
    removed (the solution with zero mean, like the FFT one's)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    N = nx * ny * nz
    e3 = np.ascontiguousarray(eps, dtype=np.float64).reshape(nz, ny, nx)
    idx = np.arange(N).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    diag = np.zeros((nz, ny, nx))
    for ax3 in (2, 1, 0):  # x, y, z faces (array axes are z, y, x)
        ef = face_permittivity(e3, ax3)
        nb = np.roll(idx, -1, axis=ax3)
        # face between c and its + neighbour n couples both ways
        rows += [idx.ravel(), nb.ravel()]
        cols += [nb.ravel(), idx.ravel()]
        vals += [-ef.ravel(), -ef.ravel()]
        diag += ef + np.roll(ef, 1, axis=ax3)
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    L = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    b = 4.0 * np.pi * lambda_B * (q - q.mean())
    phi = np.zeros(N)
    phi[1:] = spl.spsolve(L[1:, 1:].tocsc(), b[1:])
    return phi - phi.mean()


class OracleSim:
    """One simulation, stepped in the order (particle move; geometry and
    moving-boundary update; charge and Poisson; EK fluxes and coupling force;
    LB stream/collide with the momentum-exchange force taken from the
    populations being streamed; electrostatic force; particle update).
    Reading: the paper does not state the order of these parts within a step;
    the EK advection uses the fluid velocity of the previous LB step.
    Parity unpinned: no closed form fixes this order (the momentum budget pins
    how the parts combine, not their order)."""

    def __init__(self, params: OrParams, particles: list, rho_init: np.ndarray,
                 static_mask: np.ndarray | None = None,
                 static_charge: np.ndarray | None = None,
                 f_init: np.ndarray | None = None,
                 permittivity: np.ndarray | None = None):
        self.L = lib()
        self.eps = None if permittivity is None else np.asarray(permittivity, dtype=np.float64).reshape(-1)
        self.p = params
        self.nx, self.ny, self.nz = params.nx, params.ny, params.nz
        self.N = N = self.nx * self.ny * self.nz
        self.ns = params.n_species
        self.np = len(particles)
        self.pt = make_particles(particles)
        self.static_mask = None if static_mask is None else np.ascontiguousarray(static_mask, dtype=np.uint8).reshape(-1)
        self.static_charge = None if static_charge is None else np.ascontiguousarray(static_charge, dtype=np.float64).reshape(-1)
        self.flag = np.zeros(N, np.uint8)
        self.owner = np.full(N, -1, np.int32)
        self.psi = np.zeros(N)
        self.rhob = np.zeros(N)
        self.geometry(self.flag, self.owner, self.psi, self.rhob)
        self.f = np.zeros(19 * N)
        self.rho = np.ascontiguousarray(rho_init, dtype=np.float64).reshape(-1).copy()
        assert self.rho.size == self.ns * N
        self.L.or_init_fields(C.byref(self.p), u8(self.flag), d(self.psi), d(self.f), d(self.rho))
        if f_init is not None:
            self.f[:] = np.asarray(f_init, dtype=np.float64).reshape(-1)
        self.u = np.zeros(3 * N)
        self.fext = np.zeros(3 * N)
        self.phi = np.zeros(N)
        self.step_count = 0
        self.last = {}

    @classmethod
    def from_state(cls, params: OrParams, particles: list, f: np.ndarray, rho: np.ndarray, u: np.ndarray,
                   flag: np.ndarray, owner: np.ndarray) -> "OracleSim":
        """A simulation resumed at a step boundary from a given state: the
        populations, solute densities, fluid velocity of the last LB update,
        boundary flags and owners (which the next step's moving-boundary
        update compares against), and the particles (with v, w and the F, T
        of the last step).  Partial volumes, particle charge, potential and
        coupling force are recomputed by the next step."""
        self = cls.__new__(cls)
        self.L = lib()
        self.eps = None
        self.p = params
        self.nx, self.ny, self.nz = params.nx, params.ny, params.nz
        self.N = N = self.nx * self.ny * self.nz
        self.ns = params.n_species
        self.np = len(particles)
        self.pt = make_particles(particles)
        self.static_mask = None
        self.static_charge = None
        self.flag = np.ascontiguousarray(flag, dtype=np.uint8).reshape(-1).copy()
        self.owner = np.ascontiguousarray(owner, dtype=np.int32).reshape(-1).copy()
        self.psi = np.zeros(N)
        self.rhob = np.zeros(N)
        self.f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1).copy()
        self.rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1).copy()
        self.u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1).copy()
        assert self.f.size == 19 * N and self.rho.size == self.ns * N and self.u.size == 3 * N
        self.fext = np.zeros(3 * N)
        self.phi = np.zeros(N)
        self.step_count = 0
        self.last = {}
        return self

    # -- phases --------------------------------------------------------------
    def geometry(self, flag, owner, psi, rhob):
        self.L.or_geometry(C.byref(self.p), self.pt, self.np, u8(self.static_mask),
                           d(self.static_charge), u8(flag), i32(owner), d(psi), d(rhob))

    def particles(self) -> list:
        """Per particle: centre x, velocity v, angular velocity w, and the total
        force F and torque T of the last step with their parts (momentum
        exchange F_hyd/T_hyd, electrostatic F_el/T_el, fluid destroyed/created
        F_cov/T_cov; zero before the first step)."""
        out = []
        for k in range(self.np):
            q = self.pt[k]
            d = {"x": np.array(q.x[:]), "v": np.array(q.v[:]), "w": np.array(q.w[:]),
                 "F": np.array(q.F[:]), "T": np.array(q.T[:])}
            for key in ("F_hyd", "T_hyd", "F_el", "T_el", "F_cov", "T_cov"):
                d[key] = np.array(self.last[key][k]) if key in self.last else np.zeros(3)
            out.append(d)
        return out

    def step(self):
        L, p, N, npart = self.L, C.byref(self.p), self.N, self.np
        L.or_move(p, self.pt, npart)
        flag_old, owner_old = self.flag.copy(), self.owner.copy()
        L_flag = np.zeros(N, np.uint8)
        L_owner = np.full(N, -1, np.int32)
        self.geometry(L_flag, L_owner, self.psi, self.rhob)
        Fcov = np.zeros(3 * max(1, npart))
        Tcov = np.zeros(3 * max(1, npart))
        counts = np.zeros(3, np.int64)
        L.or_boundary_update(p, self.pt, npart, u8(flag_old), i32(owner_old), u8(L_flag),
                             i32(L_owner), d(self.f), d(self.rho), d(Fcov), d(Tcov),
                             counts.ctypes.data_as(C.POINTER(C.c_int64)))
        self.flag, self.owner = L_flag, L_owner
        q = np.zeros(N)
        L.or_charge(p, d(self.rho), d(self.rhob), d(q))
        if self.eps is None:
            self.phi = poisson(q, self.nx, self.ny, self.nz, self.p.lambda_B)
        else:
            self.phi = poisson_dielectric(q, self.eps, self.nx, self.ny, self.nz, self.p.lambda_B)
        rho_new = np.zeros_like(self.rho)
        L.or_ek_update(p, d(self.rho), d(rho_new), d(self.phi), d(self.psi), u8(self.flag),
                       d(self.u), d(self.fext))
        self.rho = rho_new
        Fh = np.zeros(3 * max(1, npart))
        Th = np.zeros(3 * max(1, npart))
        L.or_hydro_force(p, self.pt, npart, d(self.f), u8(self.flag), i32(self.owner), d(Fh), d(Th))
        f_new = np.zeros_like(self.f)
        L.or_lb_update(p, self.pt, d(self.f), d(f_new), u8(self.flag), i32(self.owner),
                       d(self.fext), d(self.u))
        self.f = f_new
        Fe = np.zeros(3 * max(1, npart))
        Te = np.zeros(3 * max(1, npart))
        L.or_el_force(p, self.pt, npart, d(self.phi), u8(self.flag), i32(self.owner), d(Fe), d(Te))
        Fn = Fh + Fe + Fcov
        Tn = Th + Te + Tcov
        L.or_finish(p, self.pt, npart, d(Fn), d(Tn))
        self.step_count += 1
        self.last = {"F_hyd": Fh[:3 * npart].reshape(-1, 3), "T_hyd": Th[:3 * npart].reshape(-1, 3),
                     "F_el": Fe[:3 * npart].reshape(-1, 3), "T_el": Te[:3 * npart].reshape(-1, 3),
                     "F_cov": Fcov[:3 * npart].reshape(-1, 3), "T_cov": Tcov[:3 * npart].reshape(-1, 3),
                     "covered": int(counts[0]), "vacated": int(counts[1]), "pooled": int(counts[2]),
                     "flag_old": flag_old}

    def run(self, n: int):
        for _ in range(n):
            self.step()

    # -- observables ---------------------------------------------------------
    def density(self) -> np.ndarray:
        return self.rho.reshape(self.ns, self.N)

    def fluid_density(self) -> np.ndarray:
        return self.f.reshape(19, self.N).sum(axis=0)

    def fluid_momentum(self) -> np.ndarray:
        """Total momentum of the stored (post-collision) populations of fluid cells."""
        f = self.f.reshape(19, self.N)[:, self.flag == 0]
        return (D3Q19_C.T.astype(np.float64) @ f).sum(axis=1)

    def species_totals(self) -> np.ndarray:
        return self.density().sum(axis=1)


# -- single-phase entry points (arrays in, arrays out) -----------------------
def ek_update(p: OrParams, rho, phi, psi, flag, u):
    """One EK solute update with a given potential; returns (rho_new, fext)."""
    N = p.nx * p.ny * p.nz
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
    out = np.zeros_like(rho)
    fext = np.zeros(3 * N)
    lib().or_ek_update(C.byref(p), d(rho), d(out), d(np.ascontiguousarray(phi, np.float64).reshape(-1)),
                       d(np.ascontiguousarray(psi, np.float64).reshape(-1)),
                       u8(np.ascontiguousarray(flag, np.uint8).reshape(-1)),
                       d(np.ascontiguousarray(u, np.float64).reshape(-1)), d(fext))
    return out, fext


def lb_update(p: OrParams, f, flag, owner, fext, particles=None):
    """One LB stream/collide; returns (f_new, u)."""
    N = p.nx * p.ny * p.nz
    pt = make_particles(particles or [])
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
    out = np.zeros_like(f)
    u = np.zeros(3 * N)
    lib().or_lb_update(C.byref(p), pt, d(f), d(out), u8(np.ascontiguousarray(flag, np.uint8).reshape(-1)),
                       i32(np.ascontiguousarray(owner, np.int32).reshape(-1)),
                       d(np.ascontiguousarray(fext, np.float64).reshape(-1)), d(u))
    return out, u


def geometry(p: OrParams, particles, static_mask=None, static_charge=None):
    """Returns (flag, owner, psi, rhob) for the given sphere specs."""
    N = p.nx * p.ny * p.nz
    pt = make_particles(particles)
    flag = np.zeros(N, np.uint8)
    owner = np.full(N, -1, np.int32)
    psi = np.zeros(N)
    rhob = np.zeros(N)
    sm = None if static_mask is None else np.ascontiguousarray(static_mask, np.uint8).reshape(-1)
    sc = None if static_charge is None else np.ascontiguousarray(static_charge, np.float64).reshape(-1)
    lib().or_geometry(C.byref(p), pt, len(particles), u8(sm), d(sc), u8(flag), i32(owner), d(psi), d(rhob))
    return flag, owner, psi, rhob


def boundary_update(p: OrParams, particles, flag_old, owner_old, flag_new, owner_new, f, rho):
    """Moving-boundary update on copies of f and rho; returns
    (f, rho, Fcov, Tcov, counts)."""
    npart = len(particles)
    pt = make_particles(particles)
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1).copy()
    rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1).copy()
    Fc = np.zeros(3 * max(1, npart))
    Tc = np.zeros(3 * max(1, npart))
    counts = np.zeros(3, np.int64)
    lib().or_boundary_update(C.byref(p), pt, npart,
                             u8(np.ascontiguousarray(flag_old, np.uint8).reshape(-1)),
                             i32(np.ascontiguousarray(owner_old, np.int32).reshape(-1)),
                             u8(np.ascontiguousarray(flag_new, np.uint8).reshape(-1)),
                             i32(np.ascontiguousarray(owner_new, np.int32).reshape(-1)),
                             d(f), d(rho), d(Fc), d(Tc), counts.ctypes.data_as(C.POINTER(C.c_int64)))
    return f, rho, Fc[:3 * npart].reshape(-1, 3), Tc[:3 * npart].reshape(-1, 3), counts


def move(p: OrParams, pt):
    lib().or_move(C.byref(p), pt, len(pt))


def finish(p: OrParams, pt, F, T):
    lib().or_finish(C.byref(p), pt, len(pt), d(np.ascontiguousarray(F, np.float64).reshape(-1)),
                    d(np.ascontiguousarray(T, np.float64).reshape(-1)))


def equilibrium(rho, u):
    """Second-order incompressible equilibrium, populations (19, N), for building
    test states only."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64).reshape(3, -1)
    cu = D3Q19_C.astype(np.float64) @ u
    usq = (u * u).sum(axis=0)
    return D3Q19_W[:, None] * (rho[None, :] + 3 * cu + 4.5 * cu * cu - 1.5 * usq[None, :])
