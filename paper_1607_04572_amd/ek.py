"""Python binding of the C ABI in include/ek.h (argument marshalling only).

The functions below carry the names of the C entry points and call them through
ctypes; every step of the method runs in the HIP kernels of libek_hip.so.
PyTorch is used only to provide device memory (the arena) and a stream.
Loading fails loudly when the library has not been built: there is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libek_hip.so")
MAX_SPECIES = 4

EK_OK = 0
ERRORS = {-1: "EK_ERR_INVALID_ARG", -2: "EK_ERR_UNSUPPORTED_SIZE", -3: "EK_ERR_UNSTABLE",
          -4: "EK_ERR_OVERLAP", -5: "EK_ERR_OOM", -6: "EK_ERR_NO_SPACE", -7: "EK_ERR_NONFINITE",
          -8: "EK_ERR_DEVICE", -9: "EK_ERR_STATE"}
EK_FP64_PLAIN, EK_FP32_DEV = 0, 1
EK_SCHEME_PARTIAL_VOLUME, EK_SCHEME_SIMPLE = 0, 1
EK_CHARGE_PSI, EK_CHARGE_UNIFORM = 0, 1
EK_VELOCITY_VERLET, EK_SYMPLECTIC_EULER = 0, 1
EK_FREE, EK_PRESCRIBED, EK_FIXED = 0, 1, 2
FIELDS = {"density": 0, "phi": 1, "velocity": 2, "fluid_density": 3, "force": 4, "psi": 5,
          "flag": 6, "owner": 7, "populations": 8, "particle_charge": 9}


class EkError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)}")
        self.code = code


class ek_species(C.Structure):
    _fields_ = [("D", C.c_double), ("valency", C.c_int), ("mean_density", C.c_double)]


class ek_params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("agrid", C.c_double), ("tau", C.c_double), ("kT", C.c_double),
                ("fluid_density", C.c_double), ("viscosity", C.c_double),
                ("n_species", C.c_int), ("species", ek_species * MAX_SPECIES),
                ("bjerrum_length", C.c_double), ("E_ext", C.c_double * 3),
                ("precision", C.c_int), ("scheme", C.c_int), ("charge_mode", C.c_int),
                ("integrator", C.c_int), ("max_particles", C.c_int),
                ("stream", C.c_void_p), ("arena", C.c_void_p), ("arena_bytes", C.c_size_t)]


class ek_particle(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("v", C.c_double * 3), ("omega", C.c_double * 3),
                ("F", C.c_double * 3), ("T", C.c_double * 3), ("F_hyd", C.c_double * 3),
                ("F_el", C.c_double * 3), ("F_cov", C.c_double * 3),
                ("radius", C.c_double), ("charge", C.c_double), ("mass", C.c_double),
                ("mode", C.c_int), ("n_boundary", C.c_int)]


class ek_sphere(C.Structure):
    _fields_ = [("x", C.c_double * 3), ("v", C.c_double * 3), ("radius", C.c_double), ("charge", C.c_double),
                ("mass", C.c_double), ("mode", C.c_int)]


class ek_diag(C.Structure):
    _fields_ = [("step", C.c_longlong), ("species_total", C.c_double * MAX_SPECIES),
                ("solute_charge", C.c_double), ("particle_charge", C.c_double),
                ("fluid_mass", C.c_double), ("fluid_momentum", C.c_double * 3),
                ("covered", C.c_longlong), ("vacated", C.c_longlong), ("pooled", C.c_longlong),
                ("boundary_cells", C.c_longlong), ("max_velocity", C.c_double)]


# ABI symbols declared in include/ek.h
SYMBOLS = ["ek_query_footprint", "ek_create", "ek_add_sphere", "ek_set_static_boundary", "ek_set_fields",
           "ek_seed_density", "ek_prepare", "ek_step", "ek_step_noalloc", "ek_get_fields", "ek_get_particles", "ek_get_diagnostics",
           "ek_get_state", "ek_set_state", "ek_set_permittivity", "ek_get_poisson_stats", "ek_profile_stages",
           "ek_copy_probe", "ek_synchronize",
           "ek_destroy", "ek_strerror"]
STAGES = ["move", "geometry", "boundary", "poisson", "forces", "ek", "lb", "finish"]
BATCH_SYMBOLS = ["ek_batch_create", "ek_batch_admit", "ek_batch_admit_seeded", "ek_batch_step", "ek_batch_poll",
                 "ek_batch_wait", "ek_batch_collect", "ek_batch_get_fields", "ek_batch_active", "ek_batch_destroy"]

_LIB = None


def lib():
    """Load libek_hip.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no fallback implementation")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.ek_query_footprint.argtypes = [P(ek_params), P(C.c_size_t)]
        L.ek_create.argtypes = [P(ek_params), P(vp)]
        L.ek_add_sphere.argtypes = [vp, P(C.c_double), C.c_double, C.c_double, C.c_double,
                                    P(C.c_double), C.c_int, P(C.c_int)]
        L.ek_set_static_boundary.argtypes = [vp, P(C.c_uint8), P(C.c_double)]
        L.ek_set_fields.argtypes = [vp, C.c_int, vp, C.c_size_t]
        L.ek_seed_density.argtypes = [vp, C.c_uint64, C.c_double]
        L.ek_prepare.argtypes = [vp]
        L.ek_step.argtypes = [vp, C.c_int]
        L.ek_step_noalloc.argtypes = [vp, C.c_int]
        L.ek_get_fields.argtypes = [vp, C.c_int, vp, C.c_size_t]
        L.ek_get_particles.argtypes = [vp, P(ek_particle), C.c_int]
        L.ek_get_diagnostics.argtypes = [vp, P(ek_diag)]
        L.ek_get_state.argtypes = [vp, vp, P(C.c_size_t)]
        L.ek_set_state.argtypes = [vp, vp, C.c_size_t]
        L.ek_set_permittivity.argtypes = [vp, P(C.c_double), C.c_double, C.c_int]
        L.ek_get_poisson_stats.argtypes = [vp, P(C.c_int), P(C.c_double)]
        L.ek_profile_stages.argtypes = [vp, C.c_int, P(C.c_double), C.c_int]
        L.ek_copy_probe.argtypes = [vp, vp, C.c_size_t, vp]
        L.ek_synchronize.argtypes = [vp]
        L.ek_destroy.argtypes = [vp]
        L.ek_batch_create.argtypes = [C.c_size_t, C.c_int, vp, vp, P(vp)]
        L.ek_batch_admit.argtypes = [vp, P(ek_params), P(ek_sphere), C.c_int, P(C.c_double), C.c_longlong,
                                     P(C.c_int)]
        L.ek_batch_admit_seeded.argtypes = [vp, P(ek_params), P(ek_sphere), C.c_int, C.c_uint64, C.c_double,
                                            C.c_longlong, P(C.c_int)]
        L.ek_batch_step.argtypes = [vp, C.c_int]
        L.ek_batch_poll.argtypes = [vp, P(C.c_int), C.c_int, P(C.c_int)]
        L.ek_batch_wait.argtypes = [vp]
        L.ek_batch_collect.argtypes = [vp, C.c_int, P(ek_particle), C.c_int, P(ek_diag)]
        L.ek_batch_get_fields.argtypes = [vp, C.c_int, C.c_int, vp, C.c_size_t]
        L.ek_batch_active.argtypes = [vp, P(C.c_int), P(C.c_longlong)]
        L.ek_batch_destroy.argtypes = [vp]
        for sname in BATCH_SYMBOLS:
            getattr(L, sname).restype = C.c_int
        L.ek_strerror.argtypes = [C.c_int]
        L.ek_strerror.restype = C.c_char_p
        for s in SYMBOLS:
            if s != "ek_strerror":
                getattr(L, s).restype = C.c_int
        _LIB = L
    return _LIB


def _check(r: int, where: str):
    if r != EK_OK:
        raise EkError(r, where)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# -- the C entry points -------------------------------------------------------
def ek_query_footprint(p: ek_params) -> int:
    n = C.c_size_t(0)
    _check(lib().ek_query_footprint(C.byref(p), C.byref(n)), "ek_query_footprint")
    return int(n.value)


def ek_create(p: ek_params) -> C.c_void_p:
    h = C.c_void_p()
    _check(lib().ek_create(C.byref(p), C.byref(h)), "ek_create")
    return h


def ek_add_sphere(ctx, pos, radius, charge, mass, v0=(0.0, 0.0, 0.0), mode=EK_FREE) -> int:
    i = C.c_int(-1)
    pa = (C.c_double * 3)(*pos)
    va = (C.c_double * 3)(*v0)
    _check(lib().ek_add_sphere(ctx, pa, float(radius), float(charge), float(mass), va, int(mode), C.byref(i)),
           "ek_add_sphere")
    return i.value


def ek_set_static_boundary(ctx, mask: np.ndarray, charge: np.ndarray | None = None):
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    q = None if charge is None else np.ascontiguousarray(charge, dtype=np.float64).reshape(-1)
    _check(lib().ek_set_static_boundary(ctx, m.ctypes.data_as(C.POINTER(C.c_uint8)),
                                        None if q is None else _dptr(q)), "ek_set_static_boundary")


def ek_set_fields(ctx, field, values: np.ndarray):
    v = np.ascontiguousarray(values, dtype=np.float64).reshape(-1)
    _check(lib().ek_set_fields(ctx, FIELDS.get(field, field), v.ctypes.data, v.nbytes), "ek_set_fields")


def ek_seed_density(ctx, seed: int, noise: float):
    _check(lib().ek_seed_density(ctx, int(seed), float(noise)), "ek_seed_density")


def ek_prepare(ctx):
    _check(lib().ek_prepare(ctx), "ek_prepare")


def ek_step(ctx, n: int):
    _check(lib().ek_step(ctx, int(n)), "ek_step")


def ek_step_noalloc(ctx, n: int):
    _check(lib().ek_step_noalloc(ctx, int(n)), "ek_step_noalloc")


def ek_get_fields(ctx, field, n_cells: int, n_species: int = 1) -> np.ndarray:
    f = FIELDS.get(field, field)
    if f == FIELDS["flag"]:
        out = np.empty(n_cells, np.uint8)
    elif f == FIELDS["owner"]:
        out = np.empty(n_cells, np.int32)
    else:
        mult = {0: n_species, 2: 3, 4: 3, 8: 19}.get(f, 1)
        out = np.empty(mult * n_cells, np.float64)
    _check(lib().ek_get_fields(ctx, f, out.ctypes.data, out.nbytes), "ek_get_fields")
    return out


def ek_get_particles(ctx, n: int) -> list:
    arr = (ek_particle * max(1, n))()
    _check(lib().ek_get_particles(ctx, arr, int(n)), "ek_get_particles")
    out = []
    for k in range(n):
        q = arr[k]
        out.append({f: (np.array(getattr(q, f)[:]) if isinstance(getattr(q, f), C.Array) else getattr(q, f))
                    for f, _ in ek_particle._fields_})
    return out


def ek_get_diagnostics(ctx) -> dict:
    d = ek_diag()
    _check(lib().ek_get_diagnostics(ctx, C.byref(d)), "ek_get_diagnostics")
    return {f: (np.array(getattr(d, f)[:]) if isinstance(getattr(d, f), C.Array) else getattr(d, f))
            for f, _ in ek_diag._fields_}


def ek_get_state(ctx) -> bytes:
    n = C.c_size_t(0)
    _check(lib().ek_get_state(ctx, None, C.byref(n)), "ek_get_state")
    buf = C.create_string_buffer(n.value)
    _check(lib().ek_get_state(ctx, C.cast(buf, C.c_void_p), C.byref(n)), "ek_get_state")
    return buf.raw[:n.value]


def ek_set_state(ctx, image: bytes):
    buf = C.create_string_buffer(image, len(image))
    _check(lib().ek_set_state(ctx, C.cast(buf, C.c_void_p), len(image)), "ek_set_state")


def ek_set_permittivity(ctx, eps_r, tol: float = 1e-12, max_iter: int = 10000):
    e = None if eps_r is None else np.ascontiguousarray(eps_r, dtype=np.float64).reshape(-1)
    _check(lib().ek_set_permittivity(ctx, None if e is None else _dptr(e), float(tol), int(max_iter)),
           "ek_set_permittivity")


def ek_get_poisson_stats(ctx) -> tuple:
    it = C.c_int(0)
    res = C.c_double(0.0)
    _check(lib().ek_get_poisson_stats(ctx, C.byref(it), C.byref(res)), "ek_get_poisson_stats")
    return it.value, res.value


def ek_profile_stages(ctx, n: int) -> dict:
    out = (C.c_double * len(STAGES))()
    _check(lib().ek_profile_stages(ctx, int(n), out, len(STAGES)), "ek_profile_stages")
    return {k: float(out[i]) for i, k in enumerate(STAGES)}


def ek_copy_probe(dst_ptr: int, src_ptr: int, nbytes: int, stream_ptr: int = 0):
    _check(lib().ek_copy_probe(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), nbytes, C.c_void_p(stream_ptr)),
           "ek_copy_probe")


def ek_synchronize(ctx):
    _check(lib().ek_synchronize(ctx), "ek_synchronize")


def ek_destroy(ctx):
    _check(lib().ek_destroy(ctx), "ek_destroy")


# -- serving form ----------------------------------------------------------------
def _particles_to_dicts(arr, n):
    return [{f: (np.array(getattr(arr[k], f)[:]) if isinstance(getattr(arr[k], f), C.Array) else getattr(arr[k], f))
             for f, _ in ek_particle._fields_} for k in range(n)]


def ek_batch_create(arena_bytes: int, n_species: int, stream: int = 0, arena: int = 0):
    h = C.c_void_p()
    _check(lib().ek_batch_create(arena_bytes, n_species, C.c_void_p(stream or None), C.c_void_p(arena or None),
                                 C.byref(h)), "ek_batch_create")
    return h


def _sphere_array(spheres: list):
    arr = (ek_sphere * max(1, len(spheres)))()
    for k, sp in enumerate(spheres):
        for d in range(3):
            arr[k].x[d] = sp.x[d]
            arr[k].v[d] = sp.v[d]
        arr[k].radius, arr[k].charge, arr[k].mass, arr[k].mode = sp.R, sp.Z, sp.M, sp.mode
    return arr


def ek_batch_admit(b, p: ek_params, spheres: list, initial_density, n_steps: int) -> int:
    arr = _sphere_array(spheres)
    rho = None
    if initial_density is not None:
        rho = np.ascontiguousarray(initial_density, dtype=np.float64).reshape(-1)
    slot = C.c_int(-1)
    _check(lib().ek_batch_admit(b, C.byref(p), arr, len(spheres), None if rho is None else _dptr(rho),
                                int(n_steps), C.byref(slot)), "ek_batch_admit")
    return slot.value


def ek_batch_admit_seeded(b, p: ek_params, spheres: list, seed: int, noise: float, n_steps: int) -> int:
    arr = _sphere_array(spheres)
    slot = C.c_int(-1)
    _check(lib().ek_batch_admit_seeded(b, C.byref(p), arr, len(spheres), int(seed), float(noise), int(n_steps),
                                       C.byref(slot)), "ek_batch_admit_seeded")
    return slot.value


def ek_batch_step(b, k: int):
    _check(lib().ek_batch_step(b, int(k)), "ek_batch_step")


def ek_batch_wait(b):
    _check(lib().ek_batch_wait(b), "ek_batch_wait")


def ek_batch_poll(b, cap: int = 64) -> list:
    out = (C.c_int * cap)()
    n = C.c_int(0)
    _check(lib().ek_batch_poll(b, out, cap, C.byref(n)), "ek_batch_poll")
    return [out[i] for i in range(n.value)]


def ek_batch_collect(b, slot: int, n: int):
    arr = (ek_particle * max(1, n))()
    d = ek_diag()
    _check(lib().ek_batch_collect(b, int(slot), arr, int(n), C.byref(d)), "ek_batch_collect")
    diag = {f: (np.array(getattr(d, f)[:]) if isinstance(getattr(d, f), C.Array) else getattr(d, f))
            for f, _ in ek_diag._fields_}
    return _particles_to_dicts(arr, n), diag


def ek_batch_get_fields(b, slot: int, field, n_cells: int, n_species: int = 1) -> np.ndarray:
    f = FIELDS.get(field, field)
    if f == FIELDS["flag"]:
        out = np.empty(n_cells, np.uint8)
    elif f == FIELDS["owner"]:
        out = np.empty(n_cells, np.int32)
    else:
        mult = {0: n_species, 2: 3, 4: 3, 8: 19}.get(f, 1)
        out = np.empty(mult * n_cells, np.float64)
    _check(lib().ek_batch_get_fields(b, int(slot), f, out.ctypes.data, out.nbytes), "ek_batch_get_fields")
    return out


def ek_batch_active(b):
    n = C.c_int(0)
    cells = C.c_longlong(0)
    _check(lib().ek_batch_active(b, C.byref(n), C.byref(cells)), "ek_batch_active")
    return n.value, cells.value


def ek_batch_destroy(b):
    _check(lib().ek_batch_destroy(b), "ek_batch_destroy")


class EkBatch:
    """A batch of FP32 simulations in one arena on cuda:0 (arena and stream
    from PyTorch)."""

    def __init__(self, arena_bytes: int, n_species: int = 2, use_torch: bool = True):
        self._arena = None
        self._stream = None
        stream = arena = 0
        if use_torch:
            import torch
            dev = torch.device("cuda", 0)
            self._stream = torch.cuda.Stream(device=dev)
            self._arena = torch.empty(arena_bytes, dtype=torch.uint8, device=dev)
            torch.cuda.synchronize(dev)
            stream, arena = self._stream.cuda_stream, self._arena.data_ptr()
        self.ns = n_species
        self.h = ek_batch_create(arena_bytes, n_species, stream, arena)
        self.meta = {}

    def admit(self, w, initial_density=None, n_steps=None, seeded: bool = False) -> int:
        """seeded: the workload's seeded initial densities built on the device
        (the values of workloads.initial_densities(w), no host array)."""
        p = params_from_workload(w, max_particles=max(1, len(w.spheres)))
        steps = w.steps if n_steps is None else n_steps
        if seeded:
            slot = ek_batch_admit_seeded(self.h, p, w.spheres, w.seed, w.noise, steps)
        else:
            slot = ek_batch_admit(self.h, p, w.spheres, initial_density, steps)
        self.meta[slot] = w
        return slot

    def step(self, k: int):
        ek_batch_step(self.h, k)

    def poll(self, wait: bool = False) -> list:
        """Slots done as of the chunks that have finished (wait: of every
        queued chunk)."""
        if wait:
            ek_batch_wait(self.h)
        return ek_batch_poll(self.h)

    def field(self, slot: int, name: str) -> np.ndarray:
        w = self.meta[slot]
        return ek_batch_get_fields(self.h, slot, name, w.cells, len(w.species))

    def collect(self, slot: int):
        w = self.meta.pop(slot)
        return ek_batch_collect(self.h, slot, len(w.spheres))

    def active(self):
        return ek_batch_active(self.h)

    def close(self):
        if self.h is not None:
            ek_batch_destroy(self.h)
            self.h = None
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- convenience wrapper -------------------------------------------------------
PRECISION = {"fp64": EK_FP64_PLAIN, "fp32": EK_FP32_DEV}
SCHEME = {"pv": EK_SCHEME_PARTIAL_VOLUME, "simple": EK_SCHEME_SIMPLE}
CHARGE = {"psi": EK_CHARGE_PSI, "uniform": EK_CHARGE_UNIFORM}
INTEGRATOR = {"vv": EK_VELOCITY_VERLET, "se": EK_SYMPLECTIC_EULER}


def params_from_workload(w, max_particles: int | None = None) -> ek_params:
    p = ek_params()
    p.nx, p.ny, p.nz = w.shape
    p.agrid, p.tau, p.kT, p.fluid_density, p.viscosity = w.agrid, w.tau, w.kT, w.fluid_density, w.nu
    p.n_species = len(w.species)
    for k, s in enumerate(w.species):
        p.species[k].D, p.species[k].valency, p.species[k].mean_density = s.D, s.z, s.mean
    p.bjerrum_length = w.lambda_B
    for d in range(3):
        p.E_ext[d] = w.E[d]
    p.precision = PRECISION[w.precision]
    p.scheme = SCHEME[w.scheme]
    p.charge_mode = CHARGE[w.charge]
    p.integrator = INTEGRATOR[w.integrator]
    p.max_particles = max(1, len(w.spheres)) if max_particles is None else max_particles
    return p


class EkSim:
    """One simulation on cuda:0 built from a workload description.  Device
    memory and the stream come from PyTorch; all computation happens in the
    library's kernels."""

    def __init__(self, w, initial_density: np.ndarray | None = None, use_torch: bool = True,
                 static_mask=None, static_charge=None, seeded: bool = False, max_particles: int | None = None):
        self.w = w
        self.N = w.cells
        self.ns = len(w.species)
        p = params_from_workload(w, max_particles=max_particles)
        self._arena = None
        self._stream = None
        if use_torch:
            import torch
            dev = torch.device("cuda", 0)
            self._stream = torch.cuda.Stream(device=dev)
            nbytes = ek_query_footprint(p)
            self._arena = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            torch.cuda.synchronize(dev)
            p.stream = self._stream.cuda_stream
            p.arena = self._arena.data_ptr()
            p.arena_bytes = nbytes
        self.params = p
        self.ctx = ek_create(p)
        for s in w.spheres:
            ek_add_sphere(self.ctx, s.x, s.R, s.Z, s.M, s.v, s.mode)
        if static_mask is not None:
            ek_set_static_boundary(self.ctx, static_mask, static_charge)
        if initial_density is not None:
            ek_set_fields(self.ctx, "density", initial_density)
        elif seeded:  # workloads.initial_densities(w), built on the device
            ek_seed_density(self.ctx, w.seed, w.noise)

    def prepare(self):
        ek_prepare(self.ctx)

    def step(self, n: int = 1):
        ek_step(self.ctx, n)

    def sync(self):
        ek_synchronize(self.ctx)

    def profile(self, n: int) -> dict:
        return ek_profile_stages(self.ctx, n)

    def field(self, name: str) -> np.ndarray:
        return ek_get_fields(self.ctx, name, self.N, self.ns)

    def set_field(self, name: str, values: np.ndarray):
        ek_set_fields(self.ctx, name, values)

    def particles(self) -> list:
        return ek_get_particles(self.ctx, len(self.w.spheres))

    def diagnostics(self) -> dict:
        return ek_get_diagnostics(self.ctx)

    def close(self):
        if self.ctx is not None:
            ek_destroy(self.ctx)
            self.ctx = None
        self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
