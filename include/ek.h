/*
 * ek.h -- C ABI of the MI355X (gfx950) library for one time step of lattice
 * electrokinetics with moving charged particles, after Kuron, Rempfer,
 * Schornbaum, Bauer, Godenschwager, Holm and de Graaf, "Moving Charged
 * Particles in Lattice Boltzmann-Based Electrokinetics" (J. Chem. Phys. 2016).
 *
 * One step (ek_step) advances, on the GPU only:
 *   - the particles (Sec. III.B: velocity Verlet or symplectic Euler),
 *   - their coverage of the lattice: boundary flags, partial volumes Psi
 *     (Sec. III.D.2), LB fluid destroyed/created in covered/vacated cells
 *     (Sec. III.B, after Aidun) and solute expelled from covered cells so that
 *     every species is conserved (Sec. III.D.1),
 *   - the charge density and the periodic Poisson equation (Eq. poisson, FFT),
 *   - the Nernst-Planck link fluxes (Sec. III.C: diffusive + migrative with
 *     partial-volume smoothing, Eq. flux-pv; volume-of-fluid advection), the
 *     continuity update and the coupling force on the fluid (Eq. fluidcoupling),
 *   - the D3Q19 TRT lattice Boltzmann stream/collide with the Guo force term
 *     (Eq. guo) and velocity bounce-back on the particles (Sec. III.A/B),
 *   - the momentum-exchange force and torque (Eq. force) and the electrostatic
 *     force on each particle.
 *
 * Conventions
 *   - Every function returns EK_OK (0) or a negative EK_ERR_* code; no call
 *     throws.  ek_strerror() names a code.  A device error is latched in the
 *     context and returned by every later call on it.
 *   - The volume-of-fluid advection (Sec. III.C) displaces a cell by u tau and
 *     intersects it with its 26 neighbours only, so the method needs every
 *     velocity component below one cell per step.  The kernels test each
 *     fluid cell's velocity (stream/collide) and each free sphere's (after
 *     each kick) and latch EK_ERR_UNSTABLE (|u_d| >= 1) or EK_ERR_NONFINITE
 *     (NaN or infinity) in a device status word; a sphere that fails stops
 *     where it is.  The synchronising calls (ek_get_*, ek_synchronize) report
 *     it, and ek_step reports it once the stream has passed the step that
 *     latched it; from then on the context returns that code.
 *   - The library owns contexts and all device memory it allocates; the caller
 *     owns every host buffer passed in or out (it is read or written during
 *     the call only).  Device memory may instead be provided by the caller as
 *     an arena (e.g. a PyTorch tensor); the caller then keeps it alive and
 *     unmodified until ek_destroy.
 *   - Calls are ordered on the context's stream.  ek_step only enqueues work;
 *     ek_get_* synchronise the stream before copying.
 *   - Units: the parameters are in simulation units (agrid, tau, kT and the
 *     fluid density fix the conversion to lattice units).  Fields and particle
 *     state are exchanged in the same simulation units.  The potential is
 *     e*Phi/kT.  Cell (x,y,z) is element x + nx*(y + ny*z) of a field; its
 *     centre is at ((x+1/2) agrid, (y+1/2) agrid, (z+1/2) agrid).
 *   - One context must not be used by two host threads at once.
 */
#ifndef EK_H
#define EK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EK_MAX_SPECIES 4

/* error codes */
#define EK_OK 0
#define EK_ERR_INVALID_ARG (-1)      /* null pointer, bad enum, size mismatch, bad value */
#define EK_ERR_UNSUPPORTED_SIZE (-2) /* a box edge is not 2^a 3^b with a >= 1, or outside [8, 512] */
#define EK_ERR_UNSTABLE (-3)         /* D tau/a^2 above the explicit-diffusion bound, viscosity <= 0,
                                        a sphere's initial speed of a cell per step or more; or
                                        (latched by the device) a fluid or sphere velocity
                                        component reached one cell per step */
#define EK_ERR_OVERLAP (-4)          /* a sphere too large for the box, or intersecting another */
#define EK_ERR_OOM (-5)              /* device allocation failed or the arena is too small */
#define EK_ERR_NO_SPACE (-6)         /* no free slot / memory for a batched simulation */
#define EK_ERR_NONFINITE (-7)        /* a NaN or infinity in host input; or (latched by the
                                        device) in a fluid or sphere velocity or a global sum */
#define EK_ERR_DEVICE (-8)           /* a HIP call failed (latched) */
#define EK_ERR_STATE (-9)            /* call not allowed in the current state */

/* ek_params.precision */
#define EK_FP64_PLAIN 0   /* every field stored and stepped in FP64 */
#define EK_FP32_DEV 1     /* FP32 storage: populations and densities as deviations
                             from the reference values; FP64 for particle state,
                             global sums, moving-boundary redistribution */
/* ek_params.scheme */
#define EK_SCHEME_PARTIAL_VOLUME 0  /* Sec. III.D.2, Eq. flux-pv */
#define EK_SCHEME_SIMPLE 1          /* Sec. III.D.1, Eq. flux-disc with expel + refill */
/* ek_params.charge_mode: how a particle's charge enters Poisson's equation */
#define EK_CHARGE_PSI 0             /* rho_b = Z Psi_p / V_p (Sec. III.D.2) */
#define EK_CHARGE_UNIFORM 1         /* Z spread equally over the particle's boundary cells */
/* ek_params.integrator (Sec. III.B) */
#define EK_VELOCITY_VERLET 0
#define EK_SYMPLECTIC_EULER 1
/* ek_add_sphere mode */
#define EK_FREE 0                   /* moved by the forces */
#define EK_PRESCRIBED 1             /* moves at its given velocity */
#define EK_FIXED 2                  /* does not move (co-moving frame) */

typedef struct {
    double D;            /* diffusion coefficient D_k (Eq. flux) */
    int valency;         /* z_k */
    double mean_density; /* reference density rho_k (number per volume); the
                            FP32 path stores deviations from it */
} ek_species;

typedef struct {
    int nx, ny, nz;               /* periodic box in cells; each 2^a 3^b, a >= 1, 8..512 */
    double agrid, tau;            /* lattice spacing and time step (Sec. III.A) */
    double kT;                    /* thermal energy */
    double fluid_density;         /* fluid mass density (reference density of the LB) */
    double viscosity;             /* kinematic viscosity */
    int n_species;                /* 1..EK_MAX_SPECIES */
    ek_species species[EK_MAX_SPECIES];
    double bjerrum_length;        /* lambda_B (Eq. poisson) */
    double E_ext[3];              /* uniform external field in kT/(e * length) */
    int precision;                /* EK_FP64_PLAIN | EK_FP32_DEV */
    int scheme;                   /* EK_SCHEME_* */
    int charge_mode;              /* EK_CHARGE_* */
    int integrator;               /* EK_VELOCITY_VERLET | EK_SYMPLECTIC_EULER */
    int max_particles;            /* capacity of ek_add_sphere (1..1024) */
    void* stream;                 /* hipStream_t to order work on; NULL: the library creates one */
    void* arena;                  /* optional caller device memory (>= ek_query_footprint); NULL: library allocates */
    size_t arena_bytes;
} ek_params;

typedef struct {
    double x[3], v[3], omega[3];  /* centre, velocity, angular velocity */
    double F[3], T[3];            /* total force / torque of the last step */
    double F_hyd[3], F_el[3], F_cov[3]; /* its parts: momentum exchange (Eq. force),
                                         electrostatic, fluid destroyed/created */
    double radius, charge, mass;
    int mode;
    int n_boundary;               /* boundary cells it owns: cells whose centre is inside it
                                     (simple scheme, Fig. 1) or, with partial volumes, cells
                                     completely inside it (Psi = 1, Sec. III.D.2) */
} ek_particle;

typedef struct {
    long long step;
    double species_total[EK_MAX_SPECIES]; /* FP64 sum over cells of rho_k * agrid^3 */
    double solute_charge;                 /* sum_k z_k species_total[k] */
    double particle_charge;               /* sum over cells of rho_b * agrid^3 */
    double fluid_mass;                    /* sum over fluid cells of the LB density * agrid^3 */
    double fluid_momentum[3];
    long long covered, vacated, pooled;   /* moving-boundary events of the last step */
    long long boundary_cells;             /* cells flagged as boundary now */
    double max_velocity;                  /* max |u| over fluid cells (lattice units) */
} ek_diag;

typedef struct ek_ctx ek_ctx;

/* field ids for ek_get_fields / ek_set_fields; sizes are in elements, x fastest */
#define EK_FIELD_DENSITY 0        /* n_species * N doubles (species-major) */
#define EK_FIELD_PHI 1            /* N doubles, e*Phi/kT (periodic part; E_ext is separate) */
#define EK_FIELD_VELOCITY 2       /* 3 * N doubles, component-major; 0 in boundary cells */
#define EK_FIELD_FLUID_DENSITY 3  /* N doubles (sum of populations) */
#define EK_FIELD_FORCE 4          /* 3 * N doubles, coupling force density of the last step */
#define EK_FIELD_PSI 5            /* N doubles, partial volume in [0, 1] */
#define EK_FIELD_FLAG 6           /* N uint8: 1 boundary, 0 fluid */
#define EK_FIELD_OWNER 7          /* N int32: owning particle id, -1 for none */
#define EK_FIELD_POPULATIONS 8    /* 19 * N doubles, post-collision f_i (direction-major) */
#define EK_FIELD_PARTICLE_CHARGE 9 /* N doubles, rho_b */

/* Device bytes a context with these parameters needs (arena size). */
int ek_query_footprint(const ek_params* p, size_t* bytes);

/* Validate the parameters, take (or allocate) device memory and set the fluid
 * at rest and every species at its mean density.  Errors: INVALID_ARG,
 * UNSUPPORTED_SIZE, UNSTABLE, OOM, DEVICE. */
int ek_create(const ek_params* p, ek_ctx** out);

/* Add a sphere (Sec. III.B): centre pos, radius, valency of its charge
 * (charge = Z in units of e), mass, initial velocity v0 (may be NULL), and mode
 * EK_FREE / EK_PRESCRIBED / EK_FIXED.  Allowed before the first step only.
 * Returns its id in *id (may be NULL).  Errors: INVALID_ARG, OVERLAP (2R + 2
 * cells exceed an edge, or the sphere intersects one already added: centres
 * closer than the sum of the radii, minimum image), UNSTABLE (a component of
 * v0 of one cell per step or more), STATE (after the first step or beyond
 * max_particles). */
int ek_add_sphere(ek_ctx* c, const double pos[3], double radius, double charge, double mass,
                  const double v0[3], int mode, int* id);

/* Test hook: resting walls (mask != 0) carrying an optional fixed charge
 * density (may be NULL), both N elements.  Before the first step only. */
int ek_set_static_boundary(ek_ctx* c, const uint8_t* mask, const double* charge);

/* Overwrite a field from a host buffer of exactly the size listed above
 * (DENSITY, PHI, VELOCITY, FORCE, POPULATIONS).  DENSITY set before the first
 * step is the initial concentration: at preparation, boundary cells are
 * emptied and, in the partial-volume scheme, fluid cells keep (1 - Psi) of it. */
int ek_set_fields(ek_ctx* c, int field, const void* host, size_t bytes);

/* Seeded initial concentration computed on the device, no host buffer: the
 * workloads' input recipe (not a step of the method), rho_k(cell) =
 * mean_density_k (1 + noise (2U - 1)) with U = (splitmix64(cell ^ seed ^
 * (k << 40)) >> 11) 2^-53 (splitmix64 of Steele, Lea and Flood, 2014; cells x
 * fastest, k the species index), every operation rounded once in FP64 in that
 * order.  The result is what ek_set_fields(DENSITY) stores for the same values
 * computed on the host, and is treated as that call's is.  Errors:
 * INVALID_ARG (noise not finite or |noise| > 1), DEVICE. */
int ek_seed_density(ek_ctx* c, uint64_t seed, double noise);

/* Compute the initial coverage (flags, Psi, particle charge) and apply the
 * initial-density rule.  Called by the first ek_step if not called before. */
int ek_prepare(ek_ctx* c);

/* Enqueue n >= 0 full time steps on the context's stream (captured once in a
 * HIP graph and replayed).  Returns without waiting. */
int ek_step(ek_ctx* c, int n);

/* ek_step for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Enqueues
 * the same kernels as ek_step (same results, bit for bit) directly on the
 * context's stream -- no graph is built, nothing is allocated -- with the
 * per-(particle, chunk) partial sums of the particle kernels in a fixed device
 * array of 512 KiB that the library holds on each GPU for the life of the
 * process.  The context must be prepared (ek_prepare or an earlier ek_step;
 * EK_ERR_STATE otherwise).  EK_ERR_NO_SPACE when those partial sums, 3 x
 * particles x workgroups per particle box x 128 bytes, exceed 512 KiB (64
 * spheres of radius 6 take 295 KiB).  Every call on one GPU shares that
 * array: calls that overlap on one GPU (other host threads, other streams)
 * race and must be ordered by the caller.  The first call on a GPU resolves
 * the array's address (no allocation).  Errors otherwise as ek_step; a
 * status latched by the kernels is reported by the synchronising calls. */
int ek_step_noalloc(ek_ctx* c, int n);

/* Relative permittivity field: Poisson's equation with an inhomogeneous
 * dielectric, which the FFT solver cannot take (Sec. III.C names iterative
 * solvers for it).  eps_r: N values > 0 (x fastest), relative to the
 * permittivity that defines bjerrum_length; copied.  From the next step on
 * the potential solves
 *   sum over the 6 faces f of c: e_f (phi_c - phi_n) = 4 pi lambda_B (q_c - mean q)
 * on the periodic lattice (the 7-point form of -div(eps grad phi) =
 * 4 pi lambda_B q; e_f is the harmonic mean of the two cells' eps_r; for
 * eps_r = 1 this is the FFT solver's equation) by Jacobi-preconditioned
 * conjugate gradients in FP64, warm-started from the previous step's
 * potential, until |r| <= tol |b| (0 < tol < 1) or max_iter iterations; the
 * potential is shifted to zero mean.  The solve is driven from the host: it
 * checks its residual every 8 iterations (a wait on the stream), so steps are
 * not replayed from graphs while a permittivity is set, and ek_step returns
 * when they are done.  A solve that misses the tolerance latches
 * EK_ERR_UNSTABLE.  eps_r == NULL returns to the FFT solver.  Allocates
 * 9 N doubles of device memory (outside the arena).  Errors: INVALID_ARG,
 * NONFINITE, OOM, DEVICE. */
int ek_set_permittivity(ek_ctx* c, const double* eps_r, double tol, int max_iter);

/* Iterations and relative residual |r| / |b| of the last iterative Poisson
 * solve (0 and 0 with the FFT solver). */
int ek_get_poisson_stats(ek_ctx* c, int* iterations, double* residual);

/* Copy a field to a host buffer of exactly the listed size (synchronises). */
int ek_get_fields(ek_ctx* c, int field, void* host, size_t bytes);

/* Copy the state of the first n particles (synchronises). */
int ek_get_particles(ek_ctx* c, ek_particle* out, int n);

/* FP64 global sums computed on the device (synchronises). */
int ek_get_diagnostics(ek_ctx* c, ek_diag* out);

/* Checkpoint: the full device state as an opaque byte image.  With host ==
 * NULL, *bytes receives the size.  ek_set_state restores an image taken from a
 * context created with the same parameters and particle count. */
int ek_get_state(ek_ctx* c, void* host, size_t* bytes);
int ek_set_state(ek_ctx* c, const void* host, size_t bytes);

/* Instrumentation: run n steps without graph replay, timing each stage with
 * HIP events recorded on the context's stream.  ms_out[k] (k < n_out <=
 * EK_N_STAGES) receives the mean duration in milliseconds of stage k.  The
 * steps are real steps of the simulation.  Synchronises. */
#define EK_STAGE_MOVE 0      /* particle kick/drift and boxes */
#define EK_STAGE_GEOMETRY 1  /* flags, owners, Psi, particle charge */
#define EK_STAGE_BOUNDARY 2  /* Aidun destroy/create, expel, refill, pool */
#define EK_STAGE_POISSON 3   /* charge assembly + 5 FFT passes */
#define EK_STAGE_FORCES 4    /* momentum-exchange (populations before streaming) and electrostatic forces */
#define EK_STAGE_EK 5        /* link fluxes, continuity, coupling force; in FP64 also stream/collide (fused) */
#define EK_STAGE_LB 6        /* stream/collide as its own kernel (FP32); 0 where fused into EK_STAGE_EK */
#define EK_STAGE_FINISH 7    /* closing kick */
#define EK_N_STAGES 8
int ek_profile_stages(ek_ctx* c, int n, double* ms_out, int n_out);

/* Bandwidth probe: a plain device-to-device copy kernel of `bytes` (a
 * multiple of 16, at most 2^40) on `stream` (hipStream_t; NULL = default stream).  dst and
 * src are device pointers owned by the caller; the call only enqueues. */
int ek_copy_probe(void* dst, const void* src, size_t bytes, void* stream);

/* Wait for all enqueued work of the context. */
int ek_synchronize(ek_ctx* c);

int ek_destroy(ek_ctx* c);
const char* ek_strerror(int code);

/* ---------------------------------------------------------------------------
 * Serving form: many independent FP32 simulations of different box sizes and
 * particle counts resident in one device arena and advanced together.  Each
 * kernel of a step runs once for the whole batch (its workgroups cover the
 * concatenated work of all slots), and the step is a HIP graph, captured again
 * when an admission or retirement changes the amount of work, so requests can
 * be admitted and retired between steps.  Every simulation's arithmetic is
 * independent of the others: a request gives the same bits alone and in any
 * mix.
 * ------------------------------------------------------------------------- */
typedef struct ek_batch ek_batch;

typedef struct {
    double x[3], v[3];            /* centre and initial velocity */
    double radius, charge, mass;  /* as for ek_add_sphere */
    int mode;                     /* EK_FREE | EK_PRESCRIBED | EK_FIXED */
} ek_sphere;

#define EK_BATCH_MAX_SLOTS 64

/* Create a batch over `arena_bytes` of device memory (the caller's `arena`,
 * or allocated when NULL) for simulations with `n_species` species, ordered
 * on `stream` (NULL: the library creates one).  Errors: INVALID_ARG, OOM. */
int ek_batch_create(size_t arena_bytes, int n_species, void* stream, void* arena, ek_batch** out);

/* Admit one request: parameters (precision must be EK_FP32_DEV, n_species as
 * the batch; stream/arena/max_particles are set by the batch), its spheres,
 * an optional initial density (n_species * N doubles, or NULL for the means)
 * and the number of steps to run.  Returns the slot.  EK_ERR_NO_SPACE when no
 * slot or no contiguous arena range of the request's footprint is free.
 * The request's state is built on a stream of the batch's own and waited
 * for; the steps already queued keep running meanwhile. */
int ek_batch_admit(ek_batch* b, const ek_params* p, const ek_sphere* spheres, int n_spheres,
                   const double* initial_density, long long n_steps, int* slot);

/* ek_batch_admit with the seeded initial density of ek_seed_density(seed,
 * noise) in place of a host array: the request's initial state is built on
 * the device.  Errors as ek_batch_admit and ek_seed_density. */
int ek_batch_admit_seeded(ek_batch* b, const ek_params* p, const ek_sphere* spheres, int n_spheres,
                          uint64_t seed, double noise, long long n_steps, int* slot);

/* Enqueue a chunk of k batched steps; slots that reach their requested steps
 * stop.  Slots admitted or collected since the last call join or leave the
 * table in stream order, without waiting for the queued steps.  At most two
 * chunks are queued ahead of the host: with two queued, the call first waits
 * for the older one to finish. */
int ek_batch_step(ek_batch* b, int k);

/* Slots whose requested steps are all done, or whose simulation latched an
 * error (it then stops stepping), and not yet collected (at most cap of them
 * written to done_slots), as of the chunks that have finished.  Does not
 * wait: a slot finishing in a chunk still running is reported by a later
 * call (or after ek_batch_wait). */
int ek_batch_poll(ek_batch* b, int* done_slots, int cap, int* n_done);

/* Wait for every queued chunk; ek_batch_poll then reports their outcome. */
int ek_batch_wait(ek_batch* b);

/* Copy a slot's particles (first n) and diagnostics (either may be NULL) and
 * free the slot and its memory.  A slot whose simulation latched an error is
 * freed without copying, and its code (EK_ERR_UNSTABLE or EK_ERR_NONFINITE)
 * is returned.  A slot reported by ek_batch_poll is read without waiting for
 * the queued steps; any other slot first waits for them. */
int ek_batch_collect(ek_batch* b, int slot, ek_particle* out, int n, ek_diag* diag);

/* A field of a live slot, as ek_get_fields (tests).  Synchronises. */
int ek_batch_get_fields(ek_batch* b, int slot, int field, void* host, size_t bytes);

/* Number of slots still stepping and their total cells. */
int ek_batch_active(ek_batch* b, int* n_active, long long* cells);

int ek_batch_destroy(ek_batch* b);

#ifdef __cplusplus
}
#endif
#endif
