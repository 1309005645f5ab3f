/*
 * ek_oracle.h -- declarations of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This header belongs to the oracle and is used by
 * nothing but the oracle's own sources and its ctypes loader (oracle/oracle.py).
 * The GPU library has its own header (include/ek.h) and shares no code, no
 * header, no table and no helper with this one.
 *
 * Units: lattice units throughout (lattice spacing a = 1, time step tau = 1,
 * fluid reference density rho0 = 1).  The potential phi is dimensionless
 * (e*Phi/kT).  Cell (x, y, z) has index x + nx*(y + ny*z) and its centre at
 * (x + 1/2, y + 1/2, z + 1/2).  Populations are stored as f[i*N + cell],
 * species densities as rho[k*N + cell], vectors as v[d*N + cell].
 */
#ifndef EK_ORACLE_H
#define EK_ORACLE_H
#include <stdint.h>

#define OR_MAX_SPECIES 8

typedef struct {
    int nx, ny, nz;
    double nu;            /* kinematic viscosity */
    double kT;            /* thermal energy */
    double lambda_B;      /* Bjerrum length */
    double E[3];          /* uniform external field, kT/(e a) */
    int n_species;
    double D[OR_MAX_SPECIES];
    double z[OR_MAX_SPECIES];
    int partial_volume;   /* 1: partial-volume flux, 0: simple scheme */
    int charge_mode;      /* 0: Z*Psi_p/V_p, 1: Z/N_b on the particle's boundary cells */
    int integrator;       /* 0: velocity Verlet, 1: symplectic Euler */
} or_params;

typedef struct {
    double x[3], v[3], w[3];   /* centre, velocity, angular velocity */
    double R, Z, M;            /* radius, valency of the colloid, mass */
    int mode;                  /* 0 free, 1 prescribed velocity, 2 fixed in place */
    int pad;
    double F[3], T[3];         /* force/torque of the last completed step */
} or_particle;

/* Geometry of one unit cell vs one sphere: Psi as a count of 1/4096 sub-cells. */
int or_psi_count(double dx, double dy, double dz, double R);

void or_geometry(const or_params* p, const or_particle* pt, int np,
                 const uint8_t* static_mask, const double* static_charge,
                 uint8_t* flag, int32_t* owner, double* psi, double* rhob);

void or_init_fields(const or_params* p, const uint8_t* flag, const double* psi,
                    double* f, double* rho);

void or_boundary_update(const or_params* p, const or_particle* pt, int np,
                        const uint8_t* flag_old, const int32_t* owner_old,
                        const uint8_t* flag_new, const int32_t* owner_new,
                        double* f, double* rho,
                        double* Fcov, double* Tcov, int64_t* counts);

void or_charge(const or_params* p, const double* rho, const double* rhob, double* q);

void or_ek_update(const or_params* p, const double* rho_in, double* rho_out,
                  const double* phi, const double* psi, const uint8_t* flag,
                  const double* u, double* fext);

void or_lb_update(const or_params* p, const or_particle* pt,
                  const double* f_in, double* f_out,
                  const uint8_t* flag, const int32_t* owner,
                  const double* fext, double* u_out);

void or_hydro_force(const or_params* p, const or_particle* pt, int np,
                    const double* f_in, const uint8_t* flag, const int32_t* owner,
                    double* F, double* T);

void or_el_force(const or_params* p, const or_particle* pt, int np,
                 const double* phi, const uint8_t* flag, const int32_t* owner,
                 double* F, double* T);

int or_num_threads(void);
void or_move(const or_params* p, or_particle* pt, int np);
void or_finish(const or_params* p, or_particle* pt, int np,
               const double* Fnew, const double* Tnew);

#endif
