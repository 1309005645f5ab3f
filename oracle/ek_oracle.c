/*
 * ek_oracle.c -- plain, slow, FP64 CPU oracle for one time step of lattice
 * electrokinetics with moving charged particles (Kuron et al., "Moving
 * Charged Particles in Lattice Boltzmann-Based Electrokinetics").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code with
 * the GPU library.  Every function below is a direct, loop-by-loop statement of
 * the passage it cites; there is no blocking, fusion or reordering beyond what
 * that passage states.  Loops over cells are written in gather form (each cell
 * writes only itself), so the OpenMP pragmas do not change any result.
 *
 * Readings of passages that are silent or garbled in the paper are marked
 * "Reading:" and are listed in the design notes of the repository.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * so coverage decisions are reproducible operation by operation).
 */
#include "ek_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Number of OpenMP threads the oracle's parallel loops use, and a setter
 * (timing with a chosen number of threads; n < 1 is ignored). */
int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_num_threads(int n) {
    if (n >= 1) omp_set_num_threads(n);
}

/* ---------------------------------------------------------------------------
 * D3Q19 velocity set (Sec. III.A: rest vector, 6 face and 12 edge neighbours).
 * Order: rest; +-x, +-y, +-z; then the 12 edges as opposite pairs.
 * Weights: 1/3, 1/18, 1/36 (the standard D3Q19 weights; the paper names w_i
 * without values).
 * ------------------------------------------------------------------------- */
static const int CV[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const int OPP[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

static double weight(int i) {
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* The 13 link directions of one half of the 26-neighbourhood.  The first 9 are
 * the D3Q19 links that carry the diffusive/migrative flux; all 13 carry the
 * volume-of-fluid advective flux (Sec. III.C: the displaced cell is intersected
 * with all 26 neighbours). */
static const int HALF[13][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1},
    {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

static long ncells(const or_params* p) { return (long)p->nx * p->ny * p->nz; }

static int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

static long cell_at(const or_params* p, int x, int y, int z) {
    return (long)wrap(x, p->nx) + (long)p->nx * ((long)wrap(y, p->ny) + (long)p->ny * wrap(z, p->nz));
}

static void cell_coords(const or_params* p, long c, int* x, int* y, int* z) {
    *x = (int)(c % p->nx);
    *y = (int)((c / p->nx) % p->ny);
    *z = (int)(c / ((long)p->nx * p->ny));
}

/* Minimum-image displacement of a cell-centre coordinate from a particle
 * coordinate along one periodic axis of length L. */
static double min_image(double centre, double x, double L) {
    double d = centre - x;
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

static void cell_disp(const or_params* p, long c, const or_particle* q, double d[3]) {
    int x, y, z;
    cell_coords(p, c, &x, &y, &z);
    d[0] = min_image((double)x + 0.5, q->x[0], (double)p->nx);
    d[1] = min_image((double)y + 0.5, q->x[1], (double)p->ny);
    d[2] = min_image((double)z + 0.5, q->x[2], (double)p->nz);
}

/* Reading (simple scheme): a cell belongs to a particle iff its centre lies
 * within distance R (Fig. 1 caption: cells whose centre is inside the particle
 * are boundary nodes); the tie d^2 == R^2 counts as inside.  The
 * partial-volume scheme claims a cell only once it is completely inside the
 * particle, Psi_p = 1 (see or_geometry). */
static int centre_inside(const double d[3], double R) {
    double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    return d2 <= R * R;
}

/* ---------------------------------------------------------------------------
 * Psi: overlapped volume fraction (Sec. III.D.2).  The cell is split into 8
 * equal sub-cells; a sub-cell entirely inside or entirely outside the sphere is
 * decided, any other is split again, to a maximum depth of 4 (sub-cells of
 * edge 1/16).  Reading: an undecided depth-4 sub-cell counts iff its centre is
 * inside.  The result is returned as a count of depth-4 sub-cells (0..4096).
 * Box coordinates are relative to the sphere centre.
 * ------------------------------------------------------------------------- */
static int psi_rec(double lx, double ly, double lz, double h, int depth, double R2) {
    double hx = lx + h, hy = ly + h, hz = lz + h;
    double fx = (lx * lx > hx * hx) ? lx * lx : hx * hx;
    double fy = (ly * ly > hy * hy) ? ly * ly : hy * hy;
    double fz = (lz * lz > hz * hz) ? lz * lz : hz * hz;
    double far2 = (fx + fy) + fz;
    int leaves = 1 << (3 * (4 - depth));
    if (far2 <= R2) return leaves; /* entirely inside */
    double nx = (lx > 0.0) ? lx : ((hx < 0.0) ? hx : 0.0);
    double ny = (ly > 0.0) ? ly : ((hy < 0.0) ? hy : 0.0);
    double nz = (lz > 0.0) ? lz : ((hz < 0.0) ? hz : 0.0);
    double near2 = (nx * nx + ny * ny) + nz * nz;
    if (near2 >= R2) return 0; /* entirely outside */
    if (depth == 4) {
        double cx = lx + 0.5 * h, cy = ly + 0.5 * h, cz = lz + 0.5 * h;
        return ((cx * cx + cy * cy) + cz * cz) <= R2 ? 1 : 0;
    }
    double hh = 0.5 * h;
    int s = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                s += psi_rec(a ? lx + hh : lx, b ? ly + hh : ly, c ? lz + hh : lz, hh, depth + 1, R2);
    return s;
}

int or_psi_count(double dx, double dy, double dz, double R) {
    return psi_rec(dx - 0.5, dy - 0.5, dz - 0.5, 1.0, 0, R * R);
}

static int far_from(const double d[3], double R) {
    return fabs(d[0]) > R + 1.0 || fabs(d[1]) > R + 1.0 || fabs(d[2]) > R + 1.0;
}

static double sphere_volume(double R) { return 4.0 / 3.0 * M_PI * R * R * R; }

/* ---------------------------------------------------------------------------
 * Geometry: boundary flag, owner (lowest index of the particles that claim the
 * cell; -1 for static walls and fluid), Psi = min(1, sum_p Psi_p), and the
 * particles' charge density rho_b (Sec. III.D.2: rho_b = Z e Psi / V_p with V_p
 * the continuum volume; or, in the uniform mode, Z spread equally over the
 * particle's boundary cells) plus any static boundary charge (Sec. III.C).
 * A particle claims a cell (makes it a boundary cell):
 *   simple scheme: when the cell's centre is inside it (Fig. 1 caption);
 *   partial-volume scheme: when the cell is completely inside it, Psi_p = 1
 *   (Sec. III.D.2 defines Psi = 1 as completely inside).
 * Reading of the partial-volume rule: Sec. III.D.2 expects a claimed cell to
 * hold little solute, a residue left only by the particle's discrete steps
 * (the solute sits in the non-overlapped part, (1 - Psi) of the cell, so the
 * cell is nearly empty only as Psi approaches 1); it lets vacated cells start
 * from zero concentration; and Sec. IV.A sizes the moving particle by the
 * number of its cells with Psi = 1.  All three hold when the claim happens at
 * Psi = 1.
 * ------------------------------------------------------------------------- */
void or_geometry(const or_params* p, const or_particle* pt, int np,
                 const uint8_t* static_mask, const double* static_charge,
                 uint8_t* flag, int32_t* owner, double* psi, double* rhob) {
    long N = ncells(p);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
        int st = static_mask ? static_mask[c] != 0 : 0;
        int fl = st, ow = -1;
        double psum = 0.0, qb = static_charge ? static_charge[c] : 0.0;
        for (int k = 0; k < np; ++k) {
            double d[3];
            cell_disp(p, c, &pt[k], d);
            if (far_from(d, pt[k].R)) continue;
            int cnt = or_psi_count(d[0], d[1], d[2], pt[k].R);
            int claims = p->partial_volume ? cnt == 4096 : centre_inside(d, pt[k].R);
            if (!fl && claims) {
                fl = 1;
                ow = k;
            }
            psum += (double)cnt / 4096.0;
            if (p->charge_mode == 0) qb += pt[k].Z * ((double)cnt / 4096.0) / sphere_volume(pt[k].R);
        }
        flag[c] = (uint8_t)fl;
        owner[c] = ow;
        psi[c] = psum < 1.0 ? psum : 1.0;
        rhob[c] = qb;
    }
    if (p->charge_mode == 1 && np > 0) {
        long* nb = calloc((size_t)np, sizeof(long));
        for (long c = 0; c < N; ++c)
            if (owner[c] >= 0) nb[owner[c]]++;
        for (long c = 0; c < N; ++c)
            if (owner[c] >= 0) rhob[c] += pt[owner[c]].Z / (double)nb[owner[c]];
        free(nb);
    }
}

/* Initial state: fluid at rest with density rho0 = 1 (f_i = w_i); no solute in
 * boundary cells; in the partial-volume scheme a fluid cell holds (1 - Psi) of
 * the given concentration (the solute sits in the non-overlapped part,
 * Sec. III.D.2).  Reading: the paper does not state the initial condition. */
void or_init_fields(const or_params* p, const uint8_t* flag, const double* psi,
                    double* f, double* rho) {
    long N = ncells(p);
    for (int i = 0; i < 19; ++i)
        for (long c = 0; c < N; ++c) f[i * N + c] = weight(i);
    for (int k = 0; k < p->n_species; ++k)
        for (long c = 0; c < N; ++c) {
            if (flag[c]) rho[k * N + c] = 0.0;
            else if (p->partial_volume) rho[k * N + c] *= (1.0 - psi[c]);
        }
}

static void boundary_velocity(const or_params* p, const or_particle* pt, long c, int32_t ow, double vb[3]) {
    if (ow < 0) {
        vb[0] = vb[1] = vb[2] = 0.0;
        return;
    }
    const or_particle* q = &pt[ow];
    double r[3];
    cell_disp(p, c, q, r);
    /* Sec. III.B: v_b = v + omega x (r_b - r) */
    vb[0] = q->v[0] + (q->w[1] * r[2] - q->w[2] * r[1]);
    vb[1] = q->v[1] + (q->w[2] * r[0] - q->w[0] * r[2]);
    vb[2] = q->v[2] + (q->w[0] * r[1] - q->w[1] * r[0]);
}

static void cross_add(double T[3], const double r[3], const double v[3], double sign) {
    T[0] += sign * (r[1] * v[2] - r[2] * v[1]);
    T[1] += sign * (r[2] * v[0] - r[0] * v[2]);
    T[2] += sign * (r[0] * v[1] - r[1] * v[0]);
}

/* ---------------------------------------------------------------------------
 * Moving-boundary update after the particles moved (Sec. III.B and III.D).
 *   covered  C: fluid before, boundary now;  vacated V: boundary before, fluid
 *   now;  stable fluid S: fluid before and now.
 * 1. LB (Aidun): the fluid of a covered cell is destroyed and its momentum p_f
 *    given to the particle as a force p_f/tau; a vacated cell is filled with the
 *    equilibrium at the particle's surface velocity and the mean density of its
 *    stable-fluid D3Q19 neighbours (rho0 if none), and its momentum is taken from
 *    the particle.  Reading: the force acts at the cell centre, so it also
 *    carries a torque.
 * 2. EK expel (Sec. III.D.1): the solute of a covered cell is redistributed.
 *    Reading: equal shares to its stable-fluid D3Q19 neighbours; if it has none,
 *    to its stable-fluid D3Q27 neighbours; if none either, spread uniformly over
 *    all stable-fluid cells.
 * 3. Simple scheme only (Eqs. refill / refill-neighbours): a vacated cell takes
 *    1/(N_f+1) of each of its N_f stable-fluid D3Q19 neighbours' solute.
 *    Reading: the neighbours' loss uses the post-expel values of all vacated
 *    cells at once.  In the partial-volume scheme vacated cells start empty.
 * counts[0..2] = number of covered, vacated and pool-expelled cells.
 * ------------------------------------------------------------------------- */
void or_boundary_update(const or_params* p, const or_particle* pt, int np,
                        const uint8_t* flag_old, const int32_t* owner_old,
                        const uint8_t* flag_new, const int32_t* owner_new,
                        double* f, double* rho,
                        double* Fcov, double* Tcov, int64_t* counts) {
    (void)np;
    long N = ncells(p);
    int ns = p->n_species;
    int64_t ncov = 0, nvac = 0, npool = 0;
#define STABLE(c) (!flag_old[c] && !flag_new[c])

    /* 1. LB fluid destroy / create */
    for (long c = 0; c < N; ++c) {
        int cov = !flag_old[c] && flag_new[c];
        int vac = flag_old[c] && !flag_new[c];
        if (cov) {
            ncov++;
            int ow = owner_new[c];
            if (ow < 0) continue;
            double pf[3] = {0, 0, 0};
            for (int i = 0; i < 19; ++i)
                for (int d = 0; d < 3; ++d) pf[d] += f[i * N + c] * CV[i][d];
            double r[3];
            cell_disp(p, c, &pt[ow], r);
            for (int d = 0; d < 3; ++d) Fcov[3 * ow + d] += pf[d];
            cross_add(&Tcov[3 * ow], r, pf, 1.0);
        } else if (vac) {
            nvac++;
            int ow = owner_old[c];
            int x, y, z;
            cell_coords(p, c, &x, &y, &z);
            double sum = 0.0;
            int nf = 0;
            for (int i = 1; i < 19; ++i) {
                long n = cell_at(p, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
                if (!STABLE(n)) continue;
                double rn = 0.0;
                for (int j = 0; j < 19; ++j) rn += f[j * N + n];
                sum += rn;
                nf++;
            }
            double rbar = nf > 0 ? sum / nf : 1.0;
            double vb[3];
            boundary_velocity(p, pt, c, ow, vb);
            double usq = vb[0] * vb[0] + vb[1] * vb[1] + vb[2] * vb[2];
            double pf[3] = {0, 0, 0};
            for (int i = 0; i < 19; ++i) {
                double cu = CV[i][0] * vb[0] + CV[i][1] * vb[1] + CV[i][2] * vb[2];
                double feq = weight(i) * (rbar + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                f[i * N + c] = feq;
                for (int d = 0; d < 3; ++d) pf[d] += feq * CV[i][d];
            }
            if (ow >= 0) {
                double r[3];
                cell_disp(p, c, &pt[ow], r);
                for (int d = 0; d < 3; ++d) Fcov[3 * ow + d] -= pf[d];
                cross_add(&Tcov[3 * ow], r, pf, -1.0);
            }
        }
    }

    /* 2. expel solute from covered cells */
    double* snap = malloc(sizeof(double) * (size_t)ns * N);
    memcpy(snap, rho, sizeof(double) * (size_t)ns * N);
    int* n19 = calloc((size_t)N, sizeof(int));
    int* n27 = calloc((size_t)N, sizeof(int));
    long nS = 0;
    double pool[OR_MAX_SPECIES] = {0};
    for (long c = 0; c < N; ++c) {
        if (STABLE(c)) nS++;
        if (!(!flag_old[c] && flag_new[c])) continue;
        int x, y, z;
        cell_coords(p, c, &x, &y, &z);
        for (int i = 1; i < 19; ++i)
            if (STABLE(cell_at(p, x + CV[i][0], y + CV[i][1], z + CV[i][2]))) n19[c]++;
        for (int a = -1; a <= 1; ++a)
            for (int b = -1; b <= 1; ++b)
                for (int e = -1; e <= 1; ++e) {
                    if (!a && !b && !e) continue;
                    if (STABLE(cell_at(p, x + a, y + b, z + e))) n27[c]++;
                }
        if (n27[c] == 0) {
            npool++;
            for (int k = 0; k < ns; ++k) pool[k] += snap[k * N + c];
        }
    }
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        int cov = !flag_old[n] && flag_new[n];
        if (cov) {
            for (int k = 0; k < ns; ++k) rho[k * N + n] = 0.0;
            continue;
        }
        if (!STABLE(n)) continue;
        int x, y, z;
        cell_coords(p, n, &x, &y, &z);
        for (int k = 0; k < ns; ++k) {
            double gain = 0.0;
            for (int i = 1; i < 19; ++i) {
                long c = cell_at(p, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
                if (!flag_old[c] && flag_new[c] && n19[c] > 0) gain += snap[k * N + c] / n19[c];
            }
            for (int a = -1; a <= 1; ++a)
                for (int b = -1; b <= 1; ++b)
                    for (int e = -1; e <= 1; ++e) {
                        if (!a && !b && !e) continue;
                        long c = cell_at(p, x + a, y + b, z + e);
                        if (!flag_old[c] && flag_new[c] && n19[c] == 0 && n27[c] > 0)
                            gain += snap[k * N + c] / n27[c];
                    }
            if (nS > 0) gain += pool[k] / (double)nS;
            rho[k * N + n] = snap[k * N + n] + gain;
        }
    }

    /* 3. refill vacated cells (simple scheme) */
    if (!p->partial_volume) {
        memcpy(snap, rho, sizeof(double) * (size_t)ns * N);
        int* nf = calloc((size_t)N, sizeof(int));
        for (long v = 0; v < N; ++v) {
            if (!(flag_old[v] && !flag_new[v])) continue;
            int x, y, z;
            cell_coords(p, v, &x, &y, &z);
            for (int i = 1; i < 19; ++i)
                if (STABLE(cell_at(p, x + CV[i][0], y + CV[i][1], z + CV[i][2]))) nf[v]++;
        }
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            int vac = flag_old[n] && !flag_new[n];
            if (!vac && !STABLE(n)) continue;
            int x, y, z;
            cell_coords(p, n, &x, &y, &z);
            for (int k = 0; k < ns; ++k) {
                if (vac) {
                    double s = 0.0;
                    for (int i = 1; i < 19; ++i) {
                        long m = cell_at(p, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
                        if (STABLE(m)) s += snap[k * N + m] / (nf[n] + 1);
                    }
                    rho[k * N + n] = snap[k * N + n] + s;
                } else {
                    double loss = 0.0;
                    for (int i = 1; i < 19; ++i) {
                        long v = cell_at(p, x + CV[i][0], y + CV[i][1], z + CV[i][2]);
                        if (flag_old[v] && !flag_new[v]) loss += snap[k * N + n] / (nf[v] + 1);
                    }
                    rho[k * N + n] = snap[k * N + n] - loss;
                }
            }
        }
        free(nf);
    }
#undef STABLE
    free(snap);
    free(n19);
    free(n27);
    if (counts) {
        counts[0] = ncov;
        counts[1] = nvac;
        counts[2] = npool;
    }
}

/* Charge density entering Poisson's equation (Eq. poisson plus the boundary
 * charge of Sec. III.C / III.D.2): q = sum_k z_k rho_k + rho_b. */
void or_charge(const or_params* p, const double* rho, const double* rhob, double* q) {
    long N = ncells(p);
    for (long c = 0; c < N; ++c) {
        double s = 0.0;
        for (int k = 0; k < p->n_species; ++k) s += p->z[k] * rho[k * N + c];
        q[c] = s + rhob[c];
    }
}

/* ---------------------------------------------------------------------------
 * EK solute update (Sec. III.C and III.D.2).
 *
 * Diffusive + migrative flux on a D3Q19 link a -> b = a + s (Eq. flux-pv, the
 * partial-volume form, multiplied out so nothing is divided by 1 - Psi):
 *   j = D/(A0 |s|) * [ rho_a(1-Psi_b) - rho_b(1-Psi_a)
 *                      + z/2 (rho_a(1-Psi_b) + rho_b(1-Psi_a)) (phi_a - phi_b + E.s) ]
 * Readings: (i) the migrative term enters with + (so that positive ions move
 * down the potential and the Boltzmann distribution is stationary); (ii) the
 * factor 1/(A0|s|), A0 = 1 + 2 sqrt 2, multiplies both terms, which is the
 * normalisation under which the mean-square displacement grows by 6 D per step
 * (Sec. III.C); (iii) the external field is a uniform gradient kept outside phi.
 * In the simple scheme Psi = 0 (Eq. flux-disc).
 *
 * Advective flux by volume of fluid (Sec. III.C): the cell at a is displaced by
 * u(a) and intersected with its 26 neighbours; the fraction sent to a + s is
 * prod_d g(s_d, u_d) with g(0,u) = 1 - |u|, g(sign u, u) = |u|, else 0.
 * Link form: J_adv(a->b) = rho_a g(s; u_a) - rho_b g(-s; u_b).
 *
 * Every flux into or out of a boundary cell is zero (Sec. III.C).
 * Continuity (Sec. III.C): rho(t+1) = rho(t) - sum over the 26 outgoing links.
 * Coupling force (Eq. fluidcoupling, discrete form in Sec. III.C):
 *   f(r) = kT/2 sum_k sum_{i=1..18} j_ki(r -> r+c_i) c_i / D_k.
 * Reading: the factor 1/2 (each link's friction is shared by its two cells);
 * with it a uniform density in a uniform field gives f = sum_k z_k rho_k E.
 * ------------------------------------------------------------------------- */
static double adv_frac(int sx, int sy, int sz, const double u[3]) {
    int s[3] = {sx, sy, sz};
    double g = 1.0;
    for (int d = 0; d < 3; ++d) {
        double a = fabs(u[d]);
        if (s[d] == 0) g *= (1.0 - a);
        else if ((s[d] > 0 && u[d] > 0.0) || (s[d] < 0 && u[d] < 0.0)) g *= a;
        else return 0.0;
    }
    return g;
}

/* Flux on link a -> b along half-set direction h.  Returns the total flux per
 * species in jt[] and the diffusive/migrative flux divided by D_k in gd[]. */
static void link_flux(const or_params* p, long N, const double* rho, const double* phi,
                      const double* psi, const uint8_t* flag, const double* u,
                      long a, long b, int h, double* jt, double* gd) {
    int ns = p->n_species;
    for (int k = 0; k < ns; ++k) jt[k] = gd[k] = 0.0;
    if (flag[a] || flag[b]) return;
    int sx = HALF[h][0], sy = HALF[h][1], sz = HALF[h][2];
    double len = sqrt((double)(sx * sx + sy * sy + sz * sz));
    double A0 = 1.0 + 2.0 * sqrt(2.0);
    double pa = p->partial_volume ? psi[a] : 0.0;
    double pb = p->partial_volume ? psi[b] : 0.0;
    double dphi = phi[a] - phi[b] + (p->E[0] * sx + p->E[1] * sy + p->E[2] * sz);
    double ua[3] = {u[a], u[N + a], u[2 * N + a]};
    double ub[3] = {u[b], u[N + b], u[2 * N + b]};
    double ga = adv_frac(sx, sy, sz, ua);
    double gb = adv_frac(-sx, -sy, -sz, ub);
    for (int k = 0; k < ns; ++k) {
        double ra = rho[k * N + a], rb = rho[k * N + b];
        double g = 0.0;
        if (h < 9) {
            double A = ra * (1.0 - pb) - rb * (1.0 - pa);
            double B = ra * (1.0 - pb) + rb * (1.0 - pa);
            g = (A + 0.5 * p->z[k] * B * dphi) / (A0 * len);
        }
        gd[k] = g;
        jt[k] = p->D[k] * g + (ra * ga - rb * gb);
    }
}

void or_ek_update(const or_params* p, const double* rho_in, double* rho_out,
                  const double* phi, const double* psi, const uint8_t* flag,
                  const double* u, double* fext) {
    long N = ncells(p);
    int ns = p->n_species;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < N; ++r) {
        double dr[OR_MAX_SPECIES] = {0};
        double fe[3] = {0, 0, 0};
        if (!flag[r]) {
            int x, y, z;
            cell_coords(p, r, &x, &y, &z);
            for (int h = 0; h < 13; ++h) {
                long up = cell_at(p, x + HALF[h][0], y + HALF[h][1], z + HALF[h][2]);
                long dn = cell_at(p, x - HALF[h][0], y - HALF[h][1], z - HALF[h][2]);
                double jt1[OR_MAX_SPECIES], gd1[OR_MAX_SPECIES], jt2[OR_MAX_SPECIES], gd2[OR_MAX_SPECIES];
                link_flux(p, N, rho_in, phi, psi, flag, u, r, up, h, jt1, gd1);
                link_flux(p, N, rho_in, phi, psi, flag, u, dn, r, h, jt2, gd2);
                for (int k = 0; k < ns; ++k) {
                    dr[k] += -jt1[k] + jt2[k];
                    if (h < 9)
                        for (int d = 0; d < 3; ++d)
                            fe[d] += 0.5 * p->kT * (gd1[k] + gd2[k]) * HALF[h][d];
                }
            }
        }
        for (int k = 0; k < ns; ++k) rho_out[k * N + r] = rho_in[k * N + r] + dr[k];
        for (int d = 0; d < 3; ++d) fext[d * N + r] = fe[d];
    }
}

/* ---------------------------------------------------------------------------
 * LB stream + collide (Sec. III.A, Eq. lb, the TRT operator, the Guo force term
 * and the velocity bounce-back).  The stored populations are post-collision.
 * Streaming is written in pull form: the population arriving at fluid cell r
 * along c_i comes from r - c_i; if r - c_i is a boundary cell the population
 * that left r along -c_i is reflected, plus 6 w_i rho0 c_i.v_b (Eq. velocity
 * bounce-back, with the printed 1/rho read as 1/rho0).  Then, with the
 * populations f_i that arrived:
 *   rho = sum f_i,  j = sum f_i c_i,  u = j + f/2 (reading: the half-force
 *   velocity of the Guo scheme; the paper prints u = j/rho)
 *   f_i* = f_i + le (f_i^+ - feq_i^+) + lo (f_i^- - feq_i^-) + Delta_i
 * Reading of the equilibrium (silent in the paper): second-order incompressible
 *   feq_i = w_i [rho + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u^2]   (rho0 = 1),
 * whose odd part is built with the unshifted momentum j (the collision then
 * conserves momentum and the force enters through Delta_i only, as in the MRT
 * form the paper cites).
 *   Delta_i = 3 w_i [ f.c_i + 3/2 (c_i G c_i - Tr G / 3) ],
 *   G = (2 + le)/2 (u f + f u)  (Eq. guo; 1/rho read as 1/rho0).
 * le = -1/(3 nu + 1/2).  Reading of "lambda_o = 3/16": the TRT magic parameter
 * (1/le + 1/2)(1/lo + 1/2) = 3/16, which puts the bounce-back wall half-way.
 * Boundary cells neither collide nor stream; their populations are kept and
 * their velocity output is 0.
 * ------------------------------------------------------------------------- */
void or_lb_update(const or_params* p, const or_particle* pt,
                  const double* f_in, double* f_out,
                  const uint8_t* flag, const int32_t* owner,
                  const double* fext, double* u_out) {
    long N = ncells(p);
    double tau_e = 3.0 * p->nu + 0.5;
    double le = -1.0 / tau_e;
    double tau_o = 0.5 + (3.0 / 16.0) / (tau_e - 0.5);
    double lo = -1.0 / tau_o;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < N; ++r) {
        if (flag[r]) {
            for (int i = 0; i < 19; ++i) f_out[i * N + r] = f_in[i * N + r];
            for (int d = 0; d < 3; ++d) u_out[d * N + r] = 0.0;
            continue;
        }
        int x, y, z;
        cell_coords(p, r, &x, &y, &z);
        double fi[19];
        for (int i = 0; i < 19; ++i) {
            long src = cell_at(p, x - CV[i][0], y - CV[i][1], z - CV[i][2]);
            if (flag[src]) {
                double vb[3];
                boundary_velocity(p, pt, src, owner[src], vb);
                double cv = CV[i][0] * vb[0] + CV[i][1] * vb[1] + CV[i][2] * vb[2];
                fi[i] = f_in[OPP[i] * N + r] + 6.0 * weight(i) * cv;
            } else {
                fi[i] = f_in[i * N + src];
            }
        }
        double rho = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < 19; ++i) {
            rho += fi[i];
            for (int d = 0; d < 3; ++d) j[d] += fi[i] * CV[i][d];
        }
        double fo[3] = {fext[r], fext[N + r], fext[2 * N + r]};
        double u[3];
        for (int d = 0; d < 3; ++d) u[d] = j[d] + 0.5 * fo[d];
        double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double uf = u[0] * fo[0] + u[1] * fo[1] + u[2] * fo[2];
        for (int i = 0; i < 19; ++i) {
            int o = OPP[i];
            double w = weight(i);
            double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
            double cj = CV[i][0] * j[0] + CV[i][1] * j[1] + CV[i][2] * j[2];
            double cf = CV[i][0] * fo[0] + CV[i][1] * fo[1] + CV[i][2] * fo[2];
            double feq_even = w * (rho + 4.5 * cu * cu - 1.5 * usq);
            double feq_odd = w * 3.0 * cj;
            double fplus = 0.5 * (fi[i] + fi[o]);
            double fminus = 0.5 * (fi[i] - fi[o]);
            double cGc = (2.0 + le) * cu * cf;
            double trG = (2.0 + le) * uf;
            double delta = 3.0 * w * (cf + 1.5 * (cGc - trG / 3.0));
            f_out[i * N + r] = fi[i] + le * (fplus - feq_even) + lo * (fminus - feq_odd) + delta;
        }
        for (int d = 0; d < 3; ++d) u_out[d * N + r] = u[d];
    }
}

/* ---------------------------------------------------------------------------
 * Momentum-exchange force and torque on each particle (Sec. III.B, Eq. force).
 * For every link from a fluid cell x_f to a boundary cell x_b = x_f + c_i owned
 * by particle p, the population f_i*(x_f) is reflected; the particle receives
 *   c_i (2 f_i*(x_f) - 6 w_i rho0 c_i.v_b)
 * and the torque (r_b - r_p) x (that).  Reading: this is the form of Eq. force
 * for a particle without interior fluid, written with the population that is
 * reflected; its sign makes the drag oppose the motion.
 * ------------------------------------------------------------------------- */
void or_hydro_force(const or_params* p, const or_particle* pt, int np,
                    const double* f_in, const uint8_t* flag, const int32_t* owner,
                    double* F, double* T) {
    long N = ncells(p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < np; ++k) {
        double Fk[3] = {0, 0, 0}, Tk[3] = {0, 0, 0};
        for (long b = 0; b < N; ++b) {
            if (!flag[b] || owner[b] != k) continue;
            int x, y, z;
            cell_coords(p, b, &x, &y, &z);
            double vb[3], rb[3];
            boundary_velocity(p, pt, b, k, vb);
            cell_disp(p, b, &pt[k], rb);
            for (int i = 1; i < 19; ++i) {
                long xf = cell_at(p, x - CV[i][0], y - CV[i][1], z - CV[i][2]);
                if (flag[xf]) continue;
                double cv = CV[i][0] * vb[0] + CV[i][1] * vb[1] + CV[i][2] * vb[2];
                double t = 2.0 * f_in[i * N + xf] - 6.0 * weight(i) * cv;
                double df[3] = {CV[i][0] * t, CV[i][1] * t, CV[i][2] * t};
                for (int d = 0; d < 3; ++d) Fk[d] += df[d];
                cross_add(Tk, rb, df, 1.0);
            }
        }
        for (int d = 0; d < 3; ++d) {
            F[3 * k + d] = Fk[d];
            T[3 * k + d] = Tk[d];
        }
    }
}

/* ---------------------------------------------------------------------------
 * Electrostatic force on each particle (Sec. III.C, last paragraph on
 * electrostatics): the particle's charge density in the total field,
 *   F_p = kT sum_r rho_b,p(r) (E - grad phi(r)),  T_p = kT sum_r (r - r_p) x ...
 * Reading: grad phi by central differences.
 * ------------------------------------------------------------------------- */
void or_el_force(const or_params* p, const or_particle* pt, int np,
                 const double* phi, const uint8_t* flag, const int32_t* owner,
                 double* F, double* T) {
    (void)flag;
    long N = ncells(p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < np; ++k) {
        long nb = 0;
        if (p->charge_mode == 1)
            for (long c = 0; c < N; ++c)
                if (owner[c] == k) nb++;
        double Fk[3] = {0, 0, 0}, Tk[3] = {0, 0, 0};
        for (long c = 0; c < N; ++c) {
            double d[3];
            cell_disp(p, c, &pt[k], d);
            double qb;
            if (p->charge_mode == 1) {
                if (owner[c] != k) continue;
                qb = pt[k].Z / (double)nb;
            } else {
                if (far_from(d, pt[k].R)) continue;
                int cnt = or_psi_count(d[0], d[1], d[2], pt[k].R);
                if (cnt == 0) continue;
                qb = pt[k].Z * ((double)cnt / 4096.0) / sphere_volume(pt[k].R);
            }
            int x, y, z;
            cell_coords(p, c, &x, &y, &z);
            double g[3];
            g[0] = 0.5 * (phi[cell_at(p, x + 1, y, z)] - phi[cell_at(p, x - 1, y, z)]);
            g[1] = 0.5 * (phi[cell_at(p, x, y + 1, z)] - phi[cell_at(p, x, y - 1, z)]);
            g[2] = 0.5 * (phi[cell_at(p, x, y, z + 1)] - phi[cell_at(p, x, y, z - 1)]);
            double fc[3];
            for (int e = 0; e < 3; ++e) fc[e] = p->kT * qb * (p->E[e] - g[e]);
            for (int e = 0; e < 3; ++e) Fk[e] += fc[e];
            cross_add(Tk, d, fc, 1.0);
        }
        for (int e = 0; e < 3; ++e) {
            F[3 * k + e] = Fk[e];
            T[3 * k + e] = Tk[e];
        }
    }
}

/* ---------------------------------------------------------------------------
 * Particle integration (Sec. III.B: symplectic Euler).  Both integrators are
 * written as a kick-drift before the step and an optional kick after it:
 *   symplectic Euler: v += F_prev/M, w += T_prev/I, then x += v;
 *   velocity Verlet:  v += F_prev/(2M), x += v, ..., v += F_new/(2M).
 * I = 2/5 M R^2 (solid sphere).  Prescribed particles keep v and w; fixed
 * particles do not move.  Positions are wrapped into the periodic box.
 * ------------------------------------------------------------------------- */
void or_move(const or_params* p, or_particle* pt, int np) {
    double L[3] = {(double)p->nx, (double)p->ny, (double)p->nz};
    for (int k = 0; k < np; ++k) {
        or_particle* q = &pt[k];
        if (q->mode == 2) {
            for (int d = 0; d < 3; ++d) q->v[d] = q->w[d] = 0.0;
            continue;
        }
        if (q->mode == 0) {
            double I = 0.4 * q->M * q->R * q->R;
            double a = p->integrator == 0 ? 0.5 : 1.0;
            for (int d = 0; d < 3; ++d) {
                q->v[d] += a * q->F[d] / q->M;
                q->w[d] += a * q->T[d] / I;
            }
        }
        for (int d = 0; d < 3; ++d) {
            q->x[d] += q->v[d];
            if (q->x[d] >= L[d]) q->x[d] -= L[d];
            else if (q->x[d] < 0.0) q->x[d] += L[d];
        }
    }
}

void or_finish(const or_params* p, or_particle* pt, int np,
               const double* Fnew, const double* Tnew) {
    for (int k = 0; k < np; ++k) {
        or_particle* q = &pt[k];
        if (q->mode == 0 && p->integrator == 0) {
            double I = 0.4 * q->M * q->R * q->R;
            for (int d = 0; d < 3; ++d) {
                q->v[d] += 0.5 * Fnew[3 * k + d] / q->M;
                q->w[d] += 0.5 * Tnew[3 * k + d] / I;
            }
        }
        for (int d = 0; d < 3; ++d) {
            q->F[d] = Fnew[3 * k + d];
            q->T[d] = Tnew[3 * k + d];
        }
    }
}
