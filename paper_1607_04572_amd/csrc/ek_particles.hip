// ek_particles.hip -- particle-local kernels: integration, coverage (flags,
// owners, partial volumes Psi, particle charge), the moving-boundary update of
// the LB fluid and the solute, momentum-exchange and electrostatic forces.
//
// Work decomposition: one workgroup (or a row of workgroups) per particle,
// looping over the particle's box: the cells within R + 2 of its old or new
// centre, which contains every cell whose coverage can change in this step.
// A cell lying in several boxes is written only by the lowest-index box that
// contains it, so every kernel here is race-free without atomics, and every
// per-particle sum is a fixed-order workgroup reduction (deterministic).
//
// Coverage decisions (inside/outside a sphere) are taken in FP64 with FMA
// contraction disabled, in the same operation order as the reference
// definition, so the boundary sets are bit-identical for identical positions.
#include "ek_internal.h"

namespace ek {

constexpr int PT = 256;  // threads per particle workgroup

// ---------------------------------------------------------------------------
// Psi: overlapped volume fraction (Sec. III.D.2), defined by recursive
// subdivision: a box entirely inside counts fully, entirely outside counts
// zero, otherwise it is split into 8, down to depth 4 (edge 1/16), where an
// undecided box counts iff its centre is inside.  Result: a count of depth-4
// sub-cells (0..4096).
//
// Every sub-box corner and leaf centre is (d - 1/2) plus a multiple of 1/32,
// which FP64 represents exactly, so the recursion's result equals exactly the
// number of the 4096 leaf centres c with fl(fl(cx^2 + cy^2) + cz^2) <= R^2:
// a box decided inside has far-corner squares that bound its leaves' squares
// (rounding is monotone), and a box decided outside has leaves whose squared
// distance exceeds its near-point bound by at least 1/1024, far beyond
// rounding.  The GPU therefore classifies the whole cell first and, for cells
// cut by the surface, counts leaf centres with 16 lanes per cell (a wavefront
// resolves four cut cells at a time).
// ---------------------------------------------------------------------------
// Level-0 classification: 4096 (inside), 0 (outside) or -1 (cut by the surface).
__device__ __forceinline__ int psi_cell_class(double lx, double ly, double lz, double R2) {
#pragma clang fp contract(off)
    double hx = lx + 1.0, hy = ly + 1.0, hz = lz + 1.0;
    double fx = (lx * lx > hx * hx) ? lx * lx : hx * hx;
    double fy = (ly * ly > hy * hy) ? ly * ly : hy * hy;
    double fz = (lz * lz > hz * hz) ? lz * lz : hz * hz;
    if ((fx + fy) + fz <= R2) return 4096;
    double nx = (lx > 0.0) ? lx : ((hx < 0.0) ? hx : 0.0);
    double ny = (ly > 0.0) ? ly : ((hy < 0.0) ? hy : 0.0);
    double nz = (lz > 0.0) ? lz : ((hz < 0.0) ? hz : 0.0);
    if ((nx * nx + ny * ny) + nz * nz >= R2) return 0;
    return -1;
}

// Ordering of the LDS accesses of one wavefront (its LDS operations are
// executed in order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Leaf-centre count of a cut cell by a group of 16 lanes (the four groups of
// a wavefront count four cells at once).  Lane j of the group takes the leaf
// columns (i, j), i = 0..15, along z.  For a column with s = fl(cx^2 + cy^2),
// leaf k counts iff fl(s + cz_k^2) <= R^2, which is monotone in cz_k^2
// (rounding is monotone): with the 16 values cz_k^2 sorted (sz, in LDS), the
// column's count is the number of sorted values that pass, found by a binary
// search of 4 probes plus a test of the largest -- the same count as 16 tests,
// in 5.  The count is an integer, so the order of the partial sums does not
// matter.  Returns the group's total in every lane of the group.
__device__ __forceinline__ int group_leaf_count(double lx, double ly, double lz, double R2, double* sz) {
#pragma clang fp contract(off)
    const int j = threadIdx.x & 15, g0 = threadIdx.x & 48;  // lane in the group, group's first lane
    const double cz = lz + (double)(2 * j + 1) * 0.03125;
    const double c2 = cz * cz;
    int rank = 0;  // position of c2 among the group's 16 values (ties by index)
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const double o = __shfl(c2, g0 + k);
        rank += (o < c2 || (o == c2 && k < j)) ? 1 : 0;
    }
    sz[rank] = c2;
    wave_lds_sync();
    const double cy = ly + (double)(2 * j + 1) * 0.03125;
    const double cy2 = cy * cy;
    const double top = sz[15];
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const double cx = lx + (double)(2 * i + 1) * 0.03125;
        const double sxy = cx * cx + cy2;
        int c = 0;
#pragma unroll
        for (int st = 8; st >= 1; st >>= 1) c += (sxy + sz[c + st - 1] <= R2) ? st : 0;
        c += (sxy + top <= R2) ? 1 : 0;  // all 16 (the probes stop at 15)
        cnt += c;
    }
    wave_lds_sync();  // every lane has read sz before the group writes it again
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    return cnt;
}

// Cooperative Psi count: every lane of the wavefront calls this together; a
// lane with need == true receives the count of its cell (lx, ly, lz = cell
// corner relative to the sphere centre).  Pending cells are taken four at a
// time, one per 16-lane group.  Blocks of PT threads.
__device__ __forceinline__ int wave_psi_resolve(bool need, double lx, double ly, double lz, double R2, int mine) {
    __shared__ double psz[PT / 16][16];  // sorted leaf-layer squares of each group's cell
    unsigned long long mask = __ballot(need);
    const int lane = threadIdx.x & 63, g = lane >> 4;
    double* sz = psz[threadIdx.x >> 4];
    while (mask) {
        int src[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            src[q] = mask ? __ffsll((long long)mask) - 1 : -1;
            mask = mask ? mask & (mask - 1) : mask;
        }
        const int l = g == 0 ? src[0] : (g == 1 ? src[1] : (g == 2 ? src[2] : src[3]));
        const int ls = l < 0 ? lane : l;  // groups without a cell count their own (discarded)
        const double bx = __shfl(lx, ls), by = __shfl(ly, ls), bz = __shfl(lz, ls), br = __shfl(R2, ls);
        const int c = group_leaf_count(bx, by, bz, br, sz);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int cq = __shfl(c, 16 * q);
            if (src[q] == lane) mine = cq;
        }
    }
    return mine;
}

__device__ __forceinline__ bool centre_inside(double dx, double dy, double dz, double R) {
#pragma clang fp contract(off)
    double d2 = (dx * dx + dy * dy) + dz * dz;
    return d2 <= R * R;
}

__device__ __forceinline__ bool far_from(double dx, double dy, double dz, double R) {
    return fabs(dx) > R + 1.0 || fabs(dy) > R + 1.0 || fabs(dz) > R + 1.0;
}

// x - box_lo lies in (-n, 2n) because 0 <= x < n and -n < box_lo < n.
__device__ __forceinline__ int box_off(int x, int lo, int n) {
    int d = x - lo;
    d = d < 0 ? d + n : d;
    return d >= n ? d - n : d;
}

__device__ __forceinline__ bool in_box(const int (&lo)[3], const int (&bn)[3], int x, int y, int z, int nx, int ny,
                                       int nz) {
    return box_off(x, lo[0], nx) < bn[0] && box_off(y, lo[1], ny) < bn[1] && box_off(z, lo[2], nz) < bn[2];
}
__device__ __forceinline__ bool in_box(const PState& q, int x, int y, int z, int nx, int ny, int nz) {
    return in_box(q.box_lo, q.box_n, x, y, z, nx, ny, nz);
}

// Circular index ranges [a, a + na) and [b, b + nb) modulo n intersect
// (-n < a, b < n).
__device__ __forceinline__ bool arcs_meet(int a, int na, int b, int nb, int n) {
    int ba = b - a, ab = a - b;  // in (-2n, 2n)
    ba = ba < 0 ? ba + n : ba;
    ba = ba < 0 ? ba + n : (ba >= n ? ba - n : ba);
    ab = ab < 0 ? ab + n : ab;
    ab = ab < 0 ? ab + n : (ab >= n ? ab - n : ab);
    return ba < na || ab < nb;
}

template <typename T>
__device__ __forceinline__ void cell_disp(const Sim<T>& s, int x, int y, int z, const double (&xc)[3], double d[3]) {
#pragma clang fp contract(off)
    d[0] = min_image((double)x + 0.5, xc[0], (double)s.nx);
    d[1] = min_image((double)y + 0.5, xc[1], (double)s.ny);
    d[2] = min_image((double)z + 0.5, xc[2], (double)s.nz);
}

// The fields of one particle a box kernel uses, loaded once into registers.
struct PLocal {
    double x[3], v[3], w[3], R, Z, Vp;
    int lo[3], bn[3], nb, ncell;
    __device__ __forceinline__ explicit PLocal(const PState& q) {
        for (int d = 0; d < 3; ++d) {
            x[d] = q.x[d];
            v[d] = q.v[d];
            w[d] = q.w[d];
            lo[d] = q.box_lo[d];
            bn[d] = q.box_n[d];
        }
        R = q.R;
        Z = q.Z;
        Vp = q.Vp;
        nb = q.nb;
        ncell = bn[0] * bn[1] * bn[2];
    }
};

// Box cell t (0 <= t < ncell) -> global coordinates; the divisions by the
// box extents use multiply-high where the operands allow it.
struct BoxWalk {
    int lo[3], bn[3], n01;
    bool fast;
    FDiv d0, d01;
    __device__ __forceinline__ explicit BoxWalk(const PLocal& q)
        : lo{q.lo[0], q.lo[1], q.lo[2]}, bn{q.bn[0], q.bn[1], q.bn[2]}, n01(q.bn[0] * q.bn[1]),
          fast((unsigned long long)q.ncell * (unsigned long long)n01 < (1ull << 32) && n01 < (1 << 16)),
          d0(q.bn[0]), d01(q.bn[0] * q.bn[1] < (1 << 16) ? q.bn[0] * q.bn[1] : 1) {}
    template <typename T>
    __device__ __forceinline__ void cell(const Sim<T>& s, int t, int& x, int& y, int& z) const {
        int q0, k;
        if (fast) {
            q0 = d0.div(t);
            k = d01.div(t);
        } else {
            q0 = t / bn[0];
            k = t / n01;
        }
        const int i = t - q0 * bn[0], j = q0 - k * bn[1];
        x = wrap1(lo[0] + i, s.nx);  // lo + i in (-n, 2n)
        y = wrap1(lo[1] + j, s.ny);
        z = wrap1(lo[2] + k, s.nz);
    }
};

// Linear index of (x, y, z) with each coordinate in [-n, 2n) (the cells of a
// box and their neighbours up to distance 2).
template <typename T>
__device__ __forceinline__ long cidx(const Sim<T>& s, int x, int y, int z) {
    return (long)wrap1(x, s.nx) + (long)s.nx * ((long)wrap1(y, s.ny) + (long)s.ny * wrap1(z, s.nz));
}

// ---------------------------------------------------------------------------
// Neighbour list of a particle's box: the particles (in increasing index,
// itself included) whose boxes intersect it, with the fields the coverage and
// ownership tests need, staged in LDS once per workgroup.  Only these can
// cover a cell of the box or own it first, so every per-cell loop over
// particles runs over this list; the result is identical to a loop over all
// particles because the others contribute nothing.  Lists longer than the
// capacity fall back to reading every particle from global memory.
// ---------------------------------------------------------------------------
constexpr int NBR_CAP = 128;
struct NbrRec {
    double x[3], R, Z, Vp;  // centre, radius, valency, volume
    int lo[3], bn[3];
};
struct NbrList {
    int n;  // entries; > NBR_CAP: overflow
    int idx[NBR_CAP];
    NbrRec rec[NBR_CAP];
};

template <typename T>
__device__ __forceinline__ void build_nbrs(const Sim<T>& s, const PLocal& me, NbrList& L) {
    __shared__ int wsum[PT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int total = 0;
    for (int base = 0; base < s.np; base += PT) {
        const int k = base + threadIdx.x;
        bool hit = false;
        if (k < s.np) {
            const PState& q = s.parts[k];
            hit = arcs_meet(me.lo[0], me.bn[0], q.box_lo[0], q.box_n[0], s.nx) &&
                  arcs_meet(me.lo[1], me.bn[1], q.box_lo[1], q.box_n[1], s.ny) &&
                  arcs_meet(me.lo[2], me.bn[2], q.box_lo[2], q.box_n[2], s.nz);
        }
        const unsigned long long m = __ballot(hit);
        if (lane == 0) wsum[wave] = __popcll(m);
        __syncthreads();
        int off = total, tot = 0;
        for (int w = 0; w < PT / 64; ++w) {
            off += w < wave ? wsum[w] : 0;
            tot += wsum[w];
        }
        if (hit) {
            const int pos = off + __popcll(m & ((1ull << lane) - 1ull));
            if (pos < NBR_CAP) L.idx[pos] = k;
        }
        total += tot;
        __syncthreads();
    }
    if (total <= NBR_CAP) {
        for (int j = threadIdx.x; j < total; j += PT) {
            const PState& q = s.parts[L.idx[j]];
            NbrRec r;
            for (int d = 0; d < 3; ++d) {
                r.x[d] = q.x[d];
                r.lo[d] = q.box_lo[d];
                r.bn[d] = q.box_n[d];
            }
            r.R = q.R;
            r.Z = q.Z;
            r.Vp = q.Vp;
            L.rec[j] = r;
        }
    }
    if (threadIdx.x == 0) L.n = total;
    __syncthreads();
}

// Entries of the list (all particles on overflow).
__device__ __forceinline__ int nbr_count(const NbrList& L, int np) { return L.n > NBR_CAP ? np : L.n; }
template <typename T>
__device__ __forceinline__ int nbr_index(const Sim<T>& s, const NbrList& L, int j) {
    return L.n > NBR_CAP ? j : L.idx[j];
}
template <typename T>
__device__ __forceinline__ NbrRec nbr_rec(const Sim<T>& s, const NbrList& L, int j) {
    if (L.n <= NBR_CAP) return L.rec[j];
    const PState& q = s.parts[j];
    NbrRec r;
    for (int d = 0; d < 3; ++d) {
        r.x[d] = q.x[d];
        r.lo[d] = q.box_lo[d];
        r.bn[d] = q.box_n[d];
    }
    r.R = q.R;
    r.Z = q.Z;
    r.Vp = q.Vp;
    return r;
}

// Is p the lowest-index particle whose box contains (x, y, z)?  (The cell is
// in p's box.)
template <typename T>
__device__ __forceinline__ bool box_owner_is(const Sim<T>& s, const NbrList& L, int p, int x, int y, int z) {
    const int n = nbr_count(L, s.np);
    for (int j = 0; j < n; ++j) {
        const int k = nbr_index(s, L, j);
        if (k >= p) break;
        if (L.n <= NBR_CAP) {
            if (in_box(L.rec[j].lo, L.rec[j].bn, x, y, z, s.nx, s.ny, s.nz)) return false;
        } else if (in_box(s.parts[k], x, y, z, s.nx, s.ny, s.nz)) {
            return false;
        }
    }
    return true;
}

__device__ __forceinline__ bool stable(uint8_t fl) { return !(fl & (F_CUR | F_PREV | F_WALL)); }
__device__ __forceinline__ bool covered(uint8_t fl) { return (fl & F_CUR) && !(fl & (F_PREV | F_WALL)); }
__device__ __forceinline__ bool vacated(uint8_t fl) { return (fl & F_PREV) && !(fl & (F_CUR | F_WALL)); }

// Deterministic workgroup sum of NV doubles (result valid in thread 0).
template <int NV>
__device__ void block_sum(double (&v)[NV]) {
    __shared__ double part[NV][PT / 64];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) part[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double x = 0.0;
            for (int w = 0; w < PT / 64; ++w) x += part[k][w];
            v[k] = x;
        }
    }
    __syncthreads();
}

// Partial-sum record of (kind, particle p, chunk).
template <typename T>
__device__ __forceinline__ double* partial_rec(const Sim<T>& s, int kind, int p, int chunk) {
    return s.partial + (((long)kind * s.np + p) * s.nchunk + chunk) * PSTRIDE;
}

// ---------------------------------------------------------------------------
// Particle move (Sec. III.B) and box of this step.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void move_particle(const Sim<T>& s, int p, int init) {
#pragma clang fp contract(off)
    PState& q = s.parts[p];
    double L[3] = {(double)s.nx, (double)s.ny, (double)s.nz};
    double xold[3] = {q.x[0], q.x[1], q.x[2]};
    double disp[3] = {0.0, 0.0, 0.0};
    if (!init) {
        if (q.mode == EK_FIXED) {
            for (int d = 0; d < 3; ++d) q.v[d] = q.w[d] = 0.0;
        } else {
            if (q.mode == EK_FREE) {
                double I = 0.4 * q.M * q.R * q.R;
                double a = s.integrator == EK_VELOCITY_VERLET ? 0.5 : 1.0;
                for (int d = 0; d < 3; ++d) {
                    q.v[d] += a * q.F[d] / q.M;
                    q.w[d] += a * q.T[d] / I;
                }
                if (const uint32_t bad = velocity_status(q.v[0], q.v[1], q.v[2])) {
                    // one cell per step or more, or not finite: the error is latched and
                    // the sphere stays where it is, so that its box stays in the lattice
                    latch_status(s.status, bad);
                    for (int d = 0; d < 3; ++d) q.v[d] = q.w[d] = 0.0;
                }
            }
            for (int d = 0; d < 3; ++d) {
                disp[d] = q.v[d];
                q.x[d] += q.v[d];
                if (q.x[d] >= L[d]) q.x[d] -= L[d];
                else if (q.x[d] < 0.0) q.x[d] += L[d];
            }
        }
    }
    int n[3] = {s.nx, s.ny, s.nz};
    for (int d = 0; d < 3; ++d) {
        double lo = fmin(xold[d], xold[d] + disp[d]), hi = fmax(xold[d], xold[d] + disp[d]);
        int ilo = (int)floor(lo - q.R) - BOX_MARGIN;
        int ihi = (int)floor(hi + q.R) + BOX_MARGIN;
        int cnt = ihi - ilo + 1;
        if (cnt >= n[d]) {
            ilo = 0;
            cnt = n[d];
        }
        q.box_lo[d] = ilo;
        q.box_n[d] = cnt;
        q.disp[d] = disp[d];
        q.Fc[d] = q.Tc[d] = 0.0;
    }
    for (int k = 0; k < MAXS; ++k) q.pool[k] = 0.0;
    q.ncov = q.nvac = q.npool = q.nflag = 0;
}

template <typename T>
__device__ __forceinline__ void move_body(const Sim<T>& s, int bx_, int by_, int gx_, int init) {
    const int p = bx_ * blockDim.x + threadIdx.x;
    if (p < s.np) move_particle(s, p, init);
}

template <typename T>
__global__ void k_move(Sim<T> s, int init) {
    move_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x, init);
}

// ---------------------------------------------------------------------------
// Coverage of the cells of each box: flag (claimed: centre inside in the simple
// scheme, Fig. 1; completely inside, Psi_p = 1, with partial volumes), owner
// (lowest claiming particle index), Psi = min(1, sum_p Psi_p), particle charge rho_b
// (Psi mode: sum_p Z_p Psi_p / V_p) plus wall charge.  The previous flag and
// owner are kept in bit1 / owner_prev for the moving-boundary update.  The
// loops are wavefront-uniform so that cut cells can be resolved cooperatively.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void geometry_body(const Sim<T>& s, int bx_, int by_, int gx_, int init) {
#pragma clang fp contract(off)
    const int p = by_;
    const PLocal me(s.parts[p]);
    const BoxWalk bw(me);
    __shared__ NbrList L;
    build_nbrs(s, me, L);
    const int nn = nbr_count(L, s.np);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // The lanes of a wavefront take box cells Wn apart (Wn = wavefronts per
    // particle), so that every wavefront samples the whole box: cut cells, each
    // resolved by a whole wavefront in turn, are then spread evenly over the
    // wavefronts instead of piling up in those whose cells lie on the surface.
    const int G = gx_ * PT, Wn = G / 64, wg = bx_ * (PT / 64) + wave;
    // The cell of the next round and its flag and owner are loaded before this
    // round's stores (a cell is read and written only by the thread of its
    // owning box, so the loads cannot see those stores), so that they do not
    // wait behind them in the in-order memory counter.
    struct Next {
        int x, y, z;
        bool active;
        long c;
        uint8_t flag;
        uint16_t owner;
    };
    auto fetch = [&](int base) {
        Next n{0, 0, 0, false, 0, 0, NO_OWNER};
        const int t = base + lane * Wn + wg;
        n.active = t < me.ncell;
        if (n.active) {
            bw.cell(s, t, n.x, n.y, n.z);
            n.active = box_owner_is(s, L, p, n.x, n.y, n.z);
        }
        if (n.active) {
            n.c = cidx(s, n.x, n.y, n.z);
            n.flag = s.flag[n.c];
            n.owner = s.owner[n.c];
        }
        return n;
    };
    Next nxt = fetch(0);
    for (int base = 0; base < me.ncell; base += G) {
        const Next here = nxt;
        if (base + G < me.ncell) nxt = fetch(base + G);
        const int x = here.x, y = here.y, z = here.z;
        const bool active = here.active;
        const long c = here.c;
        const uint8_t old = here.flag;
        uint8_t wall = old & F_WALL;
        int cur = wall ? 1 : 0;
        uint16_t ow = NO_OWNER, pso = NO_OWNER;
        double psum = 0.0;
        double qb = (active && s.wall_charge) ? s.wall_charge[c] : 0.0;
        for (int j = 0; j < nn; ++j) {
            const int k = nbr_index(s, L, j);
            const NbrRec q = nbr_rec(s, L, j);
            bool touch = active && in_box(q.lo, q.bn, x, y, z, s.nx, s.ny, s.nz);
            double d[3] = {0.0, 0.0, 0.0};
            if (touch) {
                cell_disp(s, x, y, z, q.x, d);
                touch = !far_from(d[0], d[1], d[2], q.R);
            }
            double R2 = q.R * q.R;
            double lx = d[0] - 0.5, ly = d[1] - 0.5, lz = d[2] - 0.5;
            int cnt = touch ? psi_cell_class(lx, ly, lz, R2) : 0;
            // a particle claims a cell when its centre is inside (simple scheme,
            // Fig. 1) or, with partial volumes, when the cell is completely inside
            // (Psi_p = 1, Sec. III.D.2): then a claimed cell holds almost no
            // solute and a vacated one starts empty
            if (!s.pv && touch && !cur && centre_inside(d[0], d[1], d[2], q.R)) {
                cur = 1;
                ow = (uint16_t)k;
            }
            cnt = wave_psi_resolve(touch && cnt < 0, lx, ly, lz, R2, cnt);
            if (s.pv && touch && !cur && cnt == 4096) {
                cur = 1;
                ow = (uint16_t)k;
            }
            if (touch && cnt > 0) {
                psum += (double)cnt / 4096.0;
                pso = (pso == NO_OWNER) ? (uint16_t)k : MULTI_OWNER;
                if (s.charge_mode == EK_CHARGE_PSI) qb += q.Z * ((double)cnt / 4096.0) / q.Vp;
            }
        }
        if (!active) continue;
        uint8_t prev = init ? (uint8_t)cur : (uint8_t)(old & F_CUR);
        s.flag[c] = (uint8_t)(wall | (cur ? F_CUR : 0) | (prev ? F_PREV : 0));
        s.owner_prev[c] = init ? ow : here.owner;
        s.owner[c] = ow;
        s.psi_owner[c] = pso;
        s.psi[c] = (float)(psum < 1.0 ? psum : 1.0);
        s.rhob[c] = (T)qb;
    }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_geometry(Sim<T> s, int init) {
    geometry_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x, init);
}

template <typename T>
__device__ __forceinline__ double pop_abs(const Sim<T>& s, const T* f, int i, long c, double wi) {
    return sizeof(T) == 4 ? wi + (double)f[fidx(i, c)] : (double)f[fidx(i, c)];
}

template <typename T>
__device__ __forceinline__ double rho_abs(const Sim<T>& s, const T* r, int k, long c) {
    return sizeof(T) == 4 ? s.rho_ref[k] + (double)r[(long)k * s.N + c] : (double)r[(long)k * s.N + c];
}

// ---------------------------------------------------------------------------
// LB moving boundaries (Sec. III.B, after Aidun): the fluid of a covered cell
// is destroyed and its momentum p_f goes to the particle (force p_f/tau,
// applied at the cell centre); a vacated cell is filled with the equilibrium
// at the surface velocity and the mean density of its stable-fluid D3Q19
// neighbours (1 if none), and its momentum is taken from the particle.
// Also counts the particle's boundary cells (n_b), collects the solute of
// covered cells that have no stable-fluid neighbour at all (global pool), and
// performs the solute expel for the stable cells of the box (expel_cell).
// Can a cell have a newly covered neighbour?  A covered cell is claimed by a
// particle q, so its centre lies within R_q of q's centre, and a neighbour's
// centre within R_q + sqrt 3; q's box then meets this box, so q is on the
// list.  Cells farther than R_q + 2 from every listed centre skip the load of
// their 26 neighbour flags (most of a box).
template <typename T>
__device__ __forceinline__ bool near_a_surface(const Sim<T>& s, const NbrList& L, int x, int y, int z) {
    const int n = nbr_count(L, s.np);
    for (int j = 0; j < n; ++j) {
        const NbrRec q = nbr_rec(s, L, j);
        double d[3];
        cell_disp(s, x, y, z, q.x, d);
        const double rr = q.R + 2.0;
        if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= rr * rr) return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void boundary_body(const Sim<T>& s, int bx_, int by_, int gx_) {
#pragma clang fp contract(off)
    const int p = by_;
    const PLocal me(s.parts[p]);
    const BoxWalk bw(me);
    __shared__ NbrList L;
    build_nbrs(s, me, L);
    T* f = s.f[s.cur];
    const T* rho = s.rho[s.cur];
    // 0-2 Fc, 3-5 Tc, 6..6+MAXS pool, then counts
    double acc[6 + MAXS + 5];
    for (int k = 0; k < 6 + MAXS + 5; ++k) acc[k] = 0.0;
    // the next cell's flag and owner (which this kernel does not write) are
    // loaded before this cell's dependent loads
    struct Next {
        int x, y, z;
        long c;
        uint8_t flag;
        uint16_t owner;
    };
    auto fetch = [&](int t) {
        Next n;
        bw.cell(s, t, n.x, n.y, n.z);
        n.c = cidx(s, n.x, n.y, n.z);
        n.flag = s.flag[n.c];
        n.owner = s.owner[n.c];
        return n;
    };
    const int step = s.nchunk * PT;
    Next nxt{};
    if (bx_ * PT + (int)threadIdx.x < me.ncell) nxt = fetch(bx_ * PT + threadIdx.x);
    for (int t = bx_ * PT + threadIdx.x; t < me.ncell; t += step) {
        const Next here = nxt;
        if (t + step < me.ncell) nxt = fetch(t + step);
        const int x = here.x, y = here.y, z = here.z;
        const long c = here.c;
        const uint8_t fl = here.flag;
        const uint16_t own = here.owner;
        if ((fl & F_CUR) && own == p) acc[6 + MAXS + 3] += 1.0;  // n_b
        if ((fl & (F_CUR | F_PREV)) && !(fl & F_WALL) && box_owner_is(s, L, p, x, y, z)) acc[6 + MAXS + 4] += 1.0;
        if (stable(fl) && box_owner_is(s, L, p, x, y, z) && near_a_surface(s, L, x, y, z))
            expel_cell(s, s.rho[s.cur], x, y, z, c);
        if (covered(fl) && own == p) {
            double pf[3] = {0.0, 0.0, 0.0};
            sfor<19>([&](auto I) {
                constexpr int i = I;
                double fi = pop_abs(s, f, i, c, q19w(i));
                pf[0] += fi * q19x(i);
                pf[1] += fi * q19y(i);
                pf[2] += fi * q19z(i);
            });
            double r[3];
            cell_disp(s, x, y, z, me.x, r);
            acc[0] += pf[0];
            acc[1] += pf[1];
            acc[2] += pf[2];
            acc[3] += r[1] * pf[2] - r[2] * pf[1];
            acc[4] += r[2] * pf[0] - r[0] * pf[2];
            acc[5] += r[0] * pf[1] - r[1] * pf[0];
            acc[6 + MAXS] += 1.0;
            int n27 = 0;
            for (int a = -1; a <= 1; ++a)
                for (int b = -1; b <= 1; ++b)
                    for (int e = -1; e <= 1; ++e)
                        if ((a | b | e) && stable(s.flag[cidx(s, x + a, y + b, z + e)])) n27++;
            if (n27 == 0) {
                acc[6 + MAXS + 2] += 1.0;
                for (int k = 0; k < s.ns; ++k) acc[6 + k] += rho_abs(s, rho, k, c);
            }
        }
        if (vacated(fl) && s.owner_prev[c] == p) {
            double sum = 0.0;
            int nf = 0;
            sfor<19>([&](auto I) {
                constexpr int i = I;
                if constexpr (i > 0) {
                    long n = cidx(s, x + q19x(i), y + q19y(i), z + q19z(i));
                    if (stable(s.flag[n])) {
                        double rn = 0.0;
                        // density of the neighbour (as a deviation from 1 on the FP32 path)
                        sfor<19>([&](auto J) { rn += (double)f[fidx(J, n)]; });
                        sum += rn;
                        nf++;
                    }
                }
            });
            double base = sizeof(T) == 4 ? 0.0 : 1.0;  // stored density of "no neighbour": 1
            double rbar = nf > 0 ? sum / nf : base;
            double r[3];
            cell_disp(s, x, y, z, me.x, r);
            double vb[3] = {me.v[0] + (me.w[1] * r[2] - me.w[2] * r[1]),
                            me.v[1] + (me.w[2] * r[0] - me.w[0] * r[2]),
                            me.v[2] + (me.w[0] * r[1] - me.w[1] * r[0])};
            double usq = vb[0] * vb[0] + vb[1] * vb[1] + vb[2] * vb[2];
            double pf[3] = {0.0, 0.0, 0.0};
            sfor<19>([&](auto I) {
                constexpr int i = I;
                constexpr double w = q19w(i);
                double cu = q19x(i) * vb[0] + q19y(i) * vb[1] + q19z(i) * vb[2];
                double feq = w * (rbar + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                T st = (T)feq;
                f[fidx(i, c)] = st;
                double back = (double)st;
                pf[0] += back * q19x(i);
                pf[1] += back * q19y(i);
                pf[2] += back * q19z(i);
            });
            acc[0] -= pf[0];
            acc[1] -= pf[1];
            acc[2] -= pf[2];
            acc[3] -= r[1] * pf[2] - r[2] * pf[1];
            acc[4] -= r[2] * pf[0] - r[0] * pf[2];
            acc[5] -= r[0] * pf[1] - r[1] * pf[0];
            acc[6 + MAXS + 1] += 1.0;
        }
    }
    block_sum(acc);
    if (threadIdx.x == 0) {
        double* out = partial_rec(s, PART_BOUNDARY, p, bx_);
        for (int k = 0; k < 6 + MAXS + 5; ++k) out[k] = acc[k];
    }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_boundary(Sim<T> s) {
    boundary_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

// ---------------------------------------------------------------------------
// Solute expel (Sec. III.D.1), gather form in FP64: every stable-fluid cell n
// collects, from each covered neighbour c, rho(c)/n19(c) if it is one of c's
// n19 stable D3Q19 neighbours; if c has no such neighbour, rho(c)/n27(c) from
// the D3Q27 neighbourhood.  Covered cells are emptied afterwards (boundary
// post).  Runs inside the boundary kernel: it reads flags and the densities of
// covered cells and writes those of stable cells, none of which the boundary
// work there writes or reads.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void expel_cell(const Sim<T>& s, T* rho, int x, int y, int z, long n) {
    // The 26 neighbour flags are loaded together first: almost every stable
    // cell has no covered neighbour and is done after one round of loads.
    const long ox[3] = {wrap1(x - 1, s.nx), x, wrap1(x + 1, s.nx)};
    const long oy[3] = {(long)s.nx * wrap1(y - 1, s.ny), (long)s.nx * y, (long)s.nx * wrap1(y + 1, s.ny)};
    const long nxy = (long)s.nx * s.ny;
    const long oz[3] = {nxy * wrap1(z - 1, s.nz), nxy * z, nxy * wrap1(z + 1, s.nz)};
    uint8_t nf[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) nf[q] = q == 13 ? 0 : s.flag[ox[q % 3] + oy[(q / 3) % 3] + oz[q / 9]];
    unsigned int cov = 0;
#pragma unroll
    for (int q = 0; q < 27; ++q) cov |= covered(nf[q]) ? 1u << q : 0u;
    if (!cov) return;
    double gain[MAXS] = {0.0, 0.0, 0.0, 0.0};
    bool any = false;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int e = -1; e <= 1; ++e) {
                if (!((cov >> ((a + 1) + 3 * (b + 1) + 9 * (e + 1))) & 1u)) continue;
                long c = cidx(s, x + a, y + b, z + e);
                int cx = x + a, cy = y + b, cz = z + e;
                int n19 = 0, n27 = 0;
                for (int a2 = -1; a2 <= 1; ++a2)
                    for (int b2 = -1; b2 <= 1; ++b2)
                        for (int e2 = -1; e2 <= 1; ++e2) {
                            if (!(a2 | b2 | e2)) continue;
                            if (!stable(s.flag[cidx(s, cx + a2, cy + b2, cz + e2)])) continue;
                            n27++;
                            if (abs(a2) + abs(b2) + abs(e2) <= 2) n19++;
                        }
                bool is19 = abs(a) + abs(b) + abs(e) <= 2;
                int div = 0;
                if (n19 > 0) div = is19 ? n19 : 0;
                else if (n27 > 0) div = n27;
                if (div == 0) continue;
                any = true;
                for (int k = 0; k < s.ns; ++k) gain[k] += rho_abs(s, rho, k, c) / div;
            }
    if (!any) return;
    for (int k = 0; k < s.ns; ++k) {
        double v = rho_abs(s, rho, k, n) + gain[k];
        rho[(long)k * s.N + n] = (T)(sizeof(T) == 4 ? v - s.rho_ref[k] : v);
    }
}

// Solute of covered cells with no stable-fluid neighbour in their whole
// 26-neighbourhood is spread uniformly over all stable-fluid cells.  Exits at
// once when there is none (the usual case).
template <typename T>
__device__ __forceinline__ void pool_body(const Sim<T>& s, int bx_, int by_, int gx_) {
    // the usual case, nothing pooled, costs one flag per thread and one barrier
    bool mine = false;
    for (int q = threadIdx.x; q < s.np; q += PT) mine |= s.parts[q].npool != 0;
    if (!__syncthreads_or(mine)) return;
    double pool[MAXS] = {0.0, 0.0, 0.0, 0.0};
    long nflag = 0;
    for (int q = 0; q < s.np; ++q) {
        const PState& pq = s.parts[q];
        for (int k = 0; k < MAXS; ++k) pool[k] += pq.pool[k];
        nflag += pq.nflag;
    }
    long nS = s.N - s.n_wall - nflag;
    if (nS <= 0) return;
    T* rho = s.rho[s.cur];
    for (long c = (long)bx_ * PT + threadIdx.x; c < s.N; c += (long)gx_ * PT) {
        if (!stable(s.flag[c])) continue;
        for (int k = 0; k < s.ns; ++k) {
            double v = rho_abs(s, rho, k, c) + pool[k] / (double)nS;
            rho[(long)k * s.N + c] = (T)(sizeof(T) == 4 ? v - s.rho_ref[k] : v);
        }
    }
}

// Chunk partials of the boundary kernel -> particle record (by the first
// workgroup of each particle), summed in chunk order.  Then covered cells lose
// their solute and, in the uniform charge mode, each owned cell receives
// Z / n_b of its particle's charge (every workgroup sums n_b itself).
template <typename T>
__device__ __forceinline__ void boundary_post_body(const Sim<T>& s, int bx_, int by_, int gx_) {
    constexpr int NV = 6 + MAXS + 5;
    const int p = by_;
    __shared__ double buf[MAX_CHUNKS][NV];
    __shared__ int nb_sh;
    for (int e = threadIdx.x; e < s.nchunk * NV; e += blockDim.x)
        buf[e / NV][e % NV] = partial_rec(s, PART_BOUNDARY, p, e / NV)[e % NV];
    __syncthreads();
    const int k = threadIdx.x;
    if (k < NV && (bx_ == 0 || k == 6 + MAXS + 3)) {
        double v = 0.0;
        for (int c = 0; c < s.nchunk; ++c) v += buf[c][k];
        if (k == 6 + MAXS + 3) nb_sh = (int)v;
        if (bx_ == 0) {
            PState& q = s.parts[p];
            if (k < 3) q.Fc[k] = v;
            else if (k < 6) q.Tc[k - 3] = v;
            else if (k < 6 + MAXS) q.pool[k - 6] = v;
            else if (k == 6 + MAXS) q.ncov = (int)v;
            else if (k == 6 + MAXS + 1) q.nvac = (int)v;
            else if (k == 6 + MAXS + 2) q.npool = (int)v;
            else if (k == 6 + MAXS + 3) q.nb = (int)v;
            else q.nflag = (int)v;
        }
    }
    __syncthreads();
    const int nb = nb_sh;
    const PLocal me(s.parts[p]);
    const BoxWalk bw(me);
    T* rho = s.rho[s.cur];
    for (int t = bx_ * PT + threadIdx.x; t < me.ncell; t += gx_ * PT) {
        int x, y, z;
        bw.cell(s, t, x, y, z);
        long c = cidx(s, x, y, z);
        uint8_t fl = s.flag[c];
        if (!(fl & F_CUR) || s.owner[c] != p) continue;
        if (covered(fl))
            for (int k2 = 0; k2 < s.ns; ++k2) rho[(long)k2 * s.N + c] = (T)(sizeof(T) == 4 ? -s.rho_ref[k2] : 0.0);
        if (s.charge_mode == EK_CHARGE_UNIFORM && nb > 0) {
            double qb = (s.wall_charge ? s.wall_charge[c] : 0.0) + me.Z / (double)nb;
            s.rhob[c] = (T)qb;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_boundary_post(Sim<T> s) {
    boundary_post_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

// (Run by the last workgroup of k_boundary_post instead, behind a
// device-scope release fence in every workgroup, this cost more than its own
// launch: each such fence writes the L2 back.)
template <typename T>
__global__ __launch_bounds__(PT) void k_pool(Sim<T> s) {
    pool_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}


// Initial density rule: boundary cells empty; partial-volume fluid cells keep
// (1 - Psi) of the given concentration.  Whole grid, once.
template <typename T>
__device__ __forceinline__ void init_density_body(const Sim<T>& s, int bx_, int by_, int gx_) {
    long c = (long)bx_ * PT + threadIdx.x;
    if (c >= s.N) return;
    uint8_t fl = s.flag[c];
    double psi = s.psi[c];
    for (int k = 0; k < s.ns; ++k) {
        T* r = s.rho[s.cur] + (long)k * s.N;
        double v = rho_abs(s, s.rho[s.cur], k, c);
        if (fl & F_CUR) v = 0.0;
        else if (s.pv) v *= (1.0 - psi);
        r[c] = (T)(sizeof(T) == 4 ? v - s.rho_ref[k] : v);
    }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_init_density(Sim<T> s) {
    init_density_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

// ---------------------------------------------------------------------------
// Forces on the particles.
// Momentum exchange (Sec. III.B, Eq. force): for each link from a fluid cell
// x_f to a boundary cell x_b = x_f + c_i owned by p, the reflected population
// f_i*(x_f) transfers c_i (2 f_i* - 6 w_i rho0 c_i.v_b); torque about the centre.
// Electrostatic: F = kT sum rho_b,p (E - grad phi), central differences.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void hydro_force_body(const Sim<T>& s, int bx_, int by_, int gx_) {
#pragma clang fp contract(off)
    const int p = by_;
    const PLocal me(s.parts[p]);
    const BoxWalk bw(me);
    const T* f = s.f[s.cur];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    // the next cell's flag and owner are loaded before this cell's neighbour loads
    struct Next {
        int x, y, z;
        long b;
        uint8_t flag;
        uint16_t owner;
    };
    auto fetch = [&](int t) {
        Next n;
        bw.cell(s, t, n.x, n.y, n.z);
        n.b = cidx(s, n.x, n.y, n.z);
        n.flag = s.flag[n.b];
        n.owner = s.owner[n.b];
        return n;
    };
    const int step = s.nchunk * PT;
    Next nxt{};
    if (bx_ * PT + (int)threadIdx.x < me.ncell) nxt = fetch(bx_ * PT + threadIdx.x);
    for (int t = bx_ * PT + threadIdx.x; t < me.ncell; t += step) {
        const Next here = nxt;
        if (t + step < me.ncell) nxt = fetch(t + step);
        const int x = here.x, y = here.y, z = here.z;
        const long b = here.b;
        const uint8_t fb = here.flag;
        const uint16_t ob = here.owner;
        if (!(fb & F_CUR) || ob != p) continue;
        double r[3];
        cell_disp(s, x, y, z, me.x, r);
        double vb[3] = {me.v[0] + (me.w[1] * r[2] - me.w[2] * r[1]),
                        me.v[1] + (me.w[2] * r[0] - me.w[0] * r[2]),
                        me.v[2] + (me.w[0] * r[1] - me.w[1] * r[0])};
        // the 18 neighbour flags and populations in one round of loads; links
        // into the particle contribute exact zeros
        uint8_t nfl[19];
        T pv[19];
        sfor<19>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) {
                long xf = cidx(s, x - q19x(i), y - q19y(i), z - q19z(i));
                nfl[i] = s.flag[xf];
                pv[i] = f[fidx(i, xf)];
            }
        });
        sfor<19>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) {
                constexpr double w = q19w(i);
                double cv = q19x(i) * vb[0] + q19y(i) * vb[1] + q19z(i) * vb[2];
                double fi = sizeof(T) == 4 ? w + (double)pv[i] : (double)pv[i];
                double tt = 2.0 * fi - 6.0 * w * cv;
                tt = (nfl[i] & F_CUR) ? 0.0 : tt;
                double df[3] = {q19x(i) * tt, q19y(i) * tt, q19z(i) * tt};
                acc[0] += df[0];
                acc[1] += df[1];
                acc[2] += df[2];
                acc[3] += r[1] * df[2] - r[2] * df[1];
                acc[4] += r[2] * df[0] - r[0] * df[2];
                acc[5] += r[0] * df[1] - r[1] * df[0];
            }
        });
    }
    block_sum(acc);
    if (threadIdx.x == 0) {
        double* out = partial_rec(s, PART_HYDRO, p, bx_);
        for (int k = 0; k < 6; ++k) out[k] = acc[k];
    }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_hydro_force(Sim<T> s) {
    hydro_force_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__device__ __forceinline__ void el_force_body(const Sim<T>& s, int bx_, int by_, int gx_) {
#pragma clang fp contract(off)
    const int p = by_;
    const PLocal me(s.parts[p]);
    const BoxWalk bw(me);
    const int ncell = me.ncell;
    const double R2 = me.R * me.R;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int base = bx_ * PT; base < ncell; base += s.nchunk * PT) {
        int t = base + threadIdx.x;
        int x = 0, y = 0, z = 0;
        bool active = t < ncell;
        if (active) bw.cell(s, t, x, y, z);
        long c = active ? cidx(s, x, y, z) : 0;
        double qb = 0.0;
        bool need = false;
        double d[3] = {0.0, 0.0, 0.0};
        if (active) cell_disp(s, x, y, z, me.x, d);
        if (active && s.charge_mode == EK_CHARGE_UNIFORM) {
            const uint8_t fc = s.flag[c];
            const uint16_t oc = s.owner[c];
            if ((fc & F_CUR) && oc == p && me.nb > 0) qb = me.Z / (double)me.nb;
        } else if (active) {
            const uint16_t po = s.psi_owner[c];
            const float ps = s.psi[c];
            if (po == (uint16_t)p) qb = me.Z * (double)ps / me.Vp;
            else if (po == MULTI_OWNER && !far_from(d[0], d[1], d[2], me.R)) need = true;
        }
        // cells overlapped by several spheres: this sphere's own Psi
        double lx = d[0] - 0.5, ly = d[1] - 0.5, lz = d[2] - 0.5;
        int cnt = need ? psi_cell_class(lx, ly, lz, R2) : 0;
        cnt = wave_psi_resolve(need && cnt < 0, lx, ly, lz, R2, cnt);
        if (need && cnt > 0) qb = me.Z * ((double)cnt / 4096.0) / me.Vp;
        if (qb == 0.0) continue;
        double g[3];
        g[0] = 0.5 * ((double)s.phi[cidx(s, x + 1, y, z)] - (double)s.phi[cidx(s, x - 1, y, z)]);
        g[1] = 0.5 * ((double)s.phi[cidx(s, x, y + 1, z)] - (double)s.phi[cidx(s, x, y - 1, z)]);
        g[2] = 0.5 * ((double)s.phi[cidx(s, x, y, z + 1)] - (double)s.phi[cidx(s, x, y, z - 1)]);
        double fc[3];
        for (int e = 0; e < 3; ++e) fc[e] = s.kT * qb * (s.E[e] - g[e]);
        acc[0] += fc[0];
        acc[1] += fc[1];
        acc[2] += fc[2];
        acc[3] += d[1] * fc[2] - d[2] * fc[1];
        acc[4] += d[2] * fc[0] - d[0] * fc[2];
        acc[5] += d[0] * fc[1] - d[1] * fc[0];
    }
    block_sum(acc);
    if (threadIdx.x == 0) {
        double* out = partial_rec(s, PART_EL, p, bx_);
        for (int k = 0; k < 6; ++k) out[k] = acc[k];
    }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_el_force(Sim<T> s) {
    el_force_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

// Total force of the step and the closing half kick of velocity Verlet.  One
// workgroup per particle: lane k < 12 sums component k of the hydrodynamic and
// electrostatic chunk partials in chunk order (deterministic).
template <typename T>
__device__ __forceinline__ void finish_body(const Sim<T>& s, int bx_, int by_, int gx_, bool and_move = false) {
#pragma clang fp contract(off)
    const int p = bx_, k = threadIdx.x;
    __shared__ double sum[12];
    // all chunk partials are fetched at once, then summed in chunk order
    __shared__ double buf[MAX_CHUNKS][12];
    for (int e = threadIdx.x; e < s.nchunk * 12; e += blockDim.x) {
        const int c = e / 12, q = e % 12;
        buf[c][q] = partial_rec(s, q < 6 ? PART_HYDRO : PART_EL, p, c)[q < 6 ? q : q - 6];
    }
    __syncthreads();
    if (k < 12) {
        double v = 0.0;
        for (int c = 0; c < s.nchunk; ++c) v += buf[c][k];
        sum[k] = v;
    }
    __syncthreads();
    if (k != 0) return;
    PState& q = s.parts[p];
    for (int d = 0; d < 3; ++d) {
        q.Fh[d] = sum[d];
        q.Th[d] = sum[3 + d];
        q.Fe[d] = sum[6 + d];
        q.Te[d] = sum[9 + d];
    }
    double Fn[3], Tn[3];
    for (int d = 0; d < 3; ++d) {
        Fn[d] = (q.Fh[d] + q.Fe[d]) + q.Fc[d];
        Tn[d] = (q.Th[d] + q.Te[d]) + q.Tc[d];
    }
    if (q.mode == EK_FREE && s.integrator == EK_VELOCITY_VERLET) {
        double I = 0.4 * q.M * q.R * q.R;
        for (int d = 0; d < 3; ++d) {
            q.v[d] += 0.5 * Fn[d] / q.M;
            q.w[d] += 0.5 * Tn[d] / I;
        }
        if (const uint32_t bad = velocity_status(q.v[0], q.v[1], q.v[2])) latch_status(s.status, bad);
    }
    for (int d = 0; d < 3; ++d) {
        q.F[d] = Fn[d];
        q.T[d] = Tn[d];
    }
    // inside a chain of steps the next step's kick and drift follow at once
    if (and_move) move_particle(s, p, 0);
}

template <typename T>
__global__ void k_finish(Sim<T> s, int and_move) {
    finish_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x, and_move != 0);
}

// Momentum-exchange and electrostatic forces in one launch (after the Poisson
// solve: the first reads the populations, which nothing writes before the LB
// update; the second the potential).
template <typename T>
__global__ __launch_bounds__(PT) void k_particle_forces(Sim<T> s) {
    hydro_force_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
    el_force_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

// ---------------------------------------------------------------------------
// Simple scheme (Sec. III.D.1, Eqs. refill and refill-neighbours): a vacated
// cell v with N_f stable-fluid D3Q19 neighbours receives
// sum_n rho(n) / (N_f + 1); each such neighbour n gives rho(n) / (N_f(v) + 1)
// to every vacated neighbour v (all from the post-expel values: the first
// kernel writes only vacated cells and reads only stable ones, the second
// writes only stable cells and reads only their own values and flags).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int stable19(const Sim<T>& s, int x, int y, int z) {
    int nf = 0;
    sfor<19>([&](auto I) {
        constexpr int i = I;
        if constexpr (i > 0)
            if (stable(s.flag[cidx(s, x + q19x(i), y + q19y(i), z + q19z(i))])) nf++;
    });
    return nf;
}

template <typename T>
__device__ __forceinline__ void refill_vacated_body(const Sim<T>& s, int bx_, int by_, int gx_) {
    const int p = by_;
    const PLocal me(s.parts[p]);
    const BoxWalk bw(me);
    T* rho = s.rho[s.cur];
    for (int t = bx_ * PT + threadIdx.x; t < me.ncell; t += gx_ * PT) {
        int x, y, z;
        bw.cell(s, t, x, y, z);
        long v = cidx(s, x, y, z);
        if (!vacated(s.flag[v]) || s.owner_prev[v] != p) continue;
        int nf = stable19(s, x, y, z);
        for (int k = 0; k < s.ns; ++k) {
            double acc = rho_abs(s, rho, k, v);
            sfor<19>([&](auto I) {
                constexpr int i = I;
                if constexpr (i > 0) {
                    long n = cidx(s, x + q19x(i), y + q19y(i), z + q19z(i));
                    if (stable(s.flag[n])) acc += rho_abs(s, rho, k, n) / (nf + 1);
                }
            });
            rho[(long)k * s.N + v] = (T)(sizeof(T) == 4 ? acc - s.rho_ref[k] : acc);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_refill_vacated(Sim<T> s) {
    refill_vacated_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__device__ __forceinline__ void refill_stable_body(const Sim<T>& s, int bx_, int by_, int gx_) {
    const int p = by_;
    const PLocal me(s.parts[p]);
    const BoxWalk bw(me);
    __shared__ NbrList L;
    build_nbrs(s, me, L);
    T* rho = s.rho[s.cur];
    for (int t = bx_ * PT + threadIdx.x; t < me.ncell; t += gx_ * PT) {
        int x, y, z;
        bw.cell(s, t, x, y, z);
        long n = cidx(s, x, y, z);
        if (!stable(s.flag[n]) || !box_owner_is(s, L, p, x, y, z)) continue;
        double share = 0.0;  // sum over vacated neighbours of 1/(N_f(v)+1)
        bool any = false;
        sfor<19>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) {
                int vx = x + q19x(i), vy = y + q19y(i), vz = z + q19z(i);
                if (vacated(s.flag[cidx(s, vx, vy, vz)])) {
                    any = true;
                    share += 1.0 / (stable19(s, vx, vy, vz) + 1);
                }
            }
        });
        if (!any) continue;
        for (int k = 0; k < s.ns; ++k) {
            double r = rho_abs(s, rho, k, n);
            double loss = 0.0;
            sfor<19>([&](auto I) {
                constexpr int i = I;
                if constexpr (i > 0) {
                    int vx = x + q19x(i), vy = y + q19y(i), vz = z + q19z(i);
                    if (vacated(s.flag[cidx(s, vx, vy, vz)])) loss += r / (stable19(s, vx, vy, vz) + 1);
                }
            });
            double out = r - loss;
            rho[(long)k * s.N + n] = (T)(sizeof(T) == 4 ? out - s.rho_ref[k] : out);
        }
        (void)share;
    }
}

template <typename T>
__global__ __launch_bounds__(PT) void k_refill_stable(Sim<T> s) {
    refill_stable_body<T>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static_assert(6 + MAXS + 5 <= PSTRIDE, "partial record too small");

template <typename T>
void launch_move(const Sim<T>& s, hipStream_t st, int init) {
    if (s.np == 0) return;
    hipLaunchKernelGGL(k_move<T>, dim3((s.np + 63) / 64), dim3(64), 0, st, s, init);
}

template <typename T>
void launch_geometry(const Sim<T>& s, hipStream_t st, int init) {
    if (s.np == 0) return;
    hipLaunchKernelGGL(k_geometry<T>, dim3(s.nchunk, s.np), dim3(PT), 0, st, s, init);
}

template <typename T>
void launch_boundary(const Sim<T>& s, hipStream_t st) {
    if (s.np == 0) return;
    hipLaunchKernelGGL(k_boundary<T>, dim3(s.nchunk, s.np), dim3(PT), 0, st, s);
    hipLaunchKernelGGL(k_boundary_post<T>, dim3(s.nchunk, s.np), dim3(PT), 0, st, s);
    hipLaunchKernelGGL(k_pool<T>, dim3(POOL_BLOCKS), dim3(PT), 0, st, s);
}

template <typename T>
void launch_refill(const Sim<T>& s, hipStream_t st) {
    if (s.np == 0) return;
    hipLaunchKernelGGL(k_refill_vacated<T>, dim3(s.nchunk, s.np), dim3(PT), 0, st, s);
    hipLaunchKernelGGL(k_refill_stable<T>, dim3(s.nchunk, s.np), dim3(PT), 0, st, s);
}

template <typename T>
void launch_init_density(const Sim<T>& s, hipStream_t st) {
    hipLaunchKernelGGL(k_init_density<T>, dim3((unsigned)((s.N + PT - 1) / PT)), dim3(PT), 0, st, s);
}

template <typename T>
void launch_forces(const Sim<T>& s, hipStream_t st) {
    if (s.np == 0) return;
    hipLaunchKernelGGL(k_el_force<T>, dim3(s.nchunk, s.np), dim3(PT), 0, st, s);
}

template <typename T>
void launch_particle_forces(const Sim<T>& s, hipStream_t st) {
    if (s.np == 0) return;
    hipLaunchKernelGGL(k_particle_forces<T>, dim3(s.nchunk, s.np), dim3(PT), 0, st, s);
}

template <typename T>
void launch_hydro(const Sim<T>& s, hipStream_t st) {
    if (s.np == 0) return;
    hipLaunchKernelGGL(k_hydro_force<T>, dim3(s.nchunk, s.np), dim3(PT), 0, st, s);
}

template <typename T>
void launch_finish(const Sim<T>& s, hipStream_t st, bool and_move) {
    if (s.np == 0) return;
    hipLaunchKernelGGL(k_finish<T>, dim3(s.np), dim3(64), 0, st, s, and_move ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Batched particle kernels (one workgroup per (particle, chunk) over a BatchTable)
// ---------------------------------------------------------------------------
constexpr int BATCH_PART_BLOCKS = 1024;
constexpr int BATCH_SMALL_BLOCKS = 256;
constexpr bool FLAT_PART = true;

__global__ void kb_move(const BatchTable* __restrict__ tab) {
    batch_loop<KK_MOVE>(tab, [](const Sim<float>& s, int b) { move_body<float>(s, b, 0, 0, 0); });
}
__global__ __launch_bounds__(PT) void kb_geometry(const BatchTable* __restrict__ tab) {
    batch_run<KK_PART, FLAT_PART>(tab, [](const Sim<float>& s, int b) {
        geometry_body<float>(s, b % s.nchunk, b / s.nchunk, s.nchunk, 0);
    });
}
__global__ __launch_bounds__(PT) void kb_boundary(const BatchTable* __restrict__ tab) {
    batch_run<KK_PART, FLAT_PART>(tab, [](const Sim<float>& s, int b) {
        boundary_body<float>(s, b % s.nchunk, b / s.nchunk, s.nchunk);
    });
}
__global__ __launch_bounds__(PT) void kb_boundary_post(const BatchTable* __restrict__ tab) {
    batch_run<KK_PART, FLAT_PART>(tab, [](const Sim<float>& s, int b) {
        boundary_post_body<float>(s, b % s.nchunk, b / s.nchunk, s.nchunk);
    });
}
__global__ __launch_bounds__(PT) void kb_pool(const BatchTable* __restrict__ tab) {
    batch_run<KK_POOL, FLAT_PART>(tab, [](const Sim<float>& s, int b) { pool_body<float>(s, b, 0, POOL_BLOCKS); });
}
__global__ __launch_bounds__(PT) void kb_refill_vacated(const BatchTable* __restrict__ tab) {
    batch_run<KK_PART, FLAT_PART>(tab, [](const Sim<float>& s, int b) {
        if (!s.pv) refill_vacated_body<float>(s, b % s.nchunk, b / s.nchunk, s.nchunk);
    });
}
__global__ __launch_bounds__(PT) void kb_refill_stable(const BatchTable* __restrict__ tab) {
    batch_run<KK_PART, FLAT_PART>(tab, [](const Sim<float>& s, int b) {
        if (!s.pv) refill_stable_body<float>(s, b % s.nchunk, b / s.nchunk, s.nchunk);
    });
}
__global__ __launch_bounds__(PT) void kb_particle_forces(const BatchTable* __restrict__ tab) {
    batch_run<KK_PART, FLAT_PART>(tab, [](const Sim<float>& s, int b) {
        hydro_force_body<float>(s, b % s.nchunk, b / s.nchunk, s.nchunk);
        el_force_body<float>(s, b % s.nchunk, b / s.nchunk, s.nchunk);
    });
}
__global__ void kb_finish(const BatchTable* __restrict__ tab) {
    batch_loop<KK_PRED>(tab, [](const Sim<float>& s, int b) { finish_body<float>(s, b, 0, 0); });
}

void launch_batch_particles_pre(const BatchTable* tab, const int* items, bool refill, hipStream_t st) {
    hipLaunchKernelGGL(kb_move, dim3(BATCH_SMALL_BLOCKS), dim3(64), 0, st, tab);
    hipLaunchKernelGGL(kb_geometry, dim3(batch_grid(FLAT_PART, items[KK_PART], (const void*)kb_geometry, PT, 0, BATCH_PART_BLOCKS)), dim3(PT), 0, st, tab);
    hipLaunchKernelGGL(kb_boundary, dim3(batch_grid(FLAT_PART, items[KK_PART], (const void*)kb_boundary, PT, 0, BATCH_PART_BLOCKS)), dim3(PT), 0, st, tab);
    hipLaunchKernelGGL(kb_boundary_post, dim3(batch_grid(FLAT_PART, items[KK_PART], (const void*)kb_boundary_post, PT, 0, BATCH_PART_BLOCKS)), dim3(PT), 0, st, tab);
    hipLaunchKernelGGL(kb_pool, dim3(batch_grid(FLAT_PART, items[KK_POOL], (const void*)kb_pool, PT, 0, BATCH_PART_BLOCKS)), dim3(PT), 0, st, tab);
    if (!refill) return;
    hipLaunchKernelGGL(kb_refill_vacated, dim3(batch_grid(FLAT_PART, items[KK_PART], (const void*)kb_refill_vacated, PT, 0, BATCH_PART_BLOCKS)), dim3(PT), 0, st, tab);
    hipLaunchKernelGGL(kb_refill_stable, dim3(batch_grid(FLAT_PART, items[KK_PART], (const void*)kb_refill_stable, PT, 0, BATCH_PART_BLOCKS)), dim3(PT), 0, st, tab);
}

// after the Poisson solve and before the field update (see k_particle_forces)
void launch_batch_particle_forces(const BatchTable* tab, const int* items, hipStream_t st) {
    hipLaunchKernelGGL(kb_particle_forces, dim3(batch_grid(FLAT_PART, items[KK_PART], (const void*)kb_particle_forces, PT, 0, BATCH_PART_BLOCKS)), dim3(PT), 0, st, tab);
}

void launch_batch_finish(const BatchTable* tab, hipStream_t st) {
    hipLaunchKernelGGL(kb_finish, dim3(BATCH_SMALL_BLOCKS), dim3(64), 0, st, tab);
}

#define EK_INST(T)                                                     \
    template void launch_move<T>(const Sim<T>&, hipStream_t, int);     \
    template void launch_geometry<T>(const Sim<T>&, hipStream_t, int); \
    template void launch_boundary<T>(const Sim<T>&, hipStream_t);      \
    template void launch_init_density<T>(const Sim<T>&, hipStream_t);  \
    template void launch_refill<T>(const Sim<T>&, hipStream_t);        \
    template void launch_forces<T>(const Sim<T>&, hipStream_t);        \
    template void launch_hydro<T>(const Sim<T>&, hipStream_t);         \
    template void launch_particle_forces<T>(const Sim<T>&, hipStream_t); \
    template void launch_finish<T>(const Sim<T>&, hipStream_t, bool);
EK_INST(float)
EK_INST(double)

}  // namespace ek
