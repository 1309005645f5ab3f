// ek_internal.h -- device state layout and helpers of the gfx950 library.
//
// Layout in HBM (per simulation, N = nx*ny*nz cells, x fastest; T = double on
// the FP64 path, float on the FP32 path; Np = N rounded up to a multiple of
// FB = 64 cells):
//   f[2][Np/64][19][64]  populations, ping-pong, in blocks of 64 cells that hold
//                        their 19 values contiguously (FP32: f_i - w_i)
//   rho[2][ns][N]        solute densities, ping-pong (FP32: rho_k - mean_k)
//   u[2][Np/64][3][64]   fluid velocity, double-buffered (EK reads u[cur], LB
//                        writes u[cur^1]); fext[Np/64][3][64] force density
//   phi[N], rhob[N]      potential, particle charge density (T)
//   psi[N] float         partial volume (multiples of 1/4096: exact in float)
//   flag[N] u8           bit0 boundary now, bit1 boundary before this step's
//                        move, bit2 wall
//   owner[N], owner_prev[N], psi_owner[N] u16
//   spec[ny*nz][nxs]     complex T, half spectrum, rows padded to 128-byte lines
//   FFT tables, particle records (FP64), status word, reduction scratch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>

#include "../../include/ek.h"

namespace ek {

constexpr int MAXS = EK_MAX_SPECIES;
constexpr uint16_t NO_OWNER = 0xFFFF;
constexpr uint16_t MULTI_OWNER = 0xFFFE;
constexpr uint8_t F_CUR = 1, F_PREV = 2, F_WALL = 4;
constexpr int BOX_MARGIN = 2;
constexpr int MAX_FFT = 512;
constexpr int NDIAG = MAXS + 7;       // species totals, rho_b, fluid mass, momentum(3), boundary cells, max|u|
constexpr int DIAG_BLOCKS = 1024;
constexpr int MAX_CHUNKS = 32;        // workgroups per particle box
constexpr int BOX_CELLS_PER_THREAD = 2;  // box cells per thread of a box kernel (target)
constexpr int PSTRIDE = 16;           // doubles per partial-sum record
enum { PART_BOUNDARY = 0, PART_HYDRO = 1, PART_EL = 2, PART_KINDS = 3 };

// Global-memory access through a device pointer. A pointer read from memory
// (the batched kernels take every field pointer from a table) is flat to the
// compiler, and a flat access also counts against the LDS wait counter: each
// wait for an LDS result then also waits for every global load and store in
// flight. Kernel-argument pointers are global already; the cast costs nothing.
template <typename T> using gmem = __attribute__((address_space(1))) T;
template <typename T> __device__ __forceinline__ T gld(const T* p) { return *(const gmem<T>*)p; }
template <typename T> __device__ __forceinline__ void gst(T* p, T v) { *(gmem<T>*)p = v; }
template <typename T> __device__ __forceinline__ void gst_nt(T* p, T v) { __builtin_nontemporal_store(v, (gmem<T>*)p); }

// ---------------------------------------------------------------------------
// Compile-time loops and lattice tables
// ---------------------------------------------------------------------------
template <typename F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// D3Q19: rest; +-x, +-y, +-z; 12 edges as opposite pairs.
constexpr int q19x(int i) {
    constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[i];
}
constexpr int q19y(int i) {
    constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[i];
}
constexpr int q19z(int i) {
    constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[i];
}
constexpr int q19opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
constexpr double q19w(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Half of the 26-neighbourhood: 9 D3Q19 links first, then the 4 body diagonals.
constexpr int hx(int h) {
    constexpr int t[13] = {1, 0, 0, 1, 1, 1, 1, 0, 0, 1, 1, 1, 1};
    return t[h];
}
constexpr int hy(int h) {
    constexpr int t[13] = {0, 1, 0, 1, -1, 0, 0, 1, 1, 1, 1, -1, -1};
    return t[h];
}
constexpr int hz(int h) {
    constexpr int t[13] = {0, 0, 1, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
    return t[h];
}
constexpr double hlen(int h) {
    return h < 3 ? 1.0 : (h < 9 ? 1.4142135623730950488 : 1.7320508075688772935);
}

// ---------------------------------------------------------------------------
// Particle record (always FP64; small)
// ---------------------------------------------------------------------------
struct PState {
    double x[3], v[3], w[3];
    double R, Z, M, I, Vp;
    double F[3], T[3];     // total of the last completed step (carried to the next kick)
    double Fh[3], Th[3];   // momentum exchange (this step)
    double Fe[3], Te[3];   // electrostatic (this step)
    double Fc[3], Tc[3];   // fluid destroyed / created (this step)
    double disp[3];        // displacement of this step's move
    double pool[MAXS];     // solute of covered cells with no stable-fluid neighbour
    int box_lo[3], box_n[3];
    int mode, nb;          // nb: cells owned (claimed boundary cells)
    int ncov, nvac, npool, nflag;  // event counts of this step; nflag: box cells flagged now or before
};

// Everything a kernel needs about one simulation (passed by value).
template <typename T>
struct Sim {
    int nx, ny, nz, nxh;
    int nxs;                  // row stride of the half spectrum (nxh rounded up to 128-byte lines)
    long N, Nspec;
    int ns, np;
    int pv, charge_mode, integrator;
    int cur;                  // ping-pong index of f and rho holding the current state
    double kT, lambda_B, E[3];
    double D[MAXS], z[MAXS], rho_ref[MAXS];
    T lam_e, lam_o;
    long n_wall;              // number of wall cells
    T* f[2];
    T* rho[2];
    T* u[2];                  // velocity read by EK this step (u[cur]) / written by LB (u[cur^1])
    T* fext;
    T* phi;
    T* rhob;
    float* psi;
    uint8_t* flag;
    uint16_t* owner;
    uint16_t* owner_prev;
    uint16_t* psi_owner;
    double* wall_charge;      // nullable
    T* spec;                  // interleaved complex
    T* tw[3];                 // twiddles e^{-2 pi i m/n}, interleaved, per axis
    T* k2[3];                 // 2 - 2 cos(2 pi m / n) per axis
    PState* parts;
    uint32_t* status;         // device status word (ST_* bits), zero while the state is sound
    double* scratch;          // reductions
    double* partial;          // per-(particle, chunk) partial sums of the particle kernels
    int box_max;              // bound on cells of one particle box
    int nchunk;               // workgroups per particle box in the particle kernels
};

// ---------------------------------------------------------------------------
// Device status: bits latched by the kernels that see a velocity the method
// cannot take.  The volume-of-fluid advection intersects a cell displaced by
// u tau with its neighbours only, so every component of a fluid or particle
// velocity must stay below one cell per step; a NaN or infinity means the
// state is lost.
// ---------------------------------------------------------------------------
constexpr uint32_t ST_UNSTABLE = 1u, ST_NONFINITE = 2u;

// Status bits of a velocity (lattice units): 0 if every component is finite
// and below 1 in magnitude.
template <typename V>
__device__ __forceinline__ uint32_t velocity_status(V x, V y, V z) {
    if (fabs(x) < (V)1 && fabs(y) < (V)1 && fabs(z) < (V)1) return 0u;
    return (isfinite(x) && isfinite(y) && isfinite(z)) ? ST_UNSTABLE : ST_NONFINITE;
}

// Latch status bits (a vector-memory atomic on the simulation's status word;
// taken only on the rare path where a velocity fails the test).
__device__ __forceinline__ void latch_status(uint32_t* st, uint32_t bits) {
    __hip_atomic_fetch_or((gmem<uint32_t>*)st, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Launch geometry shared by the single-simulation and batched launches
// ---------------------------------------------------------------------------
constexpr int FFT_THREADS = 512;
constexpr int FFT_ELEMS = 8;    // pencil elements per thread of an FFT workgroup
constexpr int POOL_BLOCKS = 64;

// LDS stride of an FFT pencil of length n: room for the padded indices
// i + i/8 (i < n), rounded up to an odd number of elements.
__host__ __device__ constexpr int fft_ld(int n) { return (n + (n - 1) / 8 + 1) | 1; }
// Pencils per workgroup in the x passes (P * n <= 2048).
__host__ __device__ constexpr int fft_pencils_x(int n) {
    int P = (FFT_THREADS * FFT_ELEMS / 2) / n;
    return P < 1 ? 1 : P;
}
// Consecutive kx columns per workgroup in the y and z passes: 16 (FP32) or 8
// (FP64) for coalesced 128-byte rows, fewer for long pencils (TX * n <= 4096).
__host__ __device__ constexpr int fft_tile_kx(int n, int elem_bytes) {
    int cap = (FFT_THREADS * FFT_ELEMS) / n;
    int t = elem_bytes == 4 ? 16 : 8;
    return t < cap ? t : cap;
}
// Populations are stored in blocks of FB consecutive cells that hold their 19
// populations contiguously, f[c / FB][i][c % FB]: a wavefront's 19 pulls then
// fall into a few contiguous regions instead of 19 arrays N apart (measured on
// the D3Q19 pull pattern: +6 % streaming bandwidth).  The last block is padded.
constexpr int FB = 64;
__host__ __device__ inline long fpad(long n) { return (n + FB - 1) / FB * FB; }
__host__ __device__ __forceinline__ size_t fidx(int i, size_t c) {
    return (c / FB) * (size_t)(19 * FB) + (size_t)i * FB + (c % FB);
}

// The velocity and the force density use the same blocking for their three
// components, v[c / FB][d][c % FB].
__host__ __device__ __forceinline__ size_t vidx(int d, size_t c) {
    return (c / FB) * (size_t)(3 * FB) + (size_t)d * FB + (c % FB);
}

// Row stride of the half spectrum: nx/2 + 1 complex values rounded up to whole
// 128-byte lines, so that every column tile of the y and z passes starts on a
// line (an odd stride splits each tile row over two lines and doubles the
// traffic of those passes).
__host__ __device__ inline int spec_stride(int nx, int elem_bytes) {
    const int per_line = 128 / (2 * elem_bytes);
    const int nh = nx / 2 + 1;
    return (nh + per_line - 1) / per_line * per_line;
}
// EK tiles: TXW x TYW cells per z-plane, ZC planes per workgroup.
template <typename T> struct EKTile {
    static constexpr int TXW = 32, TYW = sizeof(T) == 4 ? 8 : 4, ZC = 16;
};

// Workgroups of each kernel for one simulation.
enum {
    KK_MOVE, KK_PART, KK_PRED, KK_POOL, KK_FFTX, KK_FFTY, KK_FFTZ, KK_EK, KK_LB, KK_N
};
template <typename T>
struct Grids {
    int n[KK_N];
    int ek_gx, ek_gy;
};
template <typename T, typename S>
inline Grids<T> grids_of(const S& s) {
    Grids<T> g;
    g.n[KK_MOVE] = (s.np + 63) / 64;
    g.n[KK_PART] = s.nchunk * s.np;
    g.n[KK_PRED] = s.np;
    g.n[KK_POOL] = s.np > 0 ? POOL_BLOCKS : 0;
    int P = fft_pencils_x(s.nx);
    g.n[KK_FFTX] = (s.ny * s.nz / 2 + P - 1) / P;
    int TXy = fft_tile_kx(s.ny, sizeof(T)), TXz = fft_tile_kx(s.nz, sizeof(T));
    g.n[KK_FFTY] = ((s.nxh + TXy - 1) / TXy) * s.nz;
    g.n[KK_FFTZ] = ((s.nxh + TXz - 1) / TXz) * s.ny;
    g.ek_gx = (s.nx + EKTile<T>::TXW - 1) / EKTile<T>::TXW;
    g.ek_gy = (s.ny + EKTile<T>::TYW - 1) / EKTile<T>::TYW;
    g.n[KK_EK] = g.ek_gx * g.ek_gy * ((s.nz + EKTile<T>::ZC - 1) / EKTile<T>::ZC);
    g.n[KK_LB] = ((s.nx * s.ny + 255) / 256) * s.nz;  // whole 256-cell chunks of each z-plane
    return g;
}

// ---------------------------------------------------------------------------
// Batched (serving) form: a table of FP32 simulations in device memory.  Each
// batched kernel covers, for its kernel kind, the concatenated workgroups of
// all slots (start = prefix sums): one workgroup per item (flat, grid = the
// total) or a resident grid that walks them.  The launch sequence is captured
// in a HIP graph and captured again when a kind's total changes.
// ---------------------------------------------------------------------------
constexpr int MAX_SLOTS = 64;
struct BatchTable {
    // Device-owned: advanced by k_batch_flip.  This block alone goes back to
    // the host after each chunk of steps (BATCH_DEV_BYTES from the start).
    int active[MAX_SLOTS];           // 1 while the slot still has steps to run
    int cur[MAX_SLOTS];              // ping-pong index of each slot (sims[i].cur)
    uint32_t status[MAX_SLOTS];      // each slot's device status word (its Sim's status points here)
    long long step[MAX_SLOTS];       // steps done
    // Host-owned: uploaded and merged (k_batch_merge) when slots come or go.
    int nsims;                       // table entries in use (active or finishing)
    int keep[MAX_SLOTS];             // in an upload: 1 keeps the slot's device-owned entries
    long long target[MAX_SLOTS];     // steps requested
    int start[KK_N][MAX_SLOTS + 1];  // workgroup prefix sums per kernel kind
    Sim<float> sims[MAX_SLOTS];
};
constexpr size_t BATCH_DEV_BYTES = offsetof(BatchTable, nsims);

// Grid of a persistent batched kernel: as many workgroups as the current
// device holds at once (every CU at the kernel's occupancy), so that all of
// them are resident and each walks the same number of work items; `fallback`
// if the occupancy query fails. A non-stream query, valid during capture.
inline int resident_grid(const void* kernel, int threads, size_t lds, int fallback) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, lds) != hipSuccess || cus < 1 || per < 1)
        return fallback;
    return cus * per;
}

// Grid of a batched launch. Flat: one workgroup per work item (`items`, the
// total over the table, which the host knows when it captures the launch,
// and captures again when it changes), scheduled by the hardware like the
// single-simulation kernels; otherwise the resident persistent grid.
inline int batch_grid(bool flat, int items, const void* kernel, int threads, size_t lds, int fallback) {
    if (flat) return items > 0 ? items : 1;
    return resident_grid(kernel, threads, lds, fallback);
}

// Slot of work item w of kind KK: the last slot whose prefix sum is <= w.
template <int KK>
__device__ __forceinline__ int batch_slot(const BatchTable* tab, int n, int w) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (tab->start[KK][mid] <= w) lo = mid;
        else hi = mid;
    }
    return lo;
}

// One work item per workgroup (flat launches: the grid is the table's total).
// No loop: a loop around the body lets the compiler keep values of every
// inlined length specialisation live across iterations (the batched FFT
// passes took 170-255 VGPRs that way, 42-70 without it).
template <int KK, typename F>
__device__ __forceinline__ void batch_one(const BatchTable* tab, F&& f) {
    const int n = tab->nsims;
    const int w = blockIdx.x;
    if (w >= tab->start[KK][n]) return;
    const int lo = batch_slot<KK>(tab, n, w);
    if (tab->active[lo]) f(tab->sims[lo], w - tab->start[KK][lo]);
}

// Persistent loop over the workgroups of kernel kind KK: f(sim, local block).
// (The launch grid and the form of the kernel must agree: batch_run picks
// both from one flag.)
template <int KK, typename F>
__device__ __forceinline__ void batch_loop(const BatchTable* tab, F&& f) {
    const int n = tab->nsims;
    const int total = tab->start[KK][n];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int lo = batch_slot<KK>(tab, n, w);
        if (tab->active[lo]) f(tab->sims[lo], w - tab->start[KK][lo]);
        __syncthreads();
    }
}

template <int KK, bool FLAT, typename F>
__device__ __forceinline__ void batch_run(const BatchTable* tab, F&& f) {
    if constexpr (FLAT) batch_one<KK>(tab, f);
    else batch_loop<KK>(tab, f);
}

// i mod n for -n <= i < 2n (one conditional correction, no division).
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Division by a workgroup-uniform divisor 1 <= d < 2^16 for dividends
// 0 <= x with x * d < 2^32: q = floor(x * ceil(2^32 / d) / 2^32) is exact
// there (the rounding error of the reciprocal, below x / 2^32, never reaches
// 1/d).
struct FDiv {
    uint32_t m;
    int d;
    __device__ __forceinline__ explicit FDiv(int d_) : m(d_ == 1 ? 0u : 0xFFFFFFFFu / (uint32_t)d_ + 1u), d(d_) {}
    __device__ __forceinline__ int div(int x) const { return d == 1 ? x : (int)__umulhi((uint32_t)x, m); }
};

// Minimum-image displacement along one axis, same operation order on every
// path that decides coverage (no contraction: see the pragma at use sites).
__device__ __forceinline__ double min_image(double centre, double x, double L) {
    double d = centre - x;
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

// ---------------------------------------------------------------------------
// Host-side launchers (defined in the .hip files)
// ---------------------------------------------------------------------------
template <typename T> void launch_move(const Sim<T>& s, hipStream_t st, int init);
template <typename T> void launch_geometry(const Sim<T>& s, hipStream_t st, int init);
template <typename T> void launch_boundary(const Sim<T>& s, hipStream_t st);
template <typename T> void launch_init_density(const Sim<T>& s, hipStream_t st);
// Seeded initial concentration, simulation units mean[k] (1 + noise (2U - 1)),
// stored as the host path stores the same values (value / fac, minus the
// reference density on the FP32 path).
struct SeedArgs {
    uint64_t seed;
    double noise, fac;
    double mean[MAXS];
};
template <typename T> void launch_seed_density(const Sim<T>& s, const SeedArgs& a, hipStream_t st);
template <typename T> void launch_charge_poisson(const Sim<T>& s, hipStream_t st);
// EK + LB update; `mid` (optional) is recorded between the EK and LB kernels,
// or after the fused kernel where they are one.
template <typename T> void launch_fields(const Sim<T>& s, hipStream_t st, hipEvent_t mid = nullptr);
template <typename T> void launch_refill(const Sim<T>& s, hipStream_t st);
template <typename T> void launch_hydro(const Sim<T>& s, hipStream_t st);
template <typename T> void launch_forces(const Sim<T>& s, hipStream_t st);
template <typename T> void fill(T* p, long n, T v, hipStream_t st);
template <typename T> void fill_pops(T* f, long npad, bool dev, hipStream_t st);
template <typename T> void launch_particle_forces(const Sim<T>& s, hipStream_t st);  // hydro + electrostatic
// closing kick; and_move: also the next step's kick and drift (inside a chain of steps)
template <typename T> void launch_finish(const Sim<T>& s, hipStream_t st, bool and_move = false);
template <typename T> void launch_diagnostics(const Sim<T>& s, hipStream_t st, double* out);
// batched step pieces (FP32 tables); items[k] = total work items of kind k
// over the table (start[k][nsims] of the table the launches will read)
// refill: launch the simple scheme's refill kernels (some live slot uses that scheme)
void launch_batch_particles_pre(const BatchTable* tab, const int* items, bool refill, hipStream_t st);
void launch_batch_poisson(const BatchTable* tab, const int* items, hipStream_t st);
void launch_batch_fields(const BatchTable* tab, const int* items, int ns, hipStream_t st);
void launch_batch_particle_forces(const BatchTable* tab, const int* items, hipStream_t st);
void launch_batch_finish(const BatchTable* tab, hipStream_t st);
void launch_batch_flip(BatchTable* tab, hipStream_t st);
void launch_batch_merge(BatchTable* tab, const BatchTable* upload, hipStream_t st);
void launch_copy16(void* dst, const void* src, long n16, hipStream_t st);

// Iterative Poisson solve with a relative permittivity field (ek_poisson_cg.hip):
// device buffers (FP64, N cells each unless stated) and controls.
struct CGState {
    int nx, ny, nz;
    long N;
    double fourpi_lb;         // 4 pi lambda_B (lattice units)
    double* x;                // solution (the previous step's: warm start), zero mean
    double* r;                // residual (holds the charge before the start)
    double* p;                // search direction
    double* q;                // L p
    double* ef[3];            // face permittivities: ef[d][c] between c and c + e_d
    double* idiag;            // 1 / diagonal of L
    double* part;             // per-workgroup partial sums [1024][4]
    double* sc;               // scalars (charge sum, r.z, r.r, b.b, alpha, beta, x sum)
    double tol;               // stop at |r| <= tol |b|
    int max_iter;
};
constexpr int CG_CHECK = 8;   // iterations between convergence checks
int cg_setup(const CGState& g, const double* eps_dev, hipStream_t st);
template <typename T> int cg_solve(const Sim<T>& s, CGState& g, hipStream_t st, int* iters, double* rel_res);

// Allocation-free step: the particle kernels' partial sums in a fixed device
// array of this many bytes per GPU (ek_noalloc.hip).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)512 << 10;
hipError_t noalloc_scratch(void** out);

}  // namespace ek
