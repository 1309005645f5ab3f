// ek_api.cpp -- host side of the C ABI declared in include/ek.h: parameter
// validation, unit conversion, device memory layout, the per-step launch
// sequence (captured once per ping-pong parity into HIP graphs) and the
// host <-> device field transfers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "ek_internal.h"

using namespace ek;

namespace {

constexpr int GRAPH_CHUNK = 8;  // steps per replay of the long graph (even: parity preserved)

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool edge_ok(int n) {
    if (n < 8 || n > MAX_FFT || (n & 1)) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// Largest stable D tau / a^2 of the explicit link flux: 2 / max_k of the
// diffusive decay rate sum_i (1 - cos k.c_i) / (A0 |c_i|), reached at
// k = (0, pi, pi), where the sum is 8 + 8 sqrt 2.
double d_max() {
    const double A0 = 1.0 + 2.0 * std::sqrt(2.0);
    return 2.0 * A0 / (8.0 + 8.0 * std::sqrt(2.0));
}

struct Layout {
    size_t f, rho, u, fext, phi, rhob, psi, flag, owner, owner_prev, psi_owner, spec, tw, k2, parts, scratch,
        partial, diag, status, state_end, total;
};

Layout make_layout(const ek_params* p, size_t ts) {
    Layout L{};
    size_t N = (size_t)p->nx * p->ny * p->nz;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.f = take(2 * 19 * (size_t)fpad((long)N) * ts);
    L.rho = take(2 * (size_t)p->n_species * N * ts);
    L.u = take(2 * 3 * (size_t)fpad((long)N) * ts);
    L.fext = take(3 * (size_t)fpad((long)N) * ts);
    L.phi = take(N * ts);
    L.rhob = take(N * ts);
    L.psi = take(N * sizeof(float));
    L.flag = take(N);
    L.owner = take(N * 2);
    L.owner_prev = take(N * 2);
    L.psi_owner = take(N * 2);
    int mp = p->max_particles > 0 ? p->max_particles : 1;
    L.parts = take((size_t)mp * sizeof(PState));
    L.state_end = off;
    L.spec = take((size_t)spec_stride(p->nx, (int)ts) * p->ny * p->nz * 2 * ts);
    L.tw = take((size_t)(p->nx + p->ny + p->nz) * 2 * ts);
    L.k2 = take((size_t)(p->nx + p->ny + p->nz) * ts);
    L.scratch = take((size_t)DIAG_BLOCKS * NDIAG * sizeof(double));
    L.partial = take((size_t)PART_KINDS * mp * MAX_CHUNKS * PSTRIDE * sizeof(double));
    L.diag = take(64 * sizeof(double));
    L.status = take(sizeof(uint32_t));
    L.total = off;
    return L;
}

int validate(const ek_params* p) {
    if (!p) return EK_ERR_INVALID_ARG;
    if (!edge_ok(p->nx) || !edge_ok(p->ny) || !edge_ok(p->nz)) return EK_ERR_UNSUPPORTED_SIZE;
    if (!(p->agrid > 0) || !(p->tau > 0) || !(p->kT > 0) || !(p->fluid_density > 0)) return EK_ERR_INVALID_ARG;
    if (!std::isfinite(p->viscosity) || !std::isfinite(p->bjerrum_length) || p->bjerrum_length < 0)
        return EK_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->E_ext[d])) return EK_ERR_NONFINITE;
    if (!(p->viscosity > 0)) return EK_ERR_UNSTABLE;
    if (p->n_species < 1 || p->n_species > EK_MAX_SPECIES) return EK_ERR_INVALID_ARG;
    for (int k = 0; k < p->n_species; ++k) {
        const ek_species& s = p->species[k];
        if (!std::isfinite(s.D) || !std::isfinite(s.mean_density) || s.D < 0 || s.mean_density < 0)
            return EK_ERR_INVALID_ARG;
        double Dl = s.D * p->tau / (p->agrid * p->agrid);
        if (Dl > d_max() * (1.0 - 1e-3)) return EK_ERR_UNSTABLE;
    }
    if (p->precision != EK_FP64_PLAIN && p->precision != EK_FP32_DEV) return EK_ERR_INVALID_ARG;
    if (p->scheme != EK_SCHEME_PARTIAL_VOLUME && p->scheme != EK_SCHEME_SIMPLE) return EK_ERR_INVALID_ARG;
    if (p->charge_mode != EK_CHARGE_PSI && p->charge_mode != EK_CHARGE_UNIFORM) return EK_ERR_INVALID_ARG;
    if (p->integrator != EK_VELOCITY_VERLET && p->integrator != EK_SYMPLECTIC_EULER) return EK_ERR_INVALID_ARG;
    if (p->max_particles < 0 || p->max_particles > 1024) return EK_ERR_INVALID_ARG;
    return EK_OK;
}

}  // namespace

struct ek_ctx {
    ek_params p{};
    Layout L{};
    bool fp32 = false;
    Sim<float> sf{};
    Sim<double> sd{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    unsigned char* arena = nullptr;
    bool own_arena = false;
    double* wall_charge = nullptr;
    std::vector<PState> parts;
    bool prepared = false;
    long long step = 0;
    int err = EK_OK;
    bool use_graphs = true;
    hipGraphExec_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    // pinned copy of the device status word, refreshed after each ek_step's
    // launches, so that a later ek_step reports a latched error without waiting
    uint32_t* host_status = nullptr;
    // iterative Poisson solve with a permittivity field (null: FFT solver)
    CGState* cg = nullptr;
    void* cg_mem = nullptr;
    int cg_iters = 0;
    double cg_res = 0.0;
    bool cg_failed = false;
    // unit conversion (simulation units per lattice unit)
    double a = 1, tau = 1, rf = 1;
    long N = 0;

    int cur() const { return fp32 ? sf.cur : sd.cur; }
    void set_cur(int c) {
        sf.cur = c;
        sd.cur = c;
    }
};

#define HIPCHK(c, x)                      \
    do {                                  \
        hipError_t e_ = (x);              \
        if (e_ != hipSuccess) {           \
            (c)->err = EK_ERR_DEVICE;     \
            return EK_ERR_DEVICE;         \
        }                                 \
    } while (0)

namespace {

// EK error code of device status bits (0: none).
int status_error(uint32_t st) {
    if (st & ST_NONFINITE) return EK_ERR_NONFINITE;
    if (st & ST_UNSTABLE) return EK_ERR_UNSTABLE;
    return EK_OK;
}

// After the stream has been synchronised: latch what the kernels reported.
int check_status(ek_ctx* c) {
    uint32_t st = 0;
    HIPCHK(c, hipMemcpy(&st, c->arena + c->L.status, sizeof(st), hipMemcpyDeviceToHost));
    if (int e = status_error(st)) c->err = e;
    return c->err;
}

template <typename T>
void setup_sim(ek_ctx* c, Sim<T>& s) {
    const ek_params* p = &c->p;
    unsigned char* A = c->arena;
    const Layout& L = c->L;
    long N = c->N;
    s.nx = p->nx;
    s.ny = p->ny;
    s.nz = p->nz;
    s.nxh = p->nx / 2 + 1;
    s.nxs = spec_stride(p->nx, (int)sizeof(T));
    s.N = N;
    s.Nspec = (long)s.nxs * p->ny * p->nz;
    s.ns = p->n_species;
    s.np = 0;
    s.pv = p->scheme == EK_SCHEME_PARTIAL_VOLUME;
    s.charge_mode = p->charge_mode;
    s.integrator = p->integrator;
    s.cur = 0;
    const double a = p->agrid, tau = p->tau, rf = p->fluid_density;
    s.kT = p->kT * tau * tau / (rf * a * a * a * a * a);
    s.lambda_B = p->bjerrum_length / a;
    for (int d = 0; d < 3; ++d) s.E[d] = p->E_ext[d] * a;
    for (int k = 0; k < MAXS; ++k) s.D[k] = s.z[k] = s.rho_ref[k] = 0.0;
    for (int k = 0; k < p->n_species; ++k) {
        s.D[k] = p->species[k].D * tau / (a * a);
        s.z[k] = p->species[k].valency;
        s.rho_ref[k] = sizeof(T) == 4 ? p->species[k].mean_density * a * a * a : 0.0;
    }
    double nu = p->viscosity * tau / (a * a);
    double tp = 3.0 * nu + 0.5;
    double tm = 0.5 + (3.0 / 16.0) / (tp - 0.5);
    s.lam_e = (T)(-1.0 / tp);
    s.lam_o = (T)(-1.0 / tm);
    s.n_wall = 0;
    size_t ts = sizeof(T);
    s.f[0] = (T*)(A + L.f);
    s.f[1] = s.f[0] + 19 * fpad(N);
    s.rho[0] = (T*)(A + L.rho);
    s.rho[1] = s.rho[0] + (long)p->n_species * N;
    s.u[0] = (T*)(A + L.u);
    s.u[1] = s.u[0] + 3 * fpad(N);
    s.fext = (T*)(A + L.fext);
    s.phi = (T*)(A + L.phi);
    s.rhob = (T*)(A + L.rhob);
    s.psi = (float*)(A + L.psi);
    s.flag = A + L.flag;
    s.owner = (uint16_t*)(A + L.owner);
    s.owner_prev = (uint16_t*)(A + L.owner_prev);
    s.psi_owner = (uint16_t*)(A + L.psi_owner);
    s.wall_charge = nullptr;
    s.spec = (T*)(A + L.spec);
    T* tw = (T*)(A + L.tw);
    T* k2 = (T*)(A + L.k2);
    s.tw[0] = tw;
    s.tw[1] = tw + 2 * p->nx;
    s.tw[2] = tw + 2 * (p->nx + p->ny);
    s.k2[0] = k2;
    s.k2[1] = k2 + p->nx;
    s.k2[2] = k2 + p->nx + p->ny;
    s.parts = (PState*)(A + L.parts);
    s.status = (uint32_t*)(A + L.status);
    s.scratch = (double*)(A + L.scratch);
    s.partial = (double*)(A + L.partial);
    s.box_max = 0;
    s.nchunk = 1;
    (void)ts;
}

template <typename T>
int init_fields(ek_ctx* c, Sim<T>& s) {
    const ek_params* p = &c->p;
    hipStream_t st = c->stream;
    long N = c->N;
    bool dev = sizeof(T) == 4;
    for (int b = 0; b < 2; ++b)
        fill_pops<T>(s.f[b], fpad(N), dev, st);
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < p->n_species; ++k)
            fill<T>(s.rho[b] + (long)k * N, N,
                    dev ? (T)0 : (T)(p->species[k].mean_density * p->agrid * p->agrid * p->agrid), st);
    fill<T>(s.u[0], 2 * 3 * fpad(N), (T)0, st);
    fill<T>(s.fext, 3 * fpad(N), (T)0, st);
    fill<T>(s.phi, N, (T)0, st);
    fill<T>(s.rhob, N, (T)0, st);
    fill<float>(s.psi, N, 0.0f, st);
    fill<uint8_t>(s.flag, N, (uint8_t)0, st);
    fill<uint16_t>(s.owner, N, NO_OWNER, st);
    fill<uint16_t>(s.owner_prev, N, NO_OWNER, st);
    fill<uint16_t>(s.psi_owner, N, NO_OWNER, st);
    HIPCHK(c, hipMemsetAsync(s.status, 0, sizeof(uint32_t), st));
    // FFT tables in FP64 on the host, rounded once to T
    int n[3] = {p->nx, p->ny, p->nz};
    std::vector<T> tw, k2;
    for (int d = 0; d < 3; ++d)
        for (int m = 0; m < n[d]; ++m) {
            double ang = 2.0 * M_PI * (double)m / (double)n[d];
            tw.push_back((T)std::cos(ang));
            tw.push_back((T)-std::sin(ang));
            k2.push_back((T)(2.0 - 2.0 * std::cos(ang)));
        }
    HIPCHK(c, hipMemcpyAsync(s.tw[0], tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(s.k2[0], k2.data(), k2.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIPCHK(c, hipStreamSynchronize(st));
    HIPCHK(c, hipGetLastError());
    return EK_OK;
}

// One step.  In a chain of steps (a captured graph), `moved`: the previous
// step's closing kernel already performed this step's kick and drift;
// `chain`: this step's closing kernel performs the next step's.
// Charge assembly and Poisson solve: FFT, or the iterative solve with the
// permittivity field (host-driven: it waits for its convergence checks).
template <typename T>
void enqueue_poisson(ek_ctx* c, const Sim<T>& s) {
    if (!c->cg) {
        launch_charge_poisson(s, c->stream);
        return;
    }
    int it = 0;
    double res = 0.0;
    if (cg_solve(s, *c->cg, c->stream, &it, &res) != 0) c->cg_failed = true;
    c->cg_iters = it;
    c->cg_res = res;
    if (!(res <= c->cg->tol)) c->cg_failed = true;
}

template <typename T>
void enqueue_step(ek_ctx* c, Sim<T> s, bool moved = false, bool chain = false) {
    hipStream_t st = c->stream;
    if (!moved) launch_move(s, st, 0);
    launch_geometry(s, st, 0);
    launch_boundary(s, st);
    if (!s.pv) launch_refill(s, st);
    enqueue_poisson(c, s);
    launch_particle_forces(s, st);
    launch_fields(s, st);
    launch_finish(s, st, chain);
}

// One step with a HIP event recorded after each stage (instrumentation).
template <typename T>
void enqueue_step_timed(ek_ctx* c, Sim<T> s, hipEvent_t* ev) {
    hipStream_t st = c->stream;
    (void)hipEventRecord(ev[0], st);
    launch_move(s, st, 0);
    (void)hipEventRecord(ev[1], st);
    launch_geometry(s, st, 0);
    (void)hipEventRecord(ev[2], st);
    launch_boundary(s, st);
    if (!s.pv) launch_refill(s, st);
    (void)hipEventRecord(ev[3], st);
    enqueue_poisson(c, s);
    (void)hipEventRecord(ev[4], st);
    launch_particle_forces(s, st);
    (void)hipEventRecord(ev[5], st);
    launch_fields(s, st, ev[6]);
    (void)hipEventRecord(ev[7], st);
    launch_finish(s, st);
    (void)hipEventRecord(ev[8], st);
}

template <typename T>
int profile_steps(ek_ctx* c, Sim<T>& s, int n, double* acc) {
    hipEvent_t ev[EK_N_STAGES + 1];
    for (int k = 0; k <= EK_N_STAGES; ++k) HIPCHK(c, hipEventCreate(&ev[k]));
    int r = EK_OK;
    for (int i = 0; i < n && r == EK_OK; ++i) {
        enqueue_step_timed(c, s, ev);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(ev[EK_N_STAGES]) != hipSuccess) {
            c->err = r = EK_ERR_DEVICE;
            break;
        }
        for (int k = 0; k < EK_N_STAGES; ++k) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            acc[k] += ms;
        }
        s.cur ^= 1;
        c->set_cur(s.cur);
        c->step += 1;
    }
    for (int k = 0; k <= EK_N_STAGES; ++k) (void)hipEventDestroy(ev[k]);
    return r;
}

template <typename T>
int build_graph(ek_ctx* c, Sim<T> s, int parity, int nsteps, hipGraphExec_t* out) {
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < nsteps; ++k) {
        s.cur = (parity + k) & 1;
        enqueue_step(c, s, k > 0, k < nsteps - 1);
    }
    HIPCHK(c, hipStreamEndCapture(c->stream, &g));
    hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(c, e);
    return EK_OK;
}

template <typename T>
int run_steps(ek_ctx* c, Sim<T>& s, int n) {
    while (n > 0) {
        int par = s.cur;
        int chunk = (n >= GRAPH_CHUNK) ? 1 : 0;
        int k = chunk ? GRAPH_CHUNK : 1;
        if (c->use_graphs && !c->cg) {
            if (!c->graph[par][chunk]) {
                int r = build_graph(c, s, par, k, &c->graph[par][chunk]);
                if (r) return r;
            }
            HIPCHK(c, hipGraphLaunch(c->graph[par][chunk], c->stream));
        } else {
            Sim<T> t = s;
            for (int i = 0; i < k; ++i) {
                t.cur = (par + i) & 1;
                enqueue_step(c, t);
                if (c->cg_failed) return c->err = EK_ERR_UNSTABLE;
            }
            HIPCHK(c, hipGetLastError());
        }
        if (k & 1) c->set_cur(par ^ 1);
        c->step += k;
        n -= k;
    }
    return EK_OK;
}

// Particle count and the workgroups per particle box of the box kernels: the
// box extent for a displacement below one cell per step (larger displacements
// only make their grid-stride loops take more turns).
void set_box_chunks(ek_ctx* c) {
    int box_max = 0;
    const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
    for (const PState& q : c->parts) {
        int b = 1;
        for (int d = 0; d < 3; ++d) {
            int e = (int)std::ceil(2.0 * q.R) + 2 * BOX_MARGIN + 2;
            b *= e < n[d] ? e : n[d];
        }
        box_max = b > box_max ? b : box_max;
    }
    c->sf.np = c->sd.np = (int)c->parts.size();
    c->sf.box_max = c->sd.box_max = box_max;
    const int per = 256 * BOX_CELLS_PER_THREAD;
    int nch = (box_max + per - 1) / per;
    c->sf.nchunk = c->sd.nchunk = nch < 1 ? 1 : (nch > MAX_CHUNKS ? MAX_CHUNKS : nch);
}

template <typename T>
int prepare(ek_ctx* c, Sim<T>& s) {
    hipStream_t st = c->stream;
    int np = (int)c->parts.size();
    set_box_chunks(c);
    if (np > 0)
        HIPCHK(c, hipMemcpyAsync(s.parts, c->parts.data(), np * sizeof(PState), hipMemcpyHostToDevice, st));
    Sim<T> t = s;
    launch_move(t, st, 1);
    launch_geometry(t, st, 1);
    launch_init_density(t, st);
    launch_boundary(t, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    c->prepared = true;
    return EK_OK;
}

// conversion factors: simulation value = lattice value * factor
double field_factor(const ek_ctx* c, int field) {
    double a = c->a, tau = c->tau, rf = c->rf;
    switch (field) {
        case EK_FIELD_DENSITY: return 1.0 / (a * a * a);
        case EK_FIELD_PHI: return 1.0;
        case EK_FIELD_VELOCITY: return a / tau;
        case EK_FIELD_FLUID_DENSITY: return rf;
        case EK_FIELD_FORCE: return rf * a / (tau * tau);
        case EK_FIELD_PSI: return 1.0;
        case EK_FIELD_POPULATIONS: return rf;
        case EK_FIELD_PARTICLE_CHARGE: return 1.0 / (a * a * a);
        default: return 1.0;
    }
}

long field_elems(const ek_ctx* c, int field) {
    long N = c->N;
    switch (field) {
        case EK_FIELD_DENSITY: return (long)c->p.n_species * N;
        case EK_FIELD_VELOCITY:
        case EK_FIELD_FORCE: return 3 * N;
        case EK_FIELD_POPULATIONS: return 19 * N;
        case EK_FIELD_PHI:
        case EK_FIELD_FLUID_DENSITY:
        case EK_FIELD_PSI:
        case EK_FIELD_FLAG:
        case EK_FIELD_OWNER:
        case EK_FIELD_PARTICLE_CHARGE: return N;
        default: return -1;
    }
}

template <typename T>
int get_field(ek_ctx* c, Sim<T>& s, int field, void* host, size_t bytes) {
    long ne = field_elems(c, field);
    if (ne < 0) return EK_ERR_INVALID_ARG;
    long N = c->N;
    hipStream_t st = c->stream;
    HIPCHK(c, hipStreamSynchronize(st));
    if (int e = check_status(c)) return e;
    bool dev = sizeof(T) == 4;
    double fac = field_factor(c, field);
    if (field == EK_FIELD_FLAG) {
        if (bytes != (size_t)N) return EK_ERR_INVALID_ARG;
        std::vector<uint8_t> h(N);
        HIPCHK(c, hipMemcpy(h.data(), s.flag, N, hipMemcpyDeviceToHost));
        uint8_t* o = (uint8_t*)host;
        for (long i = 0; i < N; ++i) o[i] = (h[i] & F_CUR) ? 1 : 0;
        return EK_OK;
    }
    if (field == EK_FIELD_OWNER) {
        if (bytes != (size_t)N * sizeof(int32_t)) return EK_ERR_INVALID_ARG;
        std::vector<uint16_t> h(N);
        std::vector<uint8_t> fl(N);
        HIPCHK(c, hipMemcpy(h.data(), s.owner, N * 2, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(fl.data(), s.flag, N, hipMemcpyDeviceToHost));
        int32_t* o = (int32_t*)host;
        for (long i = 0; i < N; ++i) o[i] = ((fl[i] & F_CUR) && h[i] != NO_OWNER) ? (int32_t)h[i] : -1;
        return EK_OK;
    }
    if (bytes != (size_t)ne * sizeof(double)) return EK_ERR_INVALID_ARG;
    double* o = (double*)host;
    if (field == EK_FIELD_PSI) {
        std::vector<float> h(N);
        HIPCHK(c, hipMemcpy(h.data(), s.psi, N * sizeof(float), hipMemcpyDeviceToHost));
        for (long i = 0; i < N; ++i) o[i] = h[i];
        return EK_OK;
    }
    std::vector<T> h;
    const T* src = nullptr;
    int cur = s.cur;
    switch (field) {
        case EK_FIELD_DENSITY: src = s.rho[cur]; break;
        case EK_FIELD_PHI: src = s.phi; break;
        case EK_FIELD_VELOCITY: src = s.u[cur]; break;
        case EK_FIELD_FORCE: src = s.fext; break;
        case EK_FIELD_POPULATIONS:
        case EK_FIELD_FLUID_DENSITY: src = s.f[cur]; break;
        case EK_FIELD_PARTICLE_CHARGE: src = s.rhob; break;
    }
    const bool pops = field == EK_FIELD_POPULATIONS || field == EK_FIELD_FLUID_DENSITY;
    const bool vec = field == EK_FIELD_VELOCITY || field == EK_FIELD_FORCE;
    // populations, velocity and force are stored in blocks of FB cells
    long nsrc = pops ? 19 * fpad(N) : (vec ? 3 * fpad(N) : ne);
    h.resize(nsrc);
    HIPCHK(c, hipMemcpy(h.data(), src, nsrc * sizeof(T), hipMemcpyDeviceToHost));
    if (field == EK_FIELD_DENSITY) {
        for (int k = 0; k < c->p.n_species; ++k)
            for (long i = 0; i < N; ++i) o[k * N + i] = ((dev ? s.rho_ref[k] : 0.0) + (double)h[k * N + i]) * fac;
    } else if (field == EK_FIELD_POPULATIONS) {
        for (int q = 0; q < 19; ++q)
            for (long i = 0; i < N; ++i) o[q * N + i] = ((dev ? q19w(q) : 0.0) + (double)h[fidx(q, i)]) * fac;
    } else if (field == EK_FIELD_FLUID_DENSITY) {
        for (long i = 0; i < N; ++i) {
            double m = dev ? 1.0 : 0.0;
            for (int q = 0; q < 19; ++q) m += (double)h[fidx(q, i)];
            o[i] = m * fac;
        }
    } else if (vec) {
        for (int d = 0; d < 3; ++d)
            for (long i = 0; i < N; ++i) o[d * N + i] = (double)h[vidx(d, i)] * fac;
    } else {
        for (long i = 0; i < ne; ++i) o[i] = (double)h[i] * fac;
    }
    return EK_OK;
}

template <typename T>
int set_field(ek_ctx* c, Sim<T>& s, int field, const void* host, size_t bytes) {
    long ne = field_elems(c, field);
    long N = c->N;
    if (ne < 0 || bytes != (size_t)ne * sizeof(double)) return EK_ERR_INVALID_ARG;
    const double* in = (const double*)host;
    for (long i = 0; i < ne; ++i)
        if (!std::isfinite(in[i])) return EK_ERR_NONFINITE;
    bool dev = sizeof(T) == 4;
    double fac = field_factor(c, field);
    std::vector<T> h(ne);
    T* dst = nullptr;
    int cur = s.cur;
    switch (field) {
        case EK_FIELD_DENSITY:
            dst = s.rho[cur];
            for (int k = 0; k < c->p.n_species; ++k)
                for (long i = 0; i < N; ++i) h[k * N + i] = (T)(in[k * N + i] / fac - (dev ? s.rho_ref[k] : 0.0));
            break;
        case EK_FIELD_POPULATIONS:
            // to the blocked layout; the padding cells hold the rest state
            dst = s.f[cur];
            h.assign(19 * fpad(N), (T)0);
            for (long e = 0; e < 19 * fpad(N); ++e) h[e] = dev ? (T)0 : (T)q19w((int)((e / FB) % 19));
            for (int q = 0; q < 19; ++q)
                for (long i = 0; i < N; ++i) h[fidx(q, i)] = (T)(in[q * N + i] / fac - (dev ? q19w(q) : 0.0));
            break;
        case EK_FIELD_PHI: dst = s.phi; break;
        case EK_FIELD_VELOCITY: dst = s.u[cur]; break;
        case EK_FIELD_FORCE: dst = s.fext; break;
        default: return EK_ERR_INVALID_ARG;
    }
    if (field == EK_FIELD_PHI)
        for (long i = 0; i < ne; ++i) h[i] = (T)(in[i] / fac);
    if (field == EK_FIELD_VELOCITY || field == EK_FIELD_FORCE) {
        h.assign(3 * fpad(N), (T)0);
        for (int d = 0; d < 3; ++d)
            for (long i = 0; i < N; ++i) h[vidx(d, i)] = (T)(in[d * N + i] / fac);
    }
    HIPCHK(c, hipMemcpyAsync(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EK_OK;
}

template <typename T>
int diagnostics(ek_ctx* c, Sim<T>& s, ek_diag* out) {
    double* dout = (double*)(c->arena + c->L.diag);
    launch_diagnostics(s, c->stream, dout);
    HIPCHK(c, hipGetLastError());
    double h[NDIAG];
    HIPCHK(c, hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (int e = check_status(c)) return e;
    for (int k = 0; k < NDIAG; ++k)
        if (!std::isfinite(h[k])) return c->err = EK_ERR_NONFINITE;
    double a = c->a, tau = c->tau, rf = c->rf;
    std::memset(out, 0, sizeof(*out));
    out->step = c->step;
    for (int k = 0; k < c->p.n_species; ++k) {
        out->species_total[k] = h[k];
        out->solute_charge += c->p.species[k].valency * h[k];
    }
    out->particle_charge = h[MAXS];
    out->fluid_mass = h[MAXS + 1] * rf * a * a * a;
    for (int d = 0; d < 3; ++d) out->fluid_momentum[d] = h[MAXS + 2 + d] * rf * a * a * a * a / tau;
    out->boundary_cells = (long long)h[MAXS + 5];
    out->max_velocity = h[MAXS + 6];
    int np = (int)c->parts.size();
    if (np > 0 && c->prepared) {
        std::vector<PState> ps(np);
        HIPCHK(c, hipMemcpy(ps.data(), s.parts, np * sizeof(PState), hipMemcpyDeviceToHost));
        for (const PState& q : ps) {
            out->covered += q.ncov;
            out->vacated += q.nvac;
            out->pooled += q.npool;
        }
    }
    return EK_OK;
}

}  // namespace

template <typename T>
int seed_density(ek_ctx* c, Sim<T>& s, uint64_t seed, double noise) {
    SeedArgs a{};
    a.seed = seed;
    a.noise = noise;
    a.fac = field_factor(c, EK_FIELD_DENSITY);
    for (int k = 0; k < c->p.n_species; ++k) a.mean[k] = c->p.species[k].mean_density;
    launch_seed_density(s, a, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return EK_OK;
}

namespace {
// Steps enqueued directly on the stream (no graph, no allocation), the
// particle partial sums in the fixed scratch array at `scratch`.
template <typename T>
void enqueue_steps_direct(ek_ctx* c, Sim<T>& s, int n, double* scratch) {
    Sim<T> t = s;
    t.partial = scratch;
    const int par = s.cur;
    for (int k = 0; k < n; ++k) {
        t.cur = (par + k) & 1;
        enqueue_step(c, t, k > 0, k < n - 1);
    }
    if (n & 1) c->set_cur(par ^ 1);
    c->step += n;
}
}  // namespace

extern "C" {

const char* ek_strerror(int code) {
    switch (code) {
        case EK_OK: return "ok";
        case EK_ERR_INVALID_ARG: return "invalid argument";
        case EK_ERR_UNSUPPORTED_SIZE: return "unsupported box size (each edge 2^a 3^b, a >= 1, 8..512)";
        case EK_ERR_UNSTABLE: return "parameters outside the stability range";
        case EK_ERR_OVERLAP: return "sphere too large for the box";
        case EK_ERR_OOM: return "out of device memory";
        case EK_ERR_NO_SPACE: return "no free slot or memory";
        case EK_ERR_NONFINITE: return "non-finite input";
        case EK_ERR_DEVICE: return "HIP device error";
        case EK_ERR_STATE: return "call not allowed in the current state";
        default: return "unknown error";
    }
}

int ek_query_footprint(const ek_params* p, size_t* bytes) {
    int r = validate(p);
    if (r) return r;
    if (!bytes) return EK_ERR_INVALID_ARG;
    *bytes = make_layout(p, p->precision == EK_FP32_DEV ? 4 : 8).total;
    return EK_OK;
}

int ek_create(const ek_params* p, ek_ctx** out) {
    if (!out) return EK_ERR_INVALID_ARG;
    *out = nullptr;
    int r = validate(p);
    if (r) return r;
    ek_ctx* c = new (std::nothrow) ek_ctx();
    if (!c) return EK_ERR_OOM;
    c->p = *p;
    c->fp32 = p->precision == EK_FP32_DEV;
    c->L = make_layout(p, c->fp32 ? 4 : 8);
    c->N = (long)p->nx * p->ny * p->nz;
    c->a = p->agrid;
    c->tau = p->tau;
    c->rf = p->fluid_density;
    c->use_graphs = std::getenv("EK_DISABLE_GRAPHS") == nullptr;
    if (p->stream) {
        c->stream = (hipStream_t)p->stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return EK_ERR_DEVICE;
        }
        c->own_stream = true;
    }
    if (p->arena) {
        if (p->arena_bytes < c->L.total) {
            ek_destroy(c);
            return EK_ERR_OOM;
        }
        c->arena = (unsigned char*)p->arena;
    } else {
        if (hipMalloc(&c->arena, c->L.total) != hipSuccess) {
            (void)hipGetLastError();
            c->arena = nullptr;
            ek_destroy(c);
            return EK_ERR_OOM;
        }
        c->own_arena = true;
    }
    c->p.arena = c->arena;
    c->p.arena_bytes = c->L.total;
    setup_sim(c, c->sf);
    setup_sim(c, c->sd);
    r = c->fp32 ? init_fields(c, c->sf) : init_fields(c, c->sd);
    if (r) {
        ek_destroy(c);
        return r;
    }
    *out = c;
    return EK_OK;
}

int ek_add_sphere(ek_ctx* c, const double pos[3], double radius, double charge, double mass, const double v0[3],
                  int mode, int* id) {
    if (!c || !pos) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    if (c->prepared) return EK_ERR_STATE;
    if ((int)c->parts.size() >= c->p.max_particles) return EK_ERR_STATE;
    if (mode != EK_FREE && mode != EK_PRESCRIBED && mode != EK_FIXED) return EK_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(pos[d]) || (v0 && !std::isfinite(v0[d]))) return EK_ERR_NONFINITE;
    if (!std::isfinite(radius) || !std::isfinite(charge) || !std::isfinite(mass)) return EK_ERR_NONFINITE;
    if (!(radius > 0) || (mode == EK_FREE && !(mass > 0))) return EK_ERR_INVALID_ARG;
    double a = c->a, tau = c->tau, rf = c->rf;
    double R = radius / a;
    int n[3] = {c->p.nx, c->p.ny, c->p.nz};
    // cells within R + 1 of the centre must have a unique periodic image
    for (int d = 0; d < 3; ++d)
        if (2.0 * R + 2.0 > n[d]) return EK_ERR_OVERLAP;
    PState q;
    std::memset(&q, 0, sizeof(q));
    for (int d = 0; d < 3; ++d) {
        double x = pos[d] / a;
        x = x - n[d] * std::floor(x / n[d]);
        if (x >= n[d]) x -= n[d];
        q.x[d] = x;
    }
    // no two spheres may intersect (minimum-image distance of the centres
    // below the sum of the radii)
    for (const PState& o : c->parts) {
        double d2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            double dx = q.x[d] - o.x[d];
            if (dx > 0.5 * n[d]) dx -= n[d];
            else if (dx < -0.5 * n[d]) dx += n[d];
            d2 += dx * dx;
        }
        if (d2 < (R + o.R) * (R + o.R)) return EK_ERR_OVERLAP;
    }
    for (int d = 0; d < 3; ++d) {
        q.v[d] = (v0 && mode != EK_FIXED) ? v0[d] * tau / a : 0.0;
        if (std::fabs(q.v[d]) >= 1.0) return EK_ERR_UNSTABLE;
    }
    q.R = R;
    q.Z = charge;
    q.M = mass > 0 ? mass / (rf * a * a * a) : 1.0;
    q.I = 0.4 * q.M * q.R * q.R;
    q.Vp = 4.0 / 3.0 * M_PI * R * R * R;
    q.mode = mode;
    if (id) *id = (int)c->parts.size();
    c->parts.push_back(q);
    return EK_OK;
}

int ek_set_static_boundary(ek_ctx* c, const uint8_t* mask, const double* charge) {
    if (!c || !mask) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    if (c->prepared) return EK_ERR_STATE;
    long N = c->N;
    std::vector<uint8_t> fl(N);
    long nw = 0;
    for (long i = 0; i < N; ++i) {
        fl[i] = mask[i] ? (uint8_t)(F_WALL | F_CUR | F_PREV) : (uint8_t)0;
        nw += mask[i] ? 1 : 0;
    }
    uint8_t* dflag = c->fp32 ? c->sf.flag : c->sd.flag;
    HIPCHK(c, hipMemcpy(dflag, fl.data(), N, hipMemcpyHostToDevice));
    c->sf.n_wall = c->sd.n_wall = nw;
    if (charge) {
        std::vector<double> q(N);
        for (long i = 0; i < N; ++i) {
            if (!std::isfinite(charge[i])) return EK_ERR_NONFINITE;
            q[i] = charge[i] * c->a * c->a * c->a;
        }
        if (!c->wall_charge) HIPCHK(c, hipMalloc(&c->wall_charge, N * sizeof(double)));
        HIPCHK(c, hipMemcpy(c->wall_charge, q.data(), N * sizeof(double), hipMemcpyHostToDevice));
        c->sf.wall_charge = c->sd.wall_charge = c->wall_charge;
        if (c->fp32) {
            std::vector<float> h(q.begin(), q.end());
            HIPCHK(c, hipMemcpy(c->sf.rhob, h.data(), N * sizeof(float), hipMemcpyHostToDevice));
        } else {
            HIPCHK(c, hipMemcpy(c->sd.rhob, q.data(), N * sizeof(double), hipMemcpyHostToDevice));
        }
    }
    return EK_OK;
}

int ek_set_fields(ek_ctx* c, int field, const void* host, size_t bytes) {
    if (!c || !host) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    return c->fp32 ? set_field(c, c->sf, field, host, bytes) : set_field(c, c->sd, field, host, bytes);
}

int ek_seed_density(ek_ctx* c, uint64_t seed, double noise) {
    if (!c || !std::isfinite(noise) || std::fabs(noise) > 1.0) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    return c->fp32 ? seed_density(c, c->sf, seed, noise) : seed_density(c, c->sd, seed, noise);
}

int ek_prepare(ek_ctx* c) {
    if (!c) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    if (c->prepared) return EK_OK;
    return c->fp32 ? prepare(c, c->sf) : prepare(c, c->sd);
}

int ek_step(ek_ctx* c, int n) {
    if (!c || n < 0) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    if (!c->prepared) {
        int r = ek_prepare(c);
        if (r) return r;
    }
    if (!c->host_status) {
        if (hipHostMalloc((void**)&c->host_status, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->host_status = nullptr;
            return EK_ERR_OOM;
        }
        *c->host_status = 0;
    }
    // what the device reported up to the last completed ek_step
    if (int e = status_error(__atomic_load_n(c->host_status, __ATOMIC_RELAXED))) return c->err = e;
    int r = c->fp32 ? run_steps(c, c->sf, n) : run_steps(c, c->sd, n);
    if (r) return r;
    HIPCHK(c, hipMemcpyAsync(c->host_status, c->arena + c->L.status, sizeof(uint32_t), hipMemcpyDeviceToHost,
                             c->stream));
    return EK_OK;
}

int ek_step_noalloc(ek_ctx* c, int n) {
    if (!c || n < 0) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    if (!c->prepared || c->cg) return EK_ERR_STATE;
    const Sim<float>& sf = c->sf;
    const size_t need = (size_t)PART_KINDS * (size_t)sf.np * (size_t)sf.nchunk * PSTRIDE * sizeof(double);
    if (need > NOALLOC_SCRATCH_BYTES) return EK_ERR_NO_SPACE;
    void* scratch = nullptr;
    HIPCHK(c, noalloc_scratch(&scratch));
    if (n == 0) return EK_OK;
    if (c->fp32) enqueue_steps_direct(c, c->sf, n, (double*)scratch);
    else enqueue_steps_direct(c, c->sd, n, (double*)scratch);
    HIPCHK(c, hipGetLastError());
    return EK_OK;
}

int ek_set_permittivity(ek_ctx* c, const double* eps_r, double tol, int max_iter) {
    if (!c) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (!eps_r) {
        if (c->cg_mem) HIPCHK(c, hipFree(c->cg_mem));
        c->cg_mem = nullptr;
        delete c->cg;
        c->cg = nullptr;
        return EK_OK;
    }
    if (!(tol > 0.0 && tol < 1.0) || max_iter < 1) return EK_ERR_INVALID_ARG;
    const long N = c->N;
    for (long i = 0; i < N; ++i) {
        if (!std::isfinite(eps_r[i])) return EK_ERR_NONFINITE;
        if (!(eps_r[i] > 0.0)) return EK_ERR_INVALID_ARG;
    }
    if (!c->cg) {
        // x, r, p, q, 3 face arrays, inverse diagonal, permittivity upload: 9 N doubles
        const size_t part = (size_t)1024 * 4 * sizeof(double), sc = 64 * sizeof(double);
        const size_t bytes = 9 * (size_t)N * sizeof(double) + part + sc;
        void* mem = nullptr;
        if (hipMalloc(&mem, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return EK_ERR_OOM;
        }
        CGState* g = new (std::nothrow) CGState();
        if (!g) {
            (void)hipFree(mem);
            return EK_ERR_OOM;
        }
        double* d = (double*)mem;
        g->x = d;
        g->r = d + N;
        g->p = d + 2 * N;
        g->q = d + 3 * N;
        for (int k = 0; k < 3; ++k) g->ef[k] = d + (4 + k) * N;
        g->idiag = d + 7 * N;
        g->part = d + 9 * N;
        g->sc = g->part + 1024 * 4;
        c->cg = g;
        c->cg_mem = mem;
        HIPCHK(c, hipMemsetAsync(g->x, 0, N * sizeof(double), c->stream));
    }
    CGState* g = c->cg;
    g->nx = c->p.nx;
    g->ny = c->p.ny;
    g->nz = c->p.nz;
    g->N = N;
    g->fourpi_lb = 4.0 * M_PI * (c->fp32 ? c->sf.lambda_B : c->sd.lambda_B);
    g->tol = tol;
    g->max_iter = max_iter;
    double* eps_dev = (double*)c->cg_mem + 8 * N;
    HIPCHK(c, hipMemcpyAsync(eps_dev, eps_r, N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (cg_setup(*g, eps_dev, c->stream) != 0) return c->err = EK_ERR_DEVICE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cg_failed = false;
    return EK_OK;
}

int ek_get_poisson_stats(ek_ctx* c, int* iterations, double* residual) {
    if (!c) return EK_ERR_INVALID_ARG;
    if (iterations) *iterations = c->cg ? c->cg_iters : 0;
    if (residual) *residual = c->cg ? c->cg_res : 0.0;
    return EK_OK;
}

int ek_profile_stages(ek_ctx* c, int n, double* ms_out, int n_out) {
    if (!c || n <= 0 || !ms_out || n_out < 1 || n_out > EK_N_STAGES) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    if (!c->prepared) {
        int r = ek_prepare(c);
        if (r) return r;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double acc[EK_N_STAGES] = {0};
    int r = c->fp32 ? profile_steps(c, c->sf, n, acc) : profile_steps(c, c->sd, n, acc);
    if (r) return r;
    for (int k = 0; k < n_out; ++k) ms_out[k] = acc[k] / n;
    return EK_OK;
}

int ek_copy_probe(void* dst, const void* src, size_t bytes, void* stream) {
    if (!dst || !src || bytes % 16 || bytes > ((size_t)1 << 40)) return EK_ERR_INVALID_ARG;
    launch_copy16(dst, src, (long)(bytes / 16), (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? EK_OK : EK_ERR_DEVICE;
}

int ek_synchronize(ek_ctx* c) {
    if (!c) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return check_status(c);
}

int ek_get_fields(ek_ctx* c, int field, void* host, size_t bytes) {
    if (!c || !host) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    return c->fp32 ? get_field(c, c->sf, field, host, bytes) : get_field(c, c->sd, field, host, bytes);
}

int ek_get_particles(ek_ctx* c, ek_particle* out, int n) {
    if (!c || (!out && n > 0) || n < 0 || n > (int)c->parts.size()) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    std::vector<PState> ps(c->parts.size());
    if (c->prepared && !ps.empty()) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (int e = check_status(c)) return e;
        PState* dp = c->fp32 ? c->sf.parts : c->sd.parts;
        HIPCHK(c, hipMemcpy(ps.data(), dp, ps.size() * sizeof(PState), hipMemcpyDeviceToHost));
    } else {
        ps = c->parts;
    }
    double a = c->a, tau = c->tau, rf = c->rf;
    double fF = rf * a * a * a * a / (tau * tau), fT = fF * a;
    for (int k = 0; k < n; ++k) {
        const PState& q = ps[k];
        ek_particle& o = out[k];
        std::memset(&o, 0, sizeof(o));
        for (int d = 0; d < 3; ++d) {
            o.x[d] = q.x[d] * a;
            o.v[d] = q.v[d] * a / tau;
            o.omega[d] = q.w[d] / tau;
            o.F[d] = q.F[d] * fF;
            o.T[d] = q.T[d] * fT;
            o.F_hyd[d] = q.Fh[d] * fF;
            o.F_el[d] = q.Fe[d] * fF;
            o.F_cov[d] = q.Fc[d] * fF;
        }
        o.radius = q.R * a;
        o.charge = q.Z;
        o.mass = q.M * rf * a * a * a;
        o.mode = q.mode;
        o.n_boundary = q.nb;
    }
    return EK_OK;
}

int ek_get_diagnostics(ek_ctx* c, ek_diag* out) {
    if (!c || !out) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    return c->fp32 ? diagnostics(c, c->sf, out) : diagnostics(c, c->sd, out);
}

struct StateHeader {
    uint64_t magic;
    int64_t bytes, step;
    int32_t cur, prepared, np, precision;
};
static const uint64_t STATE_MAGIC = 0x454b53544154453aULL;

int ek_get_state(ek_ctx* c, void* host, size_t* bytes) {
    if (!c || !bytes) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    size_t need = sizeof(StateHeader) + c->L.state_end + (c->wall_charge ? c->N * sizeof(double) : 0);
    if (!host) {
        *bytes = need;
        return EK_OK;
    }
    if (*bytes < need) return EK_ERR_INVALID_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    StateHeader h{STATE_MAGIC, (int64_t)need, c->step, c->cur(), c->prepared ? 1 : 0, (int32_t)c->parts.size(),
                  c->p.precision};
    std::memcpy(host, &h, sizeof(h));
    unsigned char* dst = (unsigned char*)host + sizeof(h);
    HIPCHK(c, hipMemcpy(dst, c->arena, c->L.state_end, hipMemcpyDeviceToHost));
    if (c->wall_charge)
        HIPCHK(c, hipMemcpy(dst + c->L.state_end, c->wall_charge, c->N * sizeof(double), hipMemcpyDeviceToHost));
    *bytes = need;
    return EK_OK;
}

int ek_set_state(ek_ctx* c, const void* host, size_t bytes) {
    if (!c || !host || bytes < sizeof(StateHeader)) return EK_ERR_INVALID_ARG;
    if (c->err) return c->err;
    StateHeader h;
    std::memcpy(&h, host, sizeof(h));
    size_t need = sizeof(StateHeader) + c->L.state_end + (c->wall_charge ? c->N * sizeof(double) : 0);
    if (h.magic != STATE_MAGIC || (size_t)h.bytes != bytes || bytes != need || h.np != (int)c->parts.size() ||
        h.precision != c->p.precision)
        return EK_ERR_INVALID_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const unsigned char* src = (const unsigned char*)host + sizeof(h);
    HIPCHK(c, hipMemcpy(c->arena, src, c->L.state_end, hipMemcpyHostToDevice));
    if (c->wall_charge)
        HIPCHK(c, hipMemcpy(c->wall_charge, src + c->L.state_end, c->N * sizeof(double), hipMemcpyHostToDevice));
    c->step = h.step;
    c->set_cur(h.cur);
    if (h.prepared && !c->prepared) {
        set_box_chunks(c);
        c->prepared = true;
    }
    return EK_OK;
}

int ek_destroy(ek_ctx* c) {
    if (!c) return EK_ERR_INVALID_ARG;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (c->graph[i][j]) (void)hipGraphExecDestroy(c->graph[i][j]);
    if (c->own_arena && c->arena) (void)hipFree(c->arena);
    if (c->wall_charge) (void)hipFree(c->wall_charge);
    if (c->host_status) (void)hipHostFree(c->host_status);
    if (c->cg_mem) (void)hipFree(c->cg_mem);
    delete c->cg;
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return EK_OK;
}

}  // extern "C"

// ===========================================================================
// Serving form
// ===========================================================================
#include <map>

struct ek_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t admit_stream = nullptr;  // admissions build their state here, beside the running batch
    unsigned char* arena = nullptr;
    size_t bytes = 0;
    bool own_arena = false;
    BatchTable* dtab = nullptr;   // the live table
    BatchTable* dup = nullptr;    // device staging of an upload (k_batch_merge's source)
    BatchTable* hup = nullptr;    // pinned host staging of an upload
    hipEvent_t up_ev = nullptr;   // the last upload's copy has been read
    bool up_pending = false;
    std::map<size_t, size_t> free_ranges;  // offset -> size
    struct Slot {
        bool used = false, on_device = false, reported = false;
        ek_ctx* ctx = nullptr;
        size_t off = 0, size = 0;
        long long cells = 0;
        unsigned epoch = 0;  // admissions into this slot index so far
    } slot[MAX_SLOTS];
    // Host copies of the device-owned block taken after each chunk of steps
    // (at most two chunks are queued ahead of the host).
    struct Snap {
        unsigned char* host = nullptr;  // pinned, BATCH_DEV_BYTES
        hipEvent_t ev = nullptr;
        bool pending = false;
        long long seq = 0;
        bool on_dev[MAX_SLOTS];
        unsigned epoch[MAX_SLOTS];
    } snap[2];
    long long seq = 0, applied = 0;  // chunks queued; newest chunk reflected in h
    std::vector<std::pair<hipGraphExec_t, hipEvent_t>> retired;  // graphs possibly still queued
    BatchTable h{};
    int ns = 0;
    bool dirty = true;
    hipGraphExec_t graph = nullptr;
    int graph_items[KK_N] = {};  // work items per kind the captured launches were sized for
    bool refill = false, graph_refill = false;  // a live slot uses the simple scheme (now; when captured)
    int err = EK_OK;
};

namespace {

constexpr size_t SLOT_ALIGN = 4096;

bool range_alloc(ek_batch* b, size_t need, size_t* off) {
    need = (need + SLOT_ALIGN - 1) & ~(SLOT_ALIGN - 1);
    for (auto it = b->free_ranges.begin(); it != b->free_ranges.end(); ++it) {
        if (it->second >= need) {
            *off = it->first;
            size_t rest = it->second - need;
            size_t roff = it->first + need;
            b->free_ranges.erase(it);
            if (rest) b->free_ranges[roff] = rest;
            return true;
        }
    }
    return false;
}

void range_free(ek_batch* b, size_t off, size_t size) {
    size = (size + SLOT_ALIGN - 1) & ~(SLOT_ALIGN - 1);
    auto it = b->free_ranges.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != b->free_ranges.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        b->free_ranges.erase(nx);
    }
    if (it != b->free_ranges.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            b->free_ranges.erase(it);
        }
    }
}

#define BCHK(b, x)                    \
    do {                              \
        if ((x) != hipSuccess) {      \
            (b)->err = EK_ERR_DEVICE; \
            return EK_ERR_DEVICE;     \
        }                             \
    } while (0)

// Device-owned entries (a copy of the block) into the host mirror and the
// slots' contexts, for the slots that were on the device, with the same
// occupant, when the copy was taken.
void apply_dev(ek_batch* b, const unsigned char* blk, const bool* on_dev, const unsigned* epoch) {
    int active[MAX_SLOTS], cur[MAX_SLOTS];
    uint32_t status[MAX_SLOTS];
    long long step[MAX_SLOTS];
    std::memcpy(active, blk + offsetof(BatchTable, active), sizeof(active));
    std::memcpy(cur, blk + offsetof(BatchTable, cur), sizeof(cur));
    std::memcpy(status, blk + offsetof(BatchTable, status), sizeof(status));
    std::memcpy(step, blk + offsetof(BatchTable, step), sizeof(step));
    for (int i = 0; i < MAX_SLOTS; ++i) {
        ek_batch::Slot& s = b->slot[i];
        if (!s.used || !on_dev[i] || epoch[i] != s.epoch) continue;
        b->h.active[i] = active[i];
        b->h.cur[i] = cur[i];
        b->h.sims[i].cur = cur[i];
        b->h.status[i] = status[i];
        b->h.step[i] = step[i];
        s.ctx->set_cur(cur[i]);
        s.ctx->step = step[i];
    }
}

// Exact state: wait for everything queued, then read the block.
int pull_state(ek_batch* b) {
    BCHK(b, hipStreamSynchronize(b->stream));
    alignas(8) unsigned char blk[BATCH_DEV_BYTES];
    BCHK(b, hipMemcpy(blk, b->dtab, BATCH_DEV_BYTES, hipMemcpyDeviceToHost));
    bool on_dev[MAX_SLOTS];
    unsigned epoch[MAX_SLOTS];
    for (int i = 0; i < MAX_SLOTS; ++i) {
        on_dev[i] = b->slot[i].used && b->slot[i].on_device;
        epoch[i] = b->slot[i].epoch;
    }
    apply_dev(b, blk, on_dev, epoch);
    for (auto& sn : b->snap) sn.pending = false;  // older than this
    b->applied = b->seq;
    return EK_OK;
}

// Snapshots whose chunk has finished, oldest first; never waits unless
// `wait_one` (then for the older pending one).
int reap_snaps(ek_batch* b, bool wait_one) {
    for (int pass = 0; pass < 2; ++pass) {
        int j = -1;
        for (int q = 0; q < 2; ++q)
            if (b->snap[q].pending && (j < 0 || b->snap[q].seq < b->snap[j].seq)) j = q;
        if (j < 0) return EK_OK;
        ek_batch::Snap& sn = b->snap[j];
        hipError_t e = hipEventQuery(sn.ev);
        if (e == hipErrorNotReady) {
            if (!wait_one) return EK_OK;
            BCHK(b, hipEventSynchronize(sn.ev));
        } else {
            BCHK(b, e);
        }
        wait_one = false;
        if (sn.seq > b->applied) {
            apply_dev(b, sn.host, sn.on_dev, sn.epoch);
            b->applied = sn.seq;
        }
        sn.pending = false;
    }
    return EK_OK;
}

// Graphs replaced while launches of them may still be queued are destroyed
// once an event recorded after their last launch has passed.
void reap_graphs(ek_batch* b, bool all) {
    for (size_t k = 0; k < b->retired.size();) {
        auto& r = b->retired[k];
        if (all || hipEventQuery(r.second) != hipErrorNotReady) {
            (void)hipGraphExecDestroy(r.first);
            (void)hipEventDestroy(r.second);
            b->retired[k] = b->retired.back();
            b->retired.pop_back();
        } else {
            ++k;
        }
    }
}

// Upload the host-owned table, merged into the live one in stream order:
// no wait for the queued steps.
int push_table(ek_batch* b) {
    int n = 0;
    for (int i = 0; i < MAX_SLOTS; ++i)
        if (b->slot[i].used) n = i + 1;
    b->h.nsims = n;
    for (int k = 0; k < KK_N; ++k) b->h.start[k][0] = 0;
    b->refill = false;
    for (int i = 0; i < MAX_SLOTS; ++i) {
        const bool live = i < n && b->slot[i].used && b->h.active[i];
        if (live && !b->h.sims[i].pv) b->refill = true;
        b->h.keep[i] = b->slot[i].used && b->slot[i].on_device ? 1 : 0;
        if (i >= n) continue;
        Grids<float> g = grids_of<float>(b->h.sims[i]);
        for (int k = 0; k < KK_N; ++k) b->h.start[k][i + 1] = b->h.start[k][i] + (live ? g.n[k] : 0);
    }
    if (b->up_pending) {
        BCHK(b, hipEventSynchronize(b->up_ev));  // the staging copy of the last upload is done
        b->up_pending = false;
    }
    std::memcpy((void*)b->hup, (const void*)&b->h, sizeof(BatchTable));
    BCHK(b, hipMemcpyAsync(b->dup, b->hup, sizeof(BatchTable), hipMemcpyHostToDevice, b->stream));
    launch_batch_merge(b->dtab, b->dup, b->stream);
    BCHK(b, hipGetLastError());
    BCHK(b, hipEventRecord(b->up_ev, b->stream));
    b->up_pending = true;
    for (int i = 0; i < n; ++i)
        if (b->slot[i].used) b->slot[i].on_device = true;
    b->dirty = false;
    return EK_OK;
}

void enqueue_batch_step(ek_batch* b, const int* items) {
    launch_batch_particles_pre(b->dtab, items, b->refill, b->stream);
    launch_batch_poisson(b->dtab, items, b->stream);
    launch_batch_particle_forces(b->dtab, items, b->stream);
    launch_batch_fields(b->dtab, items, b->ns, b->stream);
    launch_batch_finish(b->dtab, b->stream);
    launch_batch_flip(b->dtab, b->stream);
}

}  // namespace

extern "C" {

int ek_batch_create(size_t arena_bytes, int n_species, void* stream, void* arena, ek_batch** out) {
    if (!out || n_species < 1 || n_species > EK_MAX_SPECIES || arena_bytes < (size_t)(64 << 20))
        return EK_ERR_INVALID_ARG;
    *out = nullptr;
    ek_batch* b = new (std::nothrow) ek_batch();
    if (!b) return EK_ERR_OOM;
    b->ns = n_species;
    b->bytes = arena_bytes;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return EK_ERR_DEVICE;
        }
        b->own_stream = true;
    }
    if (arena) {
        b->arena = (unsigned char*)arena;
    } else {
        if (hipMalloc(&b->arena, arena_bytes) != hipSuccess) {
            (void)hipGetLastError();
            b->arena = nullptr;
            ek_batch_destroy(b);
            return EK_ERR_OOM;
        }
        b->own_arena = true;
    }
    // the live table, then the device staging of uploads, then the slots
    const size_t tb = (sizeof(BatchTable) + SLOT_ALIGN - 1) & ~(SLOT_ALIGN - 1);
    b->dtab = (BatchTable*)b->arena;
    b->dup = (BatchTable*)(b->arena + tb);
    b->free_ranges[2 * tb] = (arena_bytes - 2 * tb) & ~(SLOT_ALIGN - 1);
    std::memset((void*)&b->h, 0, sizeof(BatchTable));
    bool ok = hipStreamCreateWithFlags(&b->admit_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&b->up_ev, hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc((void**)&b->hup, sizeof(BatchTable), hipHostMallocDefault) == hipSuccess;
    for (auto& sn : b->snap)
        ok = ok && hipEventCreateWithFlags(&sn.ev, hipEventDisableTiming) == hipSuccess &&
             hipHostMalloc((void**)&sn.host, BATCH_DEV_BYTES, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipMemcpy(b->dtab, &b->h, sizeof(BatchTable), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        ek_batch_destroy(b);
        return EK_ERR_DEVICE;
    }
    *out = b;
    return EK_OK;
}

namespace {
struct SeedSpec {
    bool on;
    uint64_t seed;
    double noise;
};

int batch_admit(ek_batch* b, const ek_params* p, const ek_sphere* spheres, int n_spheres,
                const double* initial_density, const SeedSpec& sd, long long n_steps, int* slot) {
    if (!b || !p || (n_spheres > 0 && !spheres) || n_spheres < 0 || n_steps < 0) return EK_ERR_INVALID_ARG;
    if (sd.on && (!std::isfinite(sd.noise) || std::fabs(sd.noise) > 1.0)) return EK_ERR_INVALID_ARG;
    if (b->err) return b->err;
    if (p->precision != EK_FP32_DEV || p->n_species != b->ns) return EK_ERR_INVALID_ARG;
    int i = 0;
    while (i < MAX_SLOTS && b->slot[i].used) ++i;
    if (i == MAX_SLOTS) return EK_ERR_NO_SPACE;
    ek_params q = *p;
    q.max_particles = n_spheres > 0 ? n_spheres : 1;
    q.stream = b->admit_stream;  // built beside the running batch, which is not waited for
    q.arena = nullptr;
    q.arena_bytes = 0;
    size_t need = 0;
    int r = ek_query_footprint(&q, &need);
    if (r) return r;
    size_t off = 0;
    if (!range_alloc(b, need, &off)) return EK_ERR_NO_SPACE;
    q.arena = b->arena + off;
    q.arena_bytes = need;
    ek_ctx* c = nullptr;
    r = ek_create(&q, &c);
    if (r) {
        range_free(b, off, need);
        return r;
    }
    for (int k = 0; k < n_spheres && !r; ++k)
        r = ek_add_sphere(c, spheres[k].x, spheres[k].radius, spheres[k].charge, spheres[k].mass, spheres[k].v,
                          spheres[k].mode, nullptr);
    if (!r && initial_density)
        r = ek_set_fields(c, EK_FIELD_DENSITY, initial_density, (size_t)q.n_species * c->N * sizeof(double));
    else if (!r && sd.on)
        r = ek_seed_density(c, sd.seed, sd.noise);
    if (!r) r = ek_prepare(c);
    if (r) {
        ek_destroy(c);
        range_free(b, off, need);
        return r;
    }
    ek_batch::Slot& s = b->slot[i];
    s.used = true;
    s.on_device = false;
    s.reported = false;
    s.ctx = c;
    s.off = off;
    s.size = need;
    s.cells = c->N;
    s.epoch += 1;
    b->h.sims[i] = c->sf;
    b->h.cur[i] = c->sf.cur;
    b->h.sims[i].status = (uint32_t*)((unsigned char*)b->dtab + offsetof(BatchTable, status)) + i;
    b->h.status[i] = 0;
    b->h.step[i] = 0;
    b->h.target[i] = n_steps;
    b->h.active[i] = n_steps > 0 ? 1 : 0;
    b->dirty = true;
    if (slot) *slot = i;
    return EK_OK;
}
}  // namespace

int ek_batch_admit(ek_batch* b, const ek_params* p, const ek_sphere* spheres, int n_spheres,
                   const double* initial_density, long long n_steps, int* slot) {
    return batch_admit(b, p, spheres, n_spheres, initial_density, SeedSpec{false, 0, 0.0}, n_steps, slot);
}

int ek_batch_admit_seeded(ek_batch* b, const ek_params* p, const ek_sphere* spheres, int n_spheres,
                          uint64_t seed, double noise, long long n_steps, int* slot) {
    return batch_admit(b, p, spheres, n_spheres, nullptr, SeedSpec{true, seed, noise}, n_steps, slot);
}

int ek_batch_step(ek_batch* b, int k) {
    if (!b || k < 0) return EK_ERR_INVALID_ARG;
    if (b->err) return b->err;
    if (b->dirty) {
        int r = push_table(b);
        if (r) return r;
    }
    reap_graphs(b, false);
    // launches sized by work-item totals: capture again when the table's changed
    int items[KK_N];
    bool same = true;
    for (int kk = 0; kk < KK_N; ++kk) {
        items[kk] = b->h.start[kk][b->h.nsims];
        same = same && items[kk] == b->graph_items[kk];
    }
    same = same && b->refill == b->graph_refill;
    if (b->graph && !same) {
        // launches of the old graph may still be queued: destroyed once passed
        hipEvent_t ev = nullptr;
        BCHK(b, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        BCHK(b, hipEventRecord(ev, b->stream));
        b->retired.emplace_back(b->graph, ev);
        b->graph = nullptr;
    }
    if (!b->graph) {
        hipGraph_t g = nullptr;
        BCHK(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        enqueue_batch_step(b, items);
        BCHK(b, hipStreamEndCapture(b->stream, &g));
        hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        BCHK(b, e);
        for (int kk = 0; kk < KK_N; ++kk) b->graph_items[kk] = items[kk];
        b->graph_refill = b->refill;
    }
    if (k == 0) return EK_OK;
    // at most two chunks ahead: the older one's snapshot is waited for (the
    // device still has the newer one to run meanwhile)
    if (b->snap[0].pending && b->snap[1].pending) {
        int r = reap_snaps(b, true);
        if (r) return r;
    }
    for (int i = 0; i < k; ++i) BCHK(b, hipGraphLaunch(b->graph, b->stream));
    ek_batch::Snap& sn = b->snap[b->snap[0].pending ? 1 : 0];
    BCHK(b, hipMemcpyAsync(sn.host, b->dtab, BATCH_DEV_BYTES, hipMemcpyDeviceToHost, b->stream));
    BCHK(b, hipEventRecord(sn.ev, b->stream));
    for (int i = 0; i < MAX_SLOTS; ++i) {
        sn.on_dev[i] = b->slot[i].used && b->slot[i].on_device;
        sn.epoch[i] = b->slot[i].epoch;
    }
    sn.seq = ++b->seq;
    sn.pending = true;
    return EK_OK;
}

int ek_batch_poll(ek_batch* b, int* done_slots, int cap, int* n_done) {
    if (!b || !n_done || (cap > 0 && !done_slots)) return EK_ERR_INVALID_ARG;
    if (b->err) return b->err;
    int r = reap_snaps(b, false);
    if (r) return r;
    int n = 0;
    for (int i = 0; i < MAX_SLOTS; ++i) {
        ek_batch::Slot& s = b->slot[i];
        if (!s.used || s.reported || !s.on_device) continue;
        if (b->h.step[i] >= b->h.target[i] || b->h.status[i] != 0u) {
            if (n < cap) {
                done_slots[n++] = i;
                s.reported = true;
            }
        }
    }
    *n_done = n;
    return EK_OK;
}

int ek_batch_wait(ek_batch* b) {
    if (!b) return EK_ERR_INVALID_ARG;
    if (b->err) return b->err;
    return pull_state(b);
}

int ek_batch_get_fields(ek_batch* b, int slot, int field, void* host, size_t bytes) {
    if (!b || slot < 0 || slot >= MAX_SLOTS || !b->slot[slot].used) return EK_ERR_INVALID_ARG;
    if (b->err) return b->err;
    int r = pull_state(b);
    if (r) return r;
    return ek_get_fields(b->slot[slot].ctx, field, host, bytes);
}

int ek_batch_collect(ek_batch* b, int slot, ek_particle* out, int n, ek_diag* diag) {
    if (!b || slot < 0 || slot >= MAX_SLOTS || !b->slot[slot].used) return EK_ERR_INVALID_ARG;
    if (b->err) return b->err;
    ek_batch::Slot& s = b->slot[slot];
    // A reported slot stopped in a chunk that has finished: its state is
    // final and no queued launch touches it.  Any other is waited for.
    if (!s.reported) {
        int r = pull_state(b);
        if (r) return r;
    }
    // a simulation whose kernels latched an error is retired with that error
    const int failed = s.on_device ? status_error(b->h.status[slot]) : EK_OK;
    if (!failed) {
        int r = EK_OK;
        if (out && n > 0) r = ek_get_particles(s.ctx, out, n);
        if (!r && diag) r = ek_get_diagnostics(s.ctx, diag);
        if (r) return r;
    }
    ek_destroy(s.ctx);
    range_free(b, s.off, s.size);
    const unsigned epoch = s.epoch;
    s = ek_batch::Slot();
    s.epoch = epoch;
    b->h.active[slot] = 0;
    b->h.status[slot] = 0;
    b->dirty = true;
    return failed;
}

int ek_batch_active(ek_batch* b, int* n_active, long long* cells) {
    if (!b) return EK_ERR_INVALID_ARG;
    int n = 0;
    long long c = 0;
    for (int i = 0; i < MAX_SLOTS; ++i)
        if (b->slot[i].used && b->h.active[i]) {
            ++n;
            c += b->slot[i].cells;
        }
    if (n_active) *n_active = n;
    if (cells) *cells = c;
    return EK_OK;
}

int ek_batch_destroy(ek_batch* b) {
    if (!b) return EK_ERR_INVALID_ARG;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (int i = 0; i < MAX_SLOTS; ++i)
        if (b->slot[i].used && b->slot[i].ctx) ek_destroy(b->slot[i].ctx);
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    reap_graphs(b, true);
    for (auto& sn : b->snap) {
        if (sn.ev) (void)hipEventDestroy(sn.ev);
        if (sn.host) (void)hipHostFree(sn.host);
    }
    if (b->up_ev) (void)hipEventDestroy(b->up_ev);
    if (b->hup) (void)hipHostFree(b->hup);
    if (b->admit_stream) (void)hipStreamDestroy(b->admit_stream);
    if (b->own_arena && b->arena) (void)hipFree(b->arena);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return EK_OK;
}

}  // extern "C"
