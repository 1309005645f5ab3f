// ek_util.hip -- fills and FP64 global reductions (diagnostics).
//
// The diagnostics are deterministic two-stage sums: each workgroup reduces a
// fixed strided subset of cells in a fixed order, then one workgroup adds the
// partial sums in workgroup order.
#include "ek_internal.h"

namespace ek {

constexpr int UT = 256;

template <typename T>
__global__ void k_fill(T* p, long n, T v) {
    for (long i = (long)blockIdx.x * UT + threadIdx.x; i < n; i += (long)gridDim.x * UT) p[i] = v;
}

template <typename T>
void fill(T* p, long n, T v, hipStream_t st) {
    if (n <= 0) return;
    long blocks = (n + UT - 1) / UT;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(UT), 0, st, p, n, v);
}
// Rest-state populations in the blocked layout: f = w_i (FP64 plain) or 0 (FP32
// deviations) over n_pad cells.
template <typename T>
__global__ void k_fill_pops(T* f, long npad, bool dev) {
    const long e = (long)blockIdx.x * UT + threadIdx.x;
    if (e >= 19 * npad) return;
    const int i = (int)((e / FB) % 19);
    f[e] = dev ? (T)0 : (T)q19w(i);
}

template <typename T>
void fill_pops(T* f, long npad, bool dev, hipStream_t st) {
    long blocks = (19 * npad + UT - 1) / UT;
    hipLaunchKernelGGL(k_fill_pops<T>, dim3((unsigned)blocks), dim3(UT), 0, st, f, npad, dev);
}
// splitmix64 finaliser (Steele, Lea and Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Counter stream (seed, k, cell): U = (splitmix64(cell ^ seed ^ k << 40) >> 11)
// 2^-53, exact in FP64; the density is formed with one rounding per operation
// in the order written (no contraction), so the stored values are the ones
// the host conversion gives for the same formula evaluated in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_seed_density(Sim<T> s, SeedArgs a) {
#pragma clang fp contract(off)
    const long c = (long)blockIdx.x * 256 + threadIdx.x;
    if (c >= s.N) return;
    for (int k = 0; k < s.ns; ++k) {
        const uint64_t key = a.seed ^ ((uint64_t)k << 40);
        const double u = (double)(splitmix64((uint64_t)c ^ key) >> 11) * 0x1p-53;
        const double v = a.mean[k] * (1.0 + a.noise * (2.0 * u - 1.0));
        s.rho[s.cur][(long)k * s.N + c] = (T)(v / a.fac - (sizeof(T) == 4 ? s.rho_ref[k] : 0.0));
    }
}

template <typename T>
void launch_seed_density(const Sim<T>& s, const SeedArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_seed_density<T>, dim3((unsigned)((s.N + 255) / 256)), dim3(256), 0, st, s, a);
}
template void launch_seed_density<float>(const Sim<float>&, const SeedArgs&, hipStream_t);
template void launch_seed_density<double>(const Sim<double>&, const SeedArgs&, hipStream_t);

template void fill_pops<float>(float*, long, bool, hipStream_t);
template void fill_pops<double>(double*, long, bool, hipStream_t);

template void fill<float>(float*, long, float, hipStream_t);
template void fill<double>(double*, long, double, hipStream_t);
template void fill<uint8_t>(uint8_t*, long, uint8_t, hipStream_t);
template void fill<uint16_t>(uint16_t*, long, uint16_t, hipStream_t);

template <typename T>
__global__ __launch_bounds__(UT) void k_diag_stage1(Sim<T> s) {
    constexpr bool DEV = sizeof(T) == 4;
    double acc[NDIAG];
    for (int k = 0; k < NDIAG; ++k) acc[k] = 0.0;
    const T* f = s.f[s.cur];
    const T* rho = s.rho[s.cur];
    for (long c = (long)blockIdx.x * UT + threadIdx.x; c < s.N; c += (long)gridDim.x * UT) {
        for (int k = 0; k < s.ns; ++k)
            acc[k] += (DEV ? s.rho_ref[k] : 0.0) + (double)rho[(long)k * s.N + c];
        acc[MAXS] += (double)s.rhob[c];
        if (s.flag[c] & F_CUR) {
            acc[MAXS + 5] += 1.0;
            continue;
        }
        double m = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        sfor<19>([&](auto I) {
            constexpr int i = I;
            double fi = (DEV ? q19w(i) : 0.0) + (double)f[fidx(i, c)];
            m += fi;
            jx += fi * q19x(i);
            jy += fi * q19y(i);
            jz += fi * q19z(i);
        });
        acc[MAXS + 1] += m;
        acc[MAXS + 2] += jx;
        acc[MAXS + 3] += jy;
        acc[MAXS + 4] += jz;
        const T* u = s.u[s.cur] + vidx(0, c);
        double ux = u[0], uy = u[FB], uz = u[2 * FB];
        double um = sqrt(ux * ux + uy * uy + uz * uz);
        acc[MAXS + 6] = um > acc[MAXS + 6] ? um : acc[MAXS + 6];
    }
    __shared__ double part[NDIAG][UT / 64];
    int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < NDIAG; ++k) {
        double x = acc[k];
        for (int off = 32; off > 0; off >>= 1) {
            double y = __shfl_xor(x, off);
            x = (k == MAXS + 6) ? (y > x ? y : x) : x + y;
        }
        if (lane == 0) part[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < NDIAG) {
        int k = threadIdx.x;
        double x = part[k][0];
        for (int w = 1; w < UT / 64; ++w) x = (k == MAXS + 6) ? (part[k][w] > x ? part[k][w] : x) : x + part[k][w];
        s.scratch[(long)blockIdx.x * NDIAG + k] = x;
    }
}

__global__ void k_diag_stage2(const double* part, int nblocks, double* out) {
    int k = threadIdx.x;
    if (k >= NDIAG) return;
    double x = part[k];
    for (int b = 1; b < nblocks; ++b) {
        double y = part[(long)b * NDIAG + k];
        x = (k == MAXS + 6) ? (y > x ? y : x) : x + y;
    }
    out[k] = x;
}

template <typename T>
void launch_diagnostics(const Sim<T>& s, hipStream_t st, double* out) {
    long blocks = (s.N + UT - 1) / UT;
    if (blocks > DIAG_BLOCKS) blocks = DIAG_BLOCKS;
    hipLaunchKernelGGL(k_diag_stage1<T>, dim3((unsigned)blocks), dim3(UT), 0, st, s);
    hipLaunchKernelGGL(k_diag_stage2, dim3(1), dim3(64), 0, st, (const double*)s.scratch, (int)blocks, out);
}
template void launch_diagnostics<float>(const Sim<float>&, hipStream_t, double*);
template void launch_diagnostics<double>(const Sim<double>&, hipStream_t, double*);

// Plain streaming copy (bandwidth probe): each lane moves four independent
// 16-byte vectors per iteration; the tail is copied one vector at a time.
__global__ __launch_bounds__(UT) void k_copy16(float4* __restrict__ dst, const float4* __restrict__ src, long n) {
    const long i = (long)blockIdx.x * UT + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// One 16-byte element per thread over an exact grid (measured faster on
// gfx950 than grid-stride loops with several elements per thread).
void launch_copy16(void* dst, const void* src, long n16, hipStream_t st) {
    if (n16 <= 0) return;
    const long blocks = (n16 + UT - 1) / UT;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(UT), 0, st, (float4*)dst, (const float4*)src, n16);
}

// End of a batched step: every active slot toggles its ping-pong buffers and
// counts the step; a slot that reached its requested steps, or whose kernels
// latched an error status, stops.
__global__ void k_batch_flip(BatchTable* tab) {
    int i = threadIdx.x;
    if (i >= tab->nsims || !tab->active[i]) return;
    tab->sims[i].cur ^= 1;
    tab->cur[i] = tab->sims[i].cur;
    long long st = tab->step[i] + 1;
    tab->step[i] = st;
    if (st >= tab->target[i] || tab->status[i] != 0u) tab->active[i] = 0;
}

void launch_batch_flip(BatchTable* tab, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_flip, dim3(1), dim3(MAX_SLOTS), 0, st, tab);
}

// An uploaded table into the live one, in stream order behind the steps
// already queued: the host-owned part is taken whole; the device-owned
// entries of a slot are taken from the upload only when it does not keep
// them (a slot new since the last upload, or freed).
__global__ void k_batch_merge(BatchTable* tab, const BatchTable* up) {
    const uint32_t* src = (const uint32_t*)((const unsigned char*)up + BATCH_DEV_BYTES);
    uint32_t* dst = (uint32_t*)((unsigned char*)tab + BATCH_DEV_BYTES);
    constexpr int NW = (int)((sizeof(BatchTable) - BATCH_DEV_BYTES) / 4);
    for (int w = threadIdx.x; w < NW; w += blockDim.x) dst[w] = src[w];
    __syncthreads();
    for (int i = threadIdx.x; i < MAX_SLOTS; i += blockDim.x) {
        if (!up->keep[i]) {
            tab->active[i] = up->active[i];
            tab->cur[i] = up->cur[i];
            tab->status[i] = up->status[i];
            tab->step[i] = up->step[i];
        }
        tab->sims[i].cur = tab->cur[i];
    }
}

void launch_batch_merge(BatchTable* tab, const BatchTable* upload, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_merge, dim3(1), dim3(256), 0, st, tab, upload);
}

}  // namespace ek
