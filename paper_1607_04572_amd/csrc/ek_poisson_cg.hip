// ek_poisson_cg.hip -- Poisson's equation with an inhomogeneous relative
// permittivity eps (Sec. III.C: the FFT solver assumes a homogeneous
// dielectric; iterative solvers take a varying one), on the periodic lattice:
//   sum over the 6 faces f of c: e_f (phi_c - phi_n) = 4 pi lambda_B (q_c - mean q),
// e_f the harmonic mean of the two cells' permittivities.  The operator L on
// the left is symmetric positive semi-definite (constants span its null
// space) and the right side has zero mean, so Jacobi-preconditioned conjugate
// gradients converge; the solution is shifted to zero mean at the end.
//
// FP64 throughout, whatever the storage precision of the fields.  Every
// global dot product is a two-stage sum in a fixed order (deterministic).
// One iteration: q = L p with p.q; alpha; x += alpha p, r -= alpha q with
// r.z and r.r (z = r / diag); beta; p = z + beta p.  The host reads r.r every
// few iterations and stops at r.r <= tol^2 b.b.
#include <cmath>

#include "ek_internal.h"

namespace ek {

constexpr int CGT = 256;          // threads per workgroup
constexpr int CG_BLOCKS = 1024;   // workgroups of the grid-stride kernels (partial sums per dot product)
enum { SC_QSUM, SC_RZ, SC_RR, SC_BB, SC_ALPHA, SC_BETA, SC_XSUM, SC_N };

// Per-workgroup sum of up to three values (fixed order: shuffles, then waves).
template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* part) {
    __shared__ double w[K][CGT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) w[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double x = 0.0;
        for (int i = 0; i < CGT / 64; ++i) x += w[threadIdx.x][i];
        part[(long)blockIdx.x * 4 + threadIdx.x] = x;
    }
}

// Sum of K partial columns over the workgroups, in workgroup order (one wave).
template <int K>
__device__ __forceinline__ void partial_total(const CGState& g, double (&out)[K]) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double x = 0.0;
        for (int b = lane; b < CG_BLOCKS; b += 64) x += g.part[(long)b * 4 + k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        out[k] = x;
    }
}

__device__ __forceinline__ long cg_nbr(const CGState& g, long c, int x, int y, int z, int d, int dir) {
    // index of the neighbour of (x, y, z) along axis d in direction dir (+1/-1), periodic
    if (d == 0) {
        const int xn = dir > 0 ? (x + 1 == g.nx ? 0 : x + 1) : (x == 0 ? g.nx - 1 : x - 1);
        return c + (xn - x);
    }
    if (d == 1) {
        const int yn = dir > 0 ? (y + 1 == g.ny ? 0 : y + 1) : (y == 0 ? g.ny - 1 : y - 1);
        return c + (long)(yn - y) * g.nx;
    }
    const int zn = dir > 0 ? (z + 1 == g.nz ? 0 : z + 1) : (z == 0 ? g.nz - 1 : z - 1);
    return c + (long)(zn - z) * g.nx * g.ny;
}

// (L v)_c = sum over faces e_f (v_c - v_n); ef[d][c] is the face between c and c + e_d.
__device__ __forceinline__ double cg_apply(const CGState& g, const double* v, long c) {
    const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((long)g.nx * g.ny));
    const double vc = v[c];
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const long cp = cg_nbr(g, c, x, y, z, d, +1), cm = cg_nbr(g, c, x, y, z, d, -1);
        s += g.ef[d][c] * (vc - v[cp]);
        s += g.ef[d][cm] * (vc - v[cm]);
    }
    return s;
}

// Face coefficients (harmonic means) and the inverse diagonal.
__global__ __launch_bounds__(CGT) void k_cg_faces(CGState g, const double* __restrict__ eps) {
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT) {
        const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((long)g.nx * g.ny));
        for (int d = 0; d < 3; ++d) {
            const long cp = cg_nbr(g, c, x, y, z, d, +1);
            const double a = eps[c], b = eps[cp];
            g.ef[d][c] = 2.0 * a * b / (a + b);
        }
    }
}
__global__ __launch_bounds__(CGT) void k_cg_diag(CGState g) {
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT) {
        const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((long)g.nx * g.ny));
        double s = 0.0;
        for (int d = 0; d < 3; ++d) s += g.ef[d][c] + g.ef[d][cg_nbr(g, c, x, y, z, d, -1)];
        g.idiag[c] = 1.0 / s;
    }
}

// Charge q = sum_k z_k rho_k + rho_b into r, and its per-workgroup sums.
template <typename T>
__global__ __launch_bounds__(CGT) void k_cg_charge(Sim<T> s, CGState g) {
    constexpr bool DEV = sizeof(T) == 4;
    const T* rho = s.rho[s.cur];
    double acc[1] = {0.0};
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT) {
        double q = (double)s.rhob[c];
        for (int k = 0; k < s.ns; ++k) q += s.z[k] * ((DEV ? s.rho_ref[k] : 0.0) + (double)rho[(long)k * s.N + c]);
        g.r[c] = q;
        acc[0] += q;
    }
    block_sums<1>(acc, g.part);
}

__global__ void k_cg_total_q(CGState g) {
    double t[1];
    partial_total<1>(g, t);
    if (threadIdx.x == 0) g.sc[SC_QSUM] = t[0];
}

// b = 4 pi lambda_B (q - mean q); r = b - L x; z = r / diag; p = z; r.z, r.r, b.b.
__global__ __launch_bounds__(CGT) void k_cg_init(CGState g) {
    const double mean = g.sc[SC_QSUM] / (double)g.N;
    double acc[3] = {0.0, 0.0, 0.0};
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT) {
        const double b = g.fourpi_lb * (g.r[c] - mean);
        const double r = b - cg_apply(g, g.x, c);
        const double z = r * g.idiag[c];
        g.r[c] = r;
        g.p[c] = z;
        acc[0] += r * z;
        acc[1] += r * r;
        acc[2] += b * b;
    }
    block_sums<3>(acc, g.part);
}
__global__ void k_cg_total_init(CGState g) {
    double t[3];
    partial_total<3>(g, t);
    if (threadIdx.x == 0) {
        g.sc[SC_RZ] = t[0];
        g.sc[SC_RR] = t[1];
        g.sc[SC_BB] = t[2];
    }
}

// q = L p and p.q
__global__ __launch_bounds__(CGT) void k_cg_ap(CGState g) {
    double acc[1] = {0.0};
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT) {
        const double q = cg_apply(g, g.p, c);
        g.q[c] = q;
        acc[0] += g.p[c] * q;
    }
    block_sums<1>(acc, g.part);
}
__global__ void k_cg_alpha(CGState g) {
    double t[1];
    partial_total<1>(g, t);
    if (threadIdx.x == 0) g.sc[SC_ALPHA] = t[0] > 0.0 ? g.sc[SC_RZ] / t[0] : 0.0;
}

// x += alpha p; r -= alpha q; r.z, r.r
__global__ __launch_bounds__(CGT) void k_cg_update(CGState g) {
    const double alpha = g.sc[SC_ALPHA];
    double acc[2] = {0.0, 0.0};
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT) {
        g.x[c] += alpha * g.p[c];
        const double r = g.r[c] - alpha * g.q[c];
        g.r[c] = r;
        acc[0] += r * (r * g.idiag[c]);
        acc[1] += r * r;
    }
    block_sums<2>(acc, g.part);
}
__global__ void k_cg_beta(CGState g) {
    double t[2];
    partial_total<2>(g, t);
    if (threadIdx.x == 0) {
        const double rz = g.sc[SC_RZ];
        g.sc[SC_BETA] = rz > 0.0 ? t[0] / rz : 0.0;
        g.sc[SC_RZ] = t[0];
        g.sc[SC_RR] = t[1];
    }
}

// p = r / diag + beta p
__global__ __launch_bounds__(CGT) void k_cg_dir(CGState g) {
    const double beta = g.sc[SC_BETA];
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT)
        g.p[c] = g.r[c] * g.idiag[c] + beta * g.p[c];
}

// mean of x, then phi = x - mean (and x shifted, the next step's start)
__global__ __launch_bounds__(CGT) void k_cg_xsum(CGState g) {
    double acc[1] = {0.0};
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT) acc[0] += g.x[c];
    block_sums<1>(acc, g.part);
}
__global__ void k_cg_total_x(CGState g) {
    double t[1];
    partial_total<1>(g, t);
    if (threadIdx.x == 0) g.sc[SC_XSUM] = t[0];
}
template <typename T>
__global__ __launch_bounds__(CGT) void k_cg_out(Sim<T> s, CGState g) {
    const double mean = g.sc[SC_XSUM] / (double)g.N;
    for (long c = (long)blockIdx.x * CGT + threadIdx.x; c < g.N; c += (long)gridDim.x * CGT) {
        const double v = g.x[c] - mean;
        g.x[c] = v;
        s.phi[c] = (T)v;
    }
}

static unsigned cg_grid(long N) {
    const long b = (N + CGT - 1) / CGT;
    return (unsigned)(b < CG_BLOCKS ? b : CG_BLOCKS);
}

// Every block writes its partial row, including blocks with no cells, since
// the totals read all CG_BLOCKS rows: launch exactly CG_BLOCKS workgroups.
int cg_setup(const CGState& g, const double* eps_dev, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_faces, dim3(cg_grid(g.N)), dim3(CGT), 0, st, g, eps_dev);
    hipLaunchKernelGGL(k_cg_diag, dim3(cg_grid(g.N)), dim3(CGT), 0, st, g);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int cg_solve(const Sim<T>& s, CGState& g, hipStream_t st, int* iters, double* rel_res) {
    const dim3 G(CG_BLOCKS), B(CGT);
    hipLaunchKernelGGL(k_cg_charge<T>, G, B, 0, st, s, g);
    hipLaunchKernelGGL(k_cg_total_q, dim3(1), dim3(64), 0, st, g);
    hipLaunchKernelGGL(k_cg_init, G, B, 0, st, g);
    hipLaunchKernelGGL(k_cg_total_init, dim3(1), dim3(64), 0, st, g);
    int it = 0;
    double h[SC_N] = {};
    for (;;) {
        // convergence check every CHECK iterations (one small copy and a wait)
        if (it % CG_CHECK == 0 || it >= g.max_iter) {
            if (hipMemcpyAsync(h, g.sc, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return -1;
            if (h[SC_RR] <= g.tol * g.tol * h[SC_BB] || it >= g.max_iter) break;
        }
        hipLaunchKernelGGL(k_cg_ap, G, B, 0, st, g);
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64), 0, st, g);
        hipLaunchKernelGGL(k_cg_update, G, B, 0, st, g);
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, st, g);
        hipLaunchKernelGGL(k_cg_dir, G, B, 0, st, g);
        ++it;
    }
    hipLaunchKernelGGL(k_cg_xsum, G, B, 0, st, g);
    hipLaunchKernelGGL(k_cg_total_x, dim3(1), dim3(64), 0, st, g);
    hipLaunchKernelGGL(k_cg_out<T>, G, B, 0, st, s, g);
    *iters = it;
    *rel_res = h[SC_BB] > 0.0 ? std::sqrt(h[SC_RR] / h[SC_BB]) : 0.0;
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int cg_solve<float>(const Sim<float>&, CGState&, hipStream_t, int*, double*);
template int cg_solve<double>(const Sim<double>&, CGState&, hipStream_t, int*, double*);

}  // namespace ek
