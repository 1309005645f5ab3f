// ek_poisson.hip -- periodic Poisson solve on the lattice (Eq. poisson; the
// paper uses an FFT-based solver, Sec. III.C).
//
// The charge density q = sum_k z_k rho_k + rho_b is transformed with
// hand-written mixed-radix (4, 2, 3) Stockham FFTs held in LDS, multiplied by
// the Green's function of the 7-point Laplacian, 4 pi lambda_B / K^2 with
// K^2 = sum_d (2 - 2 cos(2 pi k_d / n_d)) and the k = 0 mode set to zero
// (neutralising background), and transformed back.  Five passes over HBM:
//   X  : charge assembly + real-to-half-complex FFT along x.  Two real rows
//        (y, y+1) form one complex sequence; their spectra are separated by
//        Hermitian symmetry.  Writes the half spectrum S[z][y][kx].
//   Y  : complex FFT along y of tiles of consecutive kx (coalesced rows).
//   Z  : complex FFT along z, Green's function (with the 1/N scale), inverse
//        FFT along z, all in LDS.
//   Y' : inverse FFT along y.
//   X' : inverse half-complex-to-real FFT along x (two rows at a time) -> phi.
// On the FP32 path the densities are deviations from their means; the
// constant sum_k z_k mean_k only feeds the k = 0 mode, which is dropped.
#include "ek_internal.h"

namespace ek {

constexpr int FT = 256;  // threads per FFT workgroup

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

template <typename T>
using cpx = typename V2<T>::t;

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    cpx<T> r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) {
    cpx<T> r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) {
    cpx<T> r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> mk(T x, T y) {
    cpx<T> r;
    r.x = x;
    r.y = y;
    return r;
}

struct Plan {
    int nst;
    int r[10];
};

__device__ __forceinline__ Plan make_plan(int n) {
    Plan p;
    p.nst = 0;
    while (n % 4 == 0) { p.r[p.nst++] = 4; n /= 4; }
    while (n % 2 == 0) { p.r[p.nst++] = 2; n /= 2; }
    while (n % 3 == 0) { p.r[p.nst++] = 3; n /= 3; }
    return p;
}

// FFT of P pencils of length n stored contiguously (pencil-major) in LDS
// buffer a, using b as scratch.  Returns the buffer holding the result.
// Forward uses e^{-2 pi i m / n} from tw; INV uses the conjugate.
template <typename T, bool INV>
__device__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, int n, int P, const cpx<T>* __restrict__ tw) {
    Plan pl = make_plan(n);
    int Ns = 1;
    for (int st = 0; st < pl.nst; ++st) {
        int R = pl.r[st];
        int nR = n / R;
        int span = n / (Ns * R);
        for (int t = threadIdx.x; t < P * nR; t += blockDim.x) {
            int pen = t / nR, j = t - pen * nR;
            int k = j % Ns;
            const cpx<T>* src = a + pen * n;
            cpx<T>* dst = b + pen * n;
            cpx<T> v[4];
            for (int r = 0; r < R; ++r) {
                cpx<T> x = src[j + r * nR];
                if (r > 0 && k > 0) {
                    cpx<T> w = tw[k * r * span];
                    if (INV) w.y = -w.y;
                    x = cmul<T>(x, w);
                }
                v[r] = x;
            }
            cpx<T> o[4];
            if (R == 2) {
                o[0] = cadd<T>(v[0], v[1]);
                o[1] = csub<T>(v[0], v[1]);
            } else if (R == 4) {
                cpx<T> s02 = cadd<T>(v[0], v[2]), d02 = csub<T>(v[0], v[2]);
                cpx<T> s13 = cadd<T>(v[1], v[3]), d13 = csub<T>(v[1], v[3]);
                // -i * d13 (forward) or +i * d13 (inverse)
                cpx<T> rot = INV ? mk<T>(-d13.y, d13.x) : mk<T>(d13.y, -d13.x);
                o[0] = cadd<T>(s02, s13);
                o[2] = csub<T>(s02, s13);
                o[1] = cadd<T>(d02, rot);
                o[3] = csub<T>(d02, rot);
            } else {  // R == 3
                const T c3 = (T)-0.5;
                const T s3 = INV ? (T)0.86602540378443864676 : (T)-0.86602540378443864676;
                cpx<T> s12 = cadd<T>(v[1], v[2]), d12 = csub<T>(v[1], v[2]);
                o[0] = cadd<T>(v[0], s12);
                cpx<T> m = mk<T>(v[0].x + c3 * s12.x, v[0].y + c3 * s12.y);
                cpx<T> j = mk<T>(-s3 * d12.y, s3 * d12.x);  // i * s3 * d12
                o[1] = cadd<T>(m, j);
                o[2] = csub<T>(m, j);
            }
            int idxD = (j / Ns) * Ns * R + k;
            for (int r = 0; r < R; ++r) dst[idxD + r * Ns] = o[r];
        }
        __syncthreads();
        cpx<T>* tmp = a;
        a = b;
        b = tmp;
        Ns *= R;
    }
    return a;
}

// ---------------------------------------------------------------------------
// Pass X (forward): charge assembly + two-for-one real FFT along x.
// Work item: a pair of rows (y, y+1) at one z.  P pairs per workgroup.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(FT) void k_fft_x_fwd(Sim<T> s, int P) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* a = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* b = a + P * s.nx;
    const int n = s.nx;
    const int npairs = s.ny * s.nz / 2;
    const int pair0 = blockIdx.x * P;
    const T* rho = s.rho[s.cur];
    for (int t = threadIdx.x; t < P * n; t += FT) {
        int pen = t / n, x = t - pen * n;
        int pr = pair0 + pen;
        cpx<T> v = mk<T>(0, 0);
        if (pr < npairs) {
            int row = 2 * pr;  // row = y + ny*z with y even
            long c0 = (long)row * n + x, c1 = c0 + n;
            T q0 = s.rhob[c0], q1 = s.rhob[c1];
            for (int k = 0; k < s.ns; ++k) {
                T zk = (T)s.z[k];
                q0 += zk * rho[(long)k * s.N + c0];
                q1 += zk * rho[(long)k * s.N + c1];
            }
            v = mk<T>(q0, q1);
        }
        a[t] = v;
    }
    __syncthreads();
    cpx<T>* r = fft_lds<T, false>(a, b, n, P, reinterpret_cast<const cpx<T>*>(s.tw[0]));
    cpx<T>* S = reinterpret_cast<cpx<T>*>(s.spec);
    const int nh = s.nxh;
    for (int t = threadIdx.x; t < P * nh; t += FT) {
        int pen = t / nh, k = t - pen * nh;
        int pr = pair0 + pen;
        if (pr >= npairs) continue;
        cpx<T> A = r[pen * n + k];
        cpx<T> B = r[pen * n + (k == 0 ? 0 : n - k)];
        // Q1 = (A + conj B)/2, Q2 = (A - conj B)/(2i)
        cpx<T> q1 = mk<T>((T)0.5 * (A.x + B.x), (T)0.5 * (A.y - B.y));
        cpx<T> q2 = mk<T>((T)0.5 * (A.y + B.y), (T)-0.5 * (A.x - B.x));
        long row = 2 * pr;
        S[row * nh + k] = q1;
        S[(row + 1) * nh + k] = q2;
    }
}

// ---------------------------------------------------------------------------
// Pass X' (inverse): two half spectra -> one complex sequence -> two real rows.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(FT) void k_fft_x_inv(Sim<T> s, int P) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* a = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* b = a + P * s.nx;
    const int n = s.nx;
    const int nh = s.nxh;
    const int npairs = s.ny * s.nz / 2;
    const int pair0 = blockIdx.x * P;
    const cpx<T>* S = reinterpret_cast<const cpx<T>*>(s.spec);
    for (int t = threadIdx.x; t < P * n; t += FT) {
        int pen = t / n, k = t - pen * n;
        int pr = pair0 + pen;
        cpx<T> v = mk<T>(0, 0);
        if (pr < npairs) {
            long row = 2 * pr;
            if (k < nh) {
                cpx<T> q1 = S[row * nh + k], q2 = S[(row + 1) * nh + k];
                v = mk<T>(q1.x - q2.y, q1.y + q2.x);  // q1 + i q2
            } else {
                cpx<T> q1 = S[row * nh + (n - k)], q2 = S[(row + 1) * nh + (n - k)];
                v = mk<T>(q1.x + q2.y, -q1.y + q2.x);  // conj(q1) + i conj(q2)
            }
        }
        a[t] = v;
    }
    __syncthreads();
    cpx<T>* r = fft_lds<T, true>(a, b, n, P, reinterpret_cast<const cpx<T>*>(s.tw[0]));
    for (int t = threadIdx.x; t < P * n; t += FT) {
        int pen = t / n, x = t - pen * n;
        int pr = pair0 + pen;
        if (pr >= npairs) continue;
        long c0 = (long)(2 * pr) * n + x;
        s.phi[c0] = r[t].x;
        s.phi[c0 + n] = r[t].y;
    }
}

// ---------------------------------------------------------------------------
// Pass Y (forward or inverse): pencils along y, TX consecutive kx per group.
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__global__ __launch_bounds__(FT) void k_fft_y(Sim<T> s, int TX) {
    extern __shared__ unsigned char smem_raw[];
    const int n = s.ny, nh = s.nxh;
    cpx<T>* a = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* b = a + TX * n;
    int tiles = (nh + TX - 1) / TX;
    int z = blockIdx.x / tiles;
    int kx0 = (blockIdx.x - z * tiles) * TX;
    cpx<T>* S = reinterpret_cast<cpx<T>*>(s.spec) + (long)z * n * nh;
    for (int t = threadIdx.x; t < TX * n; t += FT) {
        int y = t / TX, i = t - y * TX;
        int kx = kx0 + i;
        a[i * n + y] = kx < nh ? S[(long)y * nh + kx] : mk<T>(0, 0);
    }
    __syncthreads();
    cpx<T>* r = fft_lds<T, INV>(a, b, n, TX, reinterpret_cast<const cpx<T>*>(s.tw[1]));
    for (int t = threadIdx.x; t < TX * n; t += FT) {
        int y = t / TX, i = t - y * TX;
        int kx = kx0 + i;
        if (kx < nh) S[(long)y * nh + kx] = r[i * n + y];
    }
}

// ---------------------------------------------------------------------------
// Pass Z: forward FFT along z, multiply by the Green's function, inverse FFT.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(FT) void k_fft_z_green(Sim<T> s, int TX) {
    extern __shared__ unsigned char smem_raw[];
    const int n = s.nz, nh = s.nxh, ny = s.ny;
    cpx<T>* a = reinterpret_cast<cpx<T>*>(smem_raw);
    cpx<T>* b = a + TX * n;
    int tiles = (nh + TX - 1) / TX;
    int ky = blockIdx.x / tiles;
    int kx0 = (blockIdx.x - ky * tiles) * TX;
    cpx<T>* S = reinterpret_cast<cpx<T>*>(s.spec);
    const long zstride = (long)ny * nh;
    for (int t = threadIdx.x; t < TX * n; t += FT) {
        int z = t / TX, i = t - z * TX;
        int kx = kx0 + i;
        a[i * n + z] = kx < nh ? S[z * zstride + (long)ky * nh + kx] : mk<T>(0, 0);
    }
    __syncthreads();
    cpx<T>* r = fft_lds<T, false>(a, b, n, TX, reinterpret_cast<const cpx<T>*>(s.tw[2]));
    cpx<T>* o = (r == a) ? b : a;
    const T scale = (T)(4.0 * 3.14159265358979323846 * s.lambda_B / (double)s.N);
    for (int t = threadIdx.x; t < TX * n; t += FT) {
        int i = t / n, kz = t - i * n;
        int kx = kx0 + i;
        T g = 0;
        if (kx < nh) {
            T K2 = s.k2[0][kx] + s.k2[1][ky] + s.k2[2][kz];
            g = (kx == 0 && ky == 0 && kz == 0) ? (T)0 : scale / K2;
        }
        cpx<T> v = r[t];
        o[t] = mk<T>(v.x * g, v.y * g);
    }
    __syncthreads();
    cpx<T>* q = fft_lds<T, true>(o, r, n, TX, reinterpret_cast<const cpx<T>*>(s.tw[2]));
    for (int t = threadIdx.x; t < TX * n; t += FT) {
        int z = t / TX, i = t - z * TX;
        int kx = kx0 + i;
        if (kx < nh) S[z * zstride + (long)ky * nh + kx] = q[i * n + z];
    }
}

template <typename T>
static int pencils_x(int n) {
    int P = 1024 / n;
    return P < 1 ? 1 : P;
}

// Consecutive kx columns per workgroup in the y and z passes: 16 (FP32) or 8
// (FP64) for coalesced 128-byte rows, fewer for long pencils so that the two
// LDS buffers stay within 64 KB.
template <typename T>
static int tile_kx(int n) {
    int cap = (int)(32768 / sizeof(cpx<T>)) / n;
    int t = sizeof(T) == 4 ? 16 : 8;
    return t < cap ? t : cap;
}

template <typename T>
void launch_charge_poisson(const Sim<T>& s, hipStream_t st) {
    const size_t cs = sizeof(cpx<T>);
    int P = pencils_x<T>(s.nx);
    int npairs = s.ny * s.nz / 2;
    int gx = (npairs + P - 1) / P;
    size_t shx = 2 * (size_t)P * s.nx * cs;
    hipLaunchKernelGGL(k_fft_x_fwd<T>, dim3(gx), dim3(FT), shx, st, s, P);
    int TXy = tile_kx<T>(s.ny), TXz = tile_kx<T>(s.nz);
    int tiles_y = (s.nxh + TXy - 1) / TXy, tiles_z = (s.nxh + TXz - 1) / TXz;
    size_t shy = 2 * (size_t)TXy * s.ny * cs;
    hipLaunchKernelGGL((k_fft_y<T, false>), dim3(tiles_y * s.nz), dim3(FT), shy, st, s, TXy);
    size_t shz = 2 * (size_t)TXz * s.nz * cs;
    hipLaunchKernelGGL(k_fft_z_green<T>, dim3(tiles_z * s.ny), dim3(FT), shz, st, s, TXz);
    hipLaunchKernelGGL((k_fft_y<T, true>), dim3(tiles_y * s.nz), dim3(FT), shy, st, s, TXy);
    hipLaunchKernelGGL(k_fft_x_inv<T>, dim3(gx), dim3(FT), shx, st, s, P);
}

template void launch_charge_poisson<float>(const Sim<float>&, hipStream_t);
template void launch_charge_poisson<double>(const Sim<double>&, hipStream_t);

}  // namespace ek
