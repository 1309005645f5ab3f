// ek_poisson.hip -- periodic Poisson solve on the lattice (Eq. poisson; the
// paper uses an FFT-based solver, Sec. III.C).
//
// The charge density q = sum_k z_k rho_k + rho_b is transformed with
// hand-written Stockham FFTs held in LDS (radix 8 with compile-time plans for
// the power-of-two lengths 32-512 and for 48 and 96, a run-time mixed-radix
// (4, 2, 3) plan for the others), multiplied by
// the Green's function of the 7-point Laplacian, 4 pi lambda_B / K^2 with
// K^2 = sum_d (2 - 2 cos(2 pi k_d / n_d)) and the k = 0 mode set to zero
// (neutralising background), and transformed back.  Five passes over HBM:
//   X  : charge assembly + real-to-half-complex FFT along x.  Two real rows
//        (y, y+1) form one complex sequence; their spectra are separated by
//        Hermitian symmetry.  Writes the half spectrum S[z][y][kx] (row stride
//        nxs >= nx/2 + 1, whole 128-byte lines).
//   Y  : complex FFT along y of tiles of consecutive kx (coalesced rows).
//   Z  : complex FFT along z, Green's function (with the 1/N scale), inverse
//        FFT along z, all in LDS.
//   Y' : inverse FFT along y.
//   X' : inverse half-complex-to-real FFT along x (two rows at a time) -> phi.
// On the FP32 path the densities are deviations from their means; the
// constant sum_k z_k mean_k only feeds the k = 0 mode, which is dropped.
#include "ek_internal.h"

namespace ek {

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

// Complex elements to and from global memory as native two-element vectors
// (the HIP vector types are classes that do not copy across address spaces).
template <typename T>
__device__ __forceinline__ cpx<T> gld_c(const cpx<T>* p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 v = *(const gmem<v2>*)p;
    return mk<T>(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void gst_c(cpx<T>* p, cpx<T> v) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 w;
    w.x = v.x;
    w.y = v.y;
    *(gmem<v2>*)p = w;
}
__device__ __forceinline__ float2 gld(const float2* p) { return gld_c<float>(p); }
__device__ __forceinline__ double2 gld(const double2* p) { return gld_c<double>(p); }
__device__ __forceinline__ void gst(float2* p, float2 v) { gst_c<float>(p, v); }
__device__ __forceinline__ void gst(double2* p, double2 v) { gst_c<double>(p, v); }

// Radix-R DFT of v[0..R) in registers (forward: e^{-2 pi i qm/R}).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_small(cpx<T> (&v)[R]) {
    if constexpr (R == 2) {
        cpx<T> a = cadd<T>(v[0], v[1]), b = csub<T>(v[0], v[1]);
        v[0] = a;
        v[1] = b;
    } else if constexpr (R == 4) {
        cpx<T> s02 = cadd<T>(v[0], v[2]), d02 = csub<T>(v[0], v[2]);
        cpx<T> s13 = cadd<T>(v[1], v[3]), d13 = csub<T>(v[1], v[3]);
        cpx<T> rot = INV ? mk<T>(-d13.y, d13.x) : mk<T>(d13.y, -d13.x);  // +i or -i times d13
        v[0] = cadd<T>(s02, s13);
        v[2] = csub<T>(s02, s13);
        v[1] = cadd<T>(d02, rot);
        v[3] = csub<T>(d02, rot);
    } else if constexpr (R == 8) {
        // even/odd split: E = DFT4(v0, v2, v4, v6), O = DFT4(v1, v3, v5, v7),
        // X[k] = E[k] + W8^k O[k], X[k+4] = E[k] - W8^k O[k]
        cpx<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<T, 4, INV>(e);
        dft_small<T, 4, INV>(o);
        const T h = (T)0.70710678118654752440;
        // W8^1 = (1 -+ i) h, W8^2 = -+ i, W8^3 = (-1 -+ i) h (upper sign forward)
        const cpx<T> t1 = INV ? mk<T>(h * (o[1].x - o[1].y), h * (o[1].x + o[1].y))
                              : mk<T>(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
        const cpx<T> t2 = INV ? mk<T>(-o[2].y, o[2].x) : mk<T>(o[2].y, -o[2].x);
        const cpx<T> t3 = INV ? mk<T>(-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y))
                              : mk<T>(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
        v[0] = cadd<T>(e[0], o[0]);
        v[4] = csub<T>(e[0], o[0]);
        v[1] = cadd<T>(e[1], t1);
        v[5] = csub<T>(e[1], t1);
        v[2] = cadd<T>(e[2], t2);
        v[6] = csub<T>(e[2], t2);
        v[3] = cadd<T>(e[3], t3);
        v[7] = csub<T>(e[3], t3);
    } else {  // R == 3
        const T c3 = (T)-0.5;
        const T s3 = INV ? (T)0.86602540378443864676 : (T)-0.86602540378443864676;
        cpx<T> s12 = cadd<T>(v[1], v[2]), d12 = csub<T>(v[1], v[2]);
        cpx<T> m = mk<T>(v[0].x + c3 * s12.x, v[0].y + c3 * s12.y);
        cpx<T> j = mk<T>(-s3 * d12.y, s3 * d12.x);
        v[0] = cadd<T>(v[0], s12);
        v[1] = cadd<T>(m, j);
        v[2] = csub<T>(m, j);
    }
}

// One in-place Stockham stage of radix R over P pencils of length n stored at
// a[p * ld + index].  Every thread first loads all inputs of its butterflies
// into registers, the workgroup synchronises, then the outputs are written to
// the same buffer (so one LDS buffer suffices).  Butterfly b of pencil p, with
// j = b mod (n/R) and k = j mod Ns, reads indices j + r n/R, multiplies by
// e^{-+2 pi i k r / (Ns R)} and writes (j div Ns) Ns R + k + r Ns.
constexpr int FT = FFT_THREADS;  // threads per FFT workgroup
constexpr int FE = FFT_ELEMS;    // pencil elements per thread (P * n <= FT * FE)

// LDS layout of a pencil: element i sits at pad(i) = i + i/8, which spreads the
// butterfly outputs of a radix-8 stage (lanes 8 or 64 elements apart) over all
// banks, and pencils are an odd number fft_ld(n) of elements apart, so that
// the writes of a column tile (consecutive lanes in consecutive pencils) do
// not share banks either.
__device__ __forceinline__ int pad(int i) { return i + (i >> 3); }

template <typename T, int R, bool INV>
__device__ __forceinline__ void stage(cpx<T>* a, int n, int P, int ld, int Ns, const cpx<T>* __restrict__ tw) {
    constexpr int NB = (FE + R - 1) / R;
    const int nR = n / R;
    const int span = n / (Ns * R);
    const int nb = P * nR;
    const FDiv dnR(nR), dNs(Ns);
    cpx<T> v[NB][R];
    int dst[NB], pens[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        int b = threadIdx.x + q * FT;
        dst[q] = -1;
        if (b < nb) {
            int pen = dnR.div(b), j = b - pen * nR;
            int jq = dNs.div(j), k = j - jq * Ns;
            const cpx<T>* src = a + pen * ld;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cpx<T> x = src[pad(j + r * nR)];
                if (r > 0 && k > 0) {
                    cpx<T> w = tw[k * r * span];
                    if (INV) w.y = -w.y;
                    x = cmul<T>(x, w);
                }
                v[q][r] = x;
            }
            dst[q] = jq * Ns * R + k;
            pens[q] = pen * ld;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (dst[q] >= 0) {
            dft_small<T, R, INV>(v[q]);
#pragma unroll
            for (int r = 0; r < R; ++r) a[pens[q] + pad(dst[q] + r * Ns)] = v[q][r];
        }
    }
    __syncthreads();
}

// pad(base + r S) for r = 0..R-1 as pad(base) plus a compile-time offset
// when S is a multiple of 8, or S = 1 with base a multiple of R and R
// dividing 8 (then the LDS addresses of a butterfly share one register).
template <int S, int R>
__device__ __forceinline__ constexpr bool pad_splits() { return S % 8 == 0 || (S == 1 && 8 % R == 0); }
template <int S, int R>
__device__ __forceinline__ constexpr int pad_step() { return S % 8 == 0 ? S + S / 8 : 1; }

// The same stage with the length, radix and stride known at compile time
// (power-of-two lengths): every index is a shift or a mask.  With the pencil
// count PC known too and PC n/R a multiple of FT, every thread has exactly NB
// butterflies and no bound is tested.  The twiddle of k = 0 is 1, whose
// product is exact, so it is not skipped (no divergent branch).
template <typename T, int N, int R, int NS, bool INV, int PC>
__device__ __forceinline__ void stage_c(cpx<T>* a, int P, int ld, const cpx<T>* __restrict__ tw) {
    constexpr int NB = (FE + R - 1) / R;
    constexpr int nR = N / R, span = N / (NS * R);
    constexpr bool EXACT = PC > 0 && PC * nR == NB * FT;
    const int nb = (PC > 0 ? PC : P) * nR;
    cpx<T> v[NB][R];
    int dst[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = threadIdx.x + q * FT;
        dst[q] = -1;
        if (EXACT || b < nb) {
            const int pen = b / nR, j = b % nR;
            const int jq = j / NS, k = j % NS;
            const cpx<T>* src = a + pen * ld;
            if constexpr (nR % 8 == 0) src += pad(j);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cpx<T> x = nR % 8 == 0 ? src[r * (nR + nR / 8)] : src[pad(j + r * nR)];
                if (NS > 1 && r > 0) {
                    cpx<T> w = tw[k * r * span];
                    if (INV) w.y = -w.y;
                    x = cmul<T>(x, w);
                }
                v[q][r] = x;
            }
            dst[q] = pen * ld + (pad_splits<NS, R>() ? pad(jq * NS * R + k) : jq * NS * R + k);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (EXACT || dst[q] >= 0) {
            dft_small<T, R, INV>(v[q]);
            if constexpr (pad_splits<NS, R>()) {
                cpx<T>* o = a + dst[q];
#pragma unroll
                for (int r = 0; r < R; ++r) o[r * pad_step<NS, R>()] = v[q][r];
            } else {
                // dst = pen ld + m: the pencil base is ld times the quotient
                const int pen = (threadIdx.x + q * FT) / nR, m = dst[q] - pen * ld;
#pragma unroll
                for (int r = 0; r < R; ++r) a[pen * ld + pad(m + r * NS)] = v[q][r];
            }
        }
    }
    __syncthreads();
}

// Radix plan of a length 2^a 3^b: 8 while a factor 8 remains, then 4 or 2,
// then the 3s (a radix-3 stage then has a stride that is a multiple of 8 or
// takes the general store path).
template <int M>
constexpr int radix_of() { return M % 8 == 0 ? 8 : (M % 4 == 0 ? 4 : (M % 2 == 0 ? 2 : 3)); }

// PC > 0: the pencil count is the compile-time PC (P is then ignored).
template <typename T, int N, bool INV, int PC = 0, int NS = 1>
__device__ __forceinline__ void fft_lds_c(cpx<T>* a, int P, int ld, const cpx<T>* __restrict__ tw) {
    if constexpr (NS < N) {
        constexpr int R = radix_of<N / NS>();
        stage_c<T, N, R, NS, INV, PC>(a, P, ld, tw);
        fft_lds_c<T, N, INV, PC, NS * R>(a, P, ld, tw);
    }
}

// In-place FFT of P pencils (P * n <= FT * FE) in LDS; all threads participate.
// Forward uses e^{-2 pi i m / n} from tw; INV the conjugate.
// Radices in the order 4, 4, ..., (2), 3, 3, ...: the greedy choice below
// takes every factor 4 first, then the remaining factor 2, then the 3s.
template <typename T, bool INV>
__device__ __forceinline__ void fft_lds(cpx<T>* a, int n, int P, int ld, const cpx<T>* __restrict__ tw) {
    int Ns = 1;
    for (int m = n; m > 1;) {
        if (m % 4 == 0) {
            stage<T, 4, INV>(a, n, P, ld, Ns, tw);
            Ns *= 4;
            m /= 4;
        } else if (m % 2 == 0) {
            stage<T, 2, INV>(a, n, P, ld, Ns, tw);
            Ns *= 2;
            m /= 2;
        } else {
            stage<T, 3, INV>(a, n, P, ld, Ns, tw);
            Ns *= 3;
            m /= 3;
        }
    }
}

// The twiddle table of one axis (n entries) is staged in LDS behind the pencil
// data, so that the stages read it at LDS latency.
template <typename T>
__device__ __forceinline__ const cpx<T>* stage_twiddles(cpx<T>* a, int data_elems, const T* tw, int n) {
    cpx<T>* t = a + data_elems;
    const cpx<T>* g = reinterpret_cast<const cpx<T>*>(tw);
    for (int m = threadIdx.x; m < n; m += FT) t[m] = gld(g + m);
    return t;
}

// Compile-time plans for the lengths of EK_FFT_LENGTHS, the runtime plan
// otherwise.
template <typename T, bool INV>
__device__ __forceinline__ void fft_any(cpx<T>* a, int n, int P, int ld, const cpx<T>* __restrict__ tw);

// Pass bodies are instantiated for a compile-time length NC (one of
// EK_FFT_LENGTHS, or 0: any length, known at run time) and, in the y and z
// passes, a compile-time group width TCC (0: the width is known at run time).
// With both known every index of the loads, stages and stores is a shift, a
// mask or a constant offset.
template <typename T, bool INV, int NC, int PC>
__device__ __forceinline__ void fft_n(cpx<T>* a, int n, int P, int ld, const cpx<T>* __restrict__ tw) {
    if constexpr (NC > 0) fft_lds_c<T, NC, INV, PC>(a, P, ld, tw);
    else fft_any<T, INV>(a, n, P, ld, tw);
}
template <int C>
__device__ __forceinline__ int cdiv(int t, const FDiv& d) {
    if constexpr (C > 0) return (int)((unsigned)t / (unsigned)C);
    else return d.div(t);
}

template <typename T, bool INV>
__device__ __forceinline__ void fft_any(cpx<T>* a, int n, int P, int ld, const cpx<T>* __restrict__ tw) {
    switch (n) {
        case 32: fft_lds_c<T, 32, INV>(a, P, ld, tw); break;
        case 64: fft_lds_c<T, 64, INV>(a, P, ld, tw); break;
        case 128: fft_lds_c<T, 128, INV>(a, P, ld, tw); break;
        case 256: fft_lds_c<T, 256, INV>(a, P, ld, tw); break;
        case 512: fft_lds_c<T, 512, INV>(a, P, ld, tw); break;
        default: fft_lds<T, INV>(a, n, P, ld, tw); break;
    }
}

// ---------------------------------------------------------------------------
// Pass X (forward): charge assembly + two-for-one real FFT along x.
// Work item: a pair of rows (y, y+1) at one z.  P pairs per workgroup.
// ---------------------------------------------------------------------------
// FULL: every pair of the workgroup exists (no bound tests); with NC known the
// P n elements also fill the XIT element slots of every thread exactly.
template <typename T, int NC, bool FULL = false>
__device__ __forceinline__ void fft_x_fwd_body(const Sim<T>& s, int bx_, int P_) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* a = reinterpret_cast<cpx<T>*>(smem_raw);
    constexpr int PC = NC > 0 ? fft_pencils_x(NC) : 0, NHC = NC > 0 ? NC / 2 + 1 : 0;
    const int n = NC > 0 ? NC : s.nx, ld = fft_ld(n), P = PC > 0 ? PC : P_;
    const int nh = NC > 0 ? NHC : s.nxh;
    const int npairs = s.ny * s.nz / 2;
    const int pair0 = bx_ * P;
    const T* rho = s.rho[s.cur];
    const FDiv dn(NC > 0 ? 1 : n), dnh(NC > 0 ? 1 : nh);
    const cpx<T>* tw = stage_twiddles<T>(a, P * ld, s.tw[0], n);
    // P n <= FT FE / 2: at most XIT elements per thread; every load is issued
    // before the first LDS store (a loop that stores as it loads would wait
    // for each element's loads in turn)
    constexpr int XIT = FE / 2;
    constexpr bool EXACT = NC > 0 && PC * NC == FT * XIT;
    long cr[XIT];
    T q0[XIT], q1[XIT];
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
        const int t = threadIdx.x + it * FT;
        cr[it] = -1;
        if (EXACT || t < P * n) {
            const int pen = cdiv<NC>(t, dn), x = t - pen * n, pr = pair0 + pen;
            if (FULL || pr < npairs) cr[it] = (long)(2 * pr) * n + x;  // row 2 pr = y + ny z with y even
        }
    }
    // the densities of every species (up to MAXS) requested in one round
    T d0[MAXS][XIT], d1[MAXS][XIT];
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
        const bool ok = (EXACT && FULL) || cr[it] >= 0;
        q0[it] = ok ? gld(s.rhob + cr[it]) : (T)0;
        q1[it] = ok ? gld(s.rhob + cr[it] + n) : (T)0;
#pragma unroll
        for (int k = 0; k < MAXS; ++k) {
            const T* rk = rho + (long)k * s.N;
            d0[k][it] = (k < s.ns && ok) ? gld(rk + cr[it]) : (T)0;
            d1[k][it] = (k < s.ns && ok) ? gld(rk + cr[it] + n) : (T)0;
        }
    }
#pragma unroll
    for (int k = 0; k < MAXS; ++k) {
        if (k >= s.ns) break;
        const T zk = (T)s.z[k];
#pragma unroll
        for (int it = 0; it < XIT; ++it) {
            q0[it] += zk * d0[k][it];
            q1[it] += zk * d1[k][it];
        }
    }
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
        const int t = threadIdx.x + it * FT;
        if (EXACT || t < P * n) {
            const int pen = cdiv<NC>(t, dn), x = t - pen * n;
            a[pen * ld + pad(x)] = mk<T>(q0[it], q1[it]);
        }
    }
    __syncthreads();
    fft_n<T, false, NC, PC>(a, n, P, ld, tw);
    const cpx<T>* r = a;
    cpx<T>* S = reinterpret_cast<cpx<T>*>(s.spec);
#pragma unroll
    for (int t = threadIdx.x; t < P * nh; t += FT) {
        int pen = cdiv<NHC>(t, dnh), k = t - pen * nh;
        int pr = pair0 + pen;
        if (!FULL && pr >= npairs) continue;
        cpx<T> A = r[pen * ld + pad(k)];
        cpx<T> B = r[pen * ld + pad(k == 0 ? 0 : n - k)];
        // Q1 = (A + conj B)/2, Q2 = (A - conj B)/(2i)
        cpx<T> q1 = mk<T>((T)0.5 * (A.x + B.x), (T)0.5 * (A.y - B.y));
        cpx<T> q2 = mk<T>((T)0.5 * (A.y + B.y), (T)-0.5 * (A.x - B.x));
        long row = 2 * pr;
        gst(S + row * s.nxs + k, q1);
        gst(S + (row + 1) * s.nxs + k, q2);
    }
}

// ---------------------------------------------------------------------------
// Pass X' (inverse): two half spectra -> one complex sequence -> two real rows.
// ---------------------------------------------------------------------------
template <typename T, int NC, bool FULL = false>
__device__ __forceinline__ void fft_x_inv_body(const Sim<T>& s, int bx_, int P_) {
    extern __shared__ unsigned char smem_raw[];
    cpx<T>* a = reinterpret_cast<cpx<T>*>(smem_raw);
    constexpr int PC = NC > 0 ? fft_pencils_x(NC) : 0;
    const int n = NC > 0 ? NC : s.nx, ld = fft_ld(n), P = PC > 0 ? PC : P_;
    const int nh = NC > 0 ? NC / 2 + 1 : s.nxh;
    const int npairs = s.ny * s.nz / 2;
    const int pair0 = bx_ * P;
    const cpx<T>* S = reinterpret_cast<const cpx<T>*>(s.spec);
    const FDiv dn(NC > 0 ? 1 : n);
    const cpx<T>* tw = stage_twiddles<T>(a, P * ld, s.tw[0], n);
    // loads first, as in the forward pass (P n <= FT FE / 2)
    constexpr int XIT = FE / 2;
    constexpr bool EXACT = NC > 0 && PC * NC == FT * XIT;
    cpx<T> q1[XIT], q2[XIT];
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
        const int t = threadIdx.x + it * FT;
        q1[it] = q2[it] = mk<T>(0, 0);
        if (EXACT || t < P * n) {
            const int pen = cdiv<NC>(t, dn), k = t - pen * n, pr = pair0 + pen;
            if (FULL || pr < npairs) {
                const long row = 2 * pr;
                const int kk = k < nh ? k : n - k;
                q1[it] = gld(S + row * s.nxs + kk);
                q2[it] = gld(S + (row + 1) * s.nxs + kk);
            }
        }
    }
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
        const int t = threadIdx.x + it * FT;
        if (EXACT || t < P * n) {
            const int pen = cdiv<NC>(t, dn), k = t - pen * n;
            const cpx<T> a1 = q1[it], a2 = q2[it];
            // k < nh: q1 + i q2; otherwise conj(q1) + i conj(q2) of the mirrored column
            a[pen * ld + pad(k)] = k < nh ? mk<T>(a1.x - a2.y, a1.y + a2.x) : mk<T>(a1.x + a2.y, -a1.y + a2.x);
        }
    }
    __syncthreads();
    fft_n<T, true, NC, PC>(a, n, P, ld, tw);
#pragma unroll
    for (int it = 0; it < XIT; ++it) {
        const int t = threadIdx.x + it * FT;
        if (!EXACT && t >= P * n) continue;
        int pen = cdiv<NC>(t, dn), x = t - pen * n;
        int pr = pair0 + pen;
        if (!FULL && pr >= npairs) continue;
        long c0 = (long)(2 * pr) * n + x;
        cpx<T> v = a[pen * ld + pad(x)];
        gst(s.phi + c0, v.x);
        gst(s.phi + c0 + n, v.y);
    }
}

// Tile of TC columns x n rows from the spectrum into LDS, a[i * ld + row] =
// get(row, i); consecutive threads take consecutive columns of a row.  In FP64
// every thread's loads (at most FE: TC n <= FT FE) are issued before its first
// LDS store; in FP32 that costs more registers (and occupancy) than it saves
// and the plain loop is faster (both measured).  TCC > 0: TC is that constant.
template <typename T, int TCC, typename G>
__device__ __forceinline__ void load_tile(cpx<T>* a, int ld, int TC, int n, const FDiv& dtc, G&& get) {
    if constexpr (sizeof(T) == 8) {
        T vx[FE], vy[FE];
#pragma unroll
        for (int it = 0; it < FE; ++it) {
            const int t = threadIdx.x + it * FT;
            vx[it] = vy[it] = (T)0;
            if (t < TC * n) {
                const int r = cdiv<TCC>(t, dtc), i = t - r * TC;
                const cpx<T> v = get(r, i);
                vx[it] = v.x;
                vy[it] = v.y;
            }
        }
#pragma unroll
        for (int it = 0; it < FE; ++it) {
            const int t = threadIdx.x + it * FT;
            if (t < TC * n) {
                const int r = cdiv<TCC>(t, dtc), i = t - r * TC;
                a[i * ld + pad(r)] = mk<T>(vx[it], vy[it]);
            }
        }
    } else {
#pragma unroll
        for (int it = 0; it < FE; ++it) {
            const int t = threadIdx.x + it * FT;
            if (t < TC * n) {
                const int r = cdiv<TCC>(t, dtc), i = t - r * TC;
                a[i * ld + pad(r)] = get(r, i);
            }
        }
    }
}

// Full groups of compile-time width TCC and length NC: row r, column i of the
// group at g[r rs + i].  Thread t takes column t mod TCC of rows t / TCC +
// it FT / TCC, so every address is a per-thread base plus a multiple of a
// uniform step (FT / TCC is a multiple of 8, so pad() splits as well).
// (groups that cover the workgroup's threads a whole number of times)
template <int TCC, int NC>
constexpr bool tile_c_ok() {
    return TCC > 0 && NC > 0 && FT % TCC == 0 && (FT / TCC) % 8 == 0 && (TCC * NC) % FT == 0;
}
template <typename T, int TCC, int NC>
__device__ __forceinline__ void load_tile_c(cpx<T>* a, int ld, const cpx<T>* g, long rs) {
    constexpr int RPI = FT / TCC, ITS = TCC * NC / FT;
    static_assert(tile_c_ok<TCC, NC>(), "group shape");
    const int r0 = threadIdx.x / TCC, i = threadIdx.x % TCC;
    const cpx<T>* src = g + (long)r0 * rs + i;
    cpx<T>* dst = a + i * ld + pad(r0);
    const long step = (long)RPI * rs;
    cpx<T> v[ITS];
#pragma unroll
    for (int it = 0; it < ITS; ++it) v[it] = gld(src + it * step);
#pragma unroll
    for (int it = 0; it < ITS; ++it) dst[it * (RPI + RPI / 8)] = v[it];
}
template <typename T, int TCC, int NC>
__device__ __forceinline__ void store_tile_c(const cpx<T>* a, int ld, cpx<T>* g, long rs) {
    constexpr int RPI = FT / TCC, ITS = TCC * NC / FT;
    const int r0 = threadIdx.x / TCC, i = threadIdx.x % TCC;
    cpx<T>* out = g + (long)r0 * rs + i;
    const cpx<T>* src = a + i * ld + pad(r0);
    const long step = (long)RPI * rs;
#pragma unroll
    for (int it = 0; it < ITS; ++it) gst(out + it * step, src[it * (RPI + RPI / 8)]);
}

// ---------------------------------------------------------------------------
// Pass Y (forward or inverse): pencils along y, TX consecutive kx per group.
// ---------------------------------------------------------------------------
// Stages of the y and z passes that move data straight between HBM and registers
// (compile-time length N and full groups of PC columns).  The same butterflies,
// twiddles (and Green's factors) as the staged pass in the same order, so the
// results are bit-identical; what goes is the staging of the group in LDS
// before the first stage, the copy out of LDS after the last stage and, in the
// z pass, the Green's pass over LDS (LDS round trips and their barriers).  Their
// lanes take the group's columns fastest (b = j PC + column), so that the HBM
// accesses of a wavefront are whole rows of PC columns; pencils an odd number
// of elements apart keep the LDS side free of bank conflicts.
// ---------------------------------------------------------------------------
constexpr int radix_rt(int m) { return m % 8 == 0 ? 8 : (m % 4 == 0 ? 4 : (m % 2 == 0 ? 2 : 3)); }
// Stride NS of the last stage of the radix plan of N.
constexpr int last_stride(int n) {
    int ns = 1;
    while (ns * radix_rt(n / ns) < n) ns *= radix_rt(n / ns);
    return ns;
}
template <int N, int PC>
constexpr bool direct_ok() {
    return PC > 0 && N >= 32 && N % 8 == 0 && FT % PC == 0;
}

// First stage (stride 1, radix 8) of a transform, its inputs read from HBM:
// pencil i of the group is g[z * rs + i], z = 0 .. N-1.
template <typename T, int N, int PC, bool INV>
__device__ __forceinline__ void stage_first_from_hbm(cpx<T>* a, int ld, const cpx<T>* __restrict__ g, long rs) {
    constexpr int R = radix_of<N>(), nR = N / R, NB = (PC * nR + FT - 1) / FT;
    constexpr bool EXACT = PC * nR == NB * FT;
    static_assert(R == 8, "radix-8 first stage");
    cpx<T> v[NB][R];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = threadIdx.x + q * FT, pen = b % PC, j = b / PC;
        if (EXACT || b < PC * nR) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = gld(g + (long)(j + r * nR) * rs + pen);
        }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = threadIdx.x + q * FT, pen = b % PC, j = b / PC;
        if (EXACT || b < PC * nR) {
            dft_small<T, R, INV>(v[q]);
            cpx<T>* o = a + pen * ld + pad(j * R);  // stride 1: outputs j R + r, one 8-element block
#pragma unroll
            for (int r = 0; r < R; ++r) o[r] = v[q][r];
        }
    }
    __syncthreads();
}

// First stage (stride 1, radix 8) of the inverse transform with the Green's
// factor applied to each input as it is read (input m of pencil i is the
// mode (kx0 + i, ky, m)).
template <typename T, int N, int PC, typename G>
__device__ __forceinline__ void stage_first_green(cpx<T>* a, int ld, G&& green) {
    constexpr int R = radix_of<N>(), nR = N / R, NB = (PC * nR + FT - 1) / FT;
    constexpr bool EXACT = PC * nR == NB * FT;
    static_assert(R == 8, "radix-8 first stage");
    cpx<T> v[NB][R];
    int dst[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = threadIdx.x + q * FT, pen = b / nR, j = b % nR;
        dst[q] = -1;
        if (EXACT || b < PC * nR) {
            const cpx<T>* src = a + pen * ld;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const cpx<T> x = src[pad(j + r * nR)];
                const T gf = green(pen, j + r * nR);
                v[q][r] = mk<T>(x.x * gf, x.y * gf);
            }
            dst[q] = pen * ld + pad(j * R);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        if (EXACT || dst[q] >= 0) {
            dft_small<T, R, true>(v[q]);
            cpx<T>* o = a + dst[q];
#pragma unroll
            for (int r = 0; r < R; ++r) o[r] = v[q][r];
        }
    }
    __syncthreads();
}

// The stages of stride NS up to (not including) the last one.
template <typename T, int N, bool INV, int PC, int NS>
__device__ __forceinline__ void stages_mid(cpx<T>* a, int ld, const cpx<T>* __restrict__ tw) {
    if constexpr (NS < last_stride(N)) {
        constexpr int R = radix_of<N / NS>();
        stage_c<T, N, R, NS, INV, PC>(a, PC, ld, tw);
        stages_mid<T, N, INV, PC, NS * R>(a, ld, tw);
    }
}

// Last stage (stride NS, NS R = N) of a transform, its outputs written to
// HBM: output z = k + r NS of pencil i at g[z * rs + i].
template <typename T, int N, int PC, bool INV>
__device__ __forceinline__ void stage_last_to_hbm(const cpx<T>* a, int ld, const cpx<T>* __restrict__ tw,
                                                  cpx<T>* __restrict__ g, long rs) {
    constexpr int NS = last_stride(N), R = N / NS, nR = N / R, NB = (PC * nR + FT - 1) / FT;
    constexpr bool EXACT = PC * nR == NB * FT;
    static_assert(nR == NS, "last stage");
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int b = threadIdx.x + q * FT, pen = b % PC, k = b / PC;  // k = j: the stage's span is 1
        if (!EXACT && b >= PC * nR) continue;
        const cpx<T>* src = a + pen * ld;
        cpx<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            cpx<T> x = src[pad(k + r * nR)];
            if (r > 0) {
                cpx<T> w = tw[k * r];
                if (INV) w.y = -w.y;
                x = cmul<T>(x, w);
            }
            v[r] = x;
        }
        dft_small<T, R, INV>(v);
#pragma unroll
        for (int r = 0; r < R; ++r) gst(g + (long)(k + r * NS) * rs + pen, v[r]);
    }
}

// ---------------------------------------------------------------------------
template <typename T, bool INV, int NC, int TCC>
__device__ __forceinline__ void fft_y_body(const Sim<T>& s, int bx_, int TX) {
    extern __shared__ unsigned char smem_raw[];
    const int n = NC > 0 ? NC : s.ny, nh = s.nxh, ld = fft_ld(n);
    cpx<T>* a = reinterpret_cast<cpx<T>*>(smem_raw);
    int tiles = (nh + TX - 1) / TX;
    int z = bx_ / tiles;
    int kx0 = (bx_ - z * tiles) * TX;
    // columns of this tile: TX, fewer in the last one (the Nyquist column alone
    // when nh = n/2 + 1 is one more than a multiple of TX)
    const int TC = TCC > 0 ? TCC : (nh - kx0 < TX ? nh - kx0 : TX);
    cpx<T>* S = reinterpret_cast<cpx<T>*>(s.spec) + (long)z * n * s.nxs;
    const FDiv dtc(TCC > 0 ? 1 : TC);
    const cpx<T>* tw = stage_twiddles<T>(a, TX * ld, s.tw[1], n);
    if constexpr (direct_ok<NC, TCC>()) {
        stage_first_from_hbm<T, NC, TCC, INV>(a, ld, S + kx0, s.nxs);
        stages_mid<T, NC, INV, TCC, radix_of<NC>()>(a, ld, tw);
        stage_last_to_hbm<T, NC, TCC, INV>(a, ld, tw, S + kx0, s.nxs);
        return;
    }
    if constexpr (tile_c_ok<TCC, NC>()) load_tile_c<T, TCC, NC>(a, ld, S + kx0, s.nxs);
    else load_tile<T, TCC>(a, ld, TC, n, dtc, [&](int y, int i) { return gld(S + (long)y * s.nxs + kx0 + i); });
    __syncthreads();
    fft_n<T, INV, NC, TCC>(a, n, TC, ld, tw);
    if constexpr (tile_c_ok<TCC, NC>()) {
        store_tile_c<T, TCC, NC>(a, ld, S + kx0, s.nxs);
    } else {
#pragma unroll
        for (int it = 0; it < FE; ++it) {
            const int t = threadIdx.x + it * FT;
            if (t >= TC * n) break;
            int y = cdiv<TCC>(t, dtc), i = t - y * TC;
            gst(S + (long)y * s.nxs + kx0 + i, a[i * ld + pad(y)]);
        }
    }
}

// ---------------------------------------------------------------------------
// Pass Z: forward FFT along z, multiply by the Green's function, inverse FFT.
// ---------------------------------------------------------------------------
template <typename T, int NC, int TCC>
__device__ __forceinline__ void fft_z_green_body(const Sim<T>& s, int bx_, int TX) {
    extern __shared__ unsigned char smem_raw[];
    const int n = NC > 0 ? NC : s.nz, nh = s.nxh, ny = s.ny, ld = fft_ld(n);
    cpx<T>* a = reinterpret_cast<cpx<T>*>(smem_raw);
    int tiles = (nh + TX - 1) / TX;
    int ky = bx_ / tiles;
    int kx0 = (bx_ - ky * tiles) * TX;
    const int TC = TCC > 0 ? TCC : (nh - kx0 < TX ? nh - kx0 : TX);  // columns of this tile
    cpx<T>* S = reinterpret_cast<cpx<T>*>(s.spec);
    const long zstride = (long)ny * s.nxs;
    const FDiv dtc(TCC > 0 ? 1 : TC), dn(NC > 0 ? 1 : n);
    const cpx<T>* tw = stage_twiddles<T>(a, TX * ld, s.tw[2], n);
    cpx<T>* G = S + (long)ky * s.nxs + kx0;  // row z of the group at G + z zstride
    const T scale = (T)(4.0 * 3.14159265358979323846 * s.lambda_B / (double)s.N);
    const T K2y = gld(s.k2[1] + ky);
    if constexpr (direct_ok<NC, TCC>()) {
        // Green's factor of mode (kx0 + i, ky, kz), as in the staged form below
        auto green = [&](int i, int kz) -> T {
            const int kx = kx0 + i;
            const T K2 = gld(s.k2[0] + kx) + K2y + gld(s.k2[2] + kz);
            T g;
            if constexpr (sizeof(T) == 4) g = scale * __builtin_amdgcn_rcpf(K2);
            else g = scale / K2;
            return (kx == 0 && ky == 0 && kz == 0) ? (T)0 : g;
        };
        stage_first_from_hbm<T, NC, TCC, false>(a, ld, G, zstride);
        stages_mid<T, NC, false, TCC, radix_of<NC>()>(a, ld, tw);
        {
            constexpr int NSL = last_stride(NC);
            stage_c<T, NC, NC / NSL, NSL, false, TCC>(a, TCC, ld, tw);  // the forward transform's last stage
        }
        stage_first_green<T, NC, TCC>(a, ld, green);
        stages_mid<T, NC, true, TCC, radix_of<NC>()>(a, ld, tw);
        stage_last_to_hbm<T, NC, TCC, true>(a, ld, tw, G, zstride);
        return;
    }
    if constexpr (tile_c_ok<TCC, NC>()) load_tile_c<T, TCC, NC>(a, ld, G, zstride);
    else load_tile<T, TCC>(a, ld, TC, n, dtc, [&](int z, int i) { return gld(G + z * zstride + i); });
    __syncthreads();
    fft_n<T, false, NC, TCC>(a, n, TC, ld, tw);
#pragma unroll
    for (int it = 0; it < FE; ++it) {
        const int t = threadIdx.x + it * FT;
        if (t >= TC * n) break;
        // with NC known: column i = t / NC advances by FT / NC per step, kz is fixed
        int i = cdiv<NC>(t, dn), kz = t - i * n;
        int kx = kx0 + i;
        T K2 = gld(s.k2[0] + kx) + K2y + gld(s.k2[2] + kz);
        // FP32: the hardware reciprocal (1 ulp) instead of a correctly rounded
        // division; FP64 divides
        T g;
        if constexpr (sizeof(T) == 4) g = scale * __builtin_amdgcn_rcpf(K2);
        else g = scale / K2;
        g = (kx == 0 && ky == 0 && kz == 0) ? (T)0 : g;
        cpx<T> v = a[i * ld + pad(kz)];
        a[i * ld + pad(kz)] = mk<T>(v.x * g, v.y * g);
    }
    __syncthreads();
    fft_n<T, true, NC, TCC>(a, n, TC, ld, tw);
    if constexpr (tile_c_ok<TCC, NC>()) {
        store_tile_c<T, TCC, NC>(a, ld, G, zstride);
    } else {
#pragma unroll
        for (int it = 0; it < FE; ++it) {
            const int t = threadIdx.x + it * FT;
            if (t >= TC * n) break;
            int z = cdiv<TCC>(t, dtc), i = t - z * TC;
            gst(G + z * zstride + i, a[i * ld + pad(z)]);
        }
    }
}

// ---------------------------------------------------------------------------
// Dispatch on the pencil length: compile-time bodies for the listed lengths
// from 32 to 512 (full groups), the run-time body otherwise.
// ---------------------------------------------------------------------------
#define EK_FFT_LENGTHS(X) X(32) X(48) X(64) X(96) X(128) X(256) X(512)

template <typename T>
__device__ __forceinline__ void x_fwd_any(const Sim<T>& s, int b, int P) {
    const bool full = (b + 1) * P <= s.ny * s.nz / 2;
    switch (s.nx) {
#define EK_CASE(L)                                                      \
    case L:                                                             \
        if (full) fft_x_fwd_body<T, L, true>(s, b, P);                  \
        else fft_x_fwd_body<T, L, false>(s, b, P);                      \
        return;
        EK_FFT_LENGTHS(EK_CASE)
#undef EK_CASE
        default: fft_x_fwd_body<T, 0>(s, b, P);
    }
}
template <typename T>
__device__ __forceinline__ void x_inv_any(const Sim<T>& s, int b, int P) {
    const bool full = (b + 1) * P <= s.ny * s.nz / 2;
    switch (s.nx) {
#define EK_CASE(L)                                                      \
    case L:                                                             \
        if (full) fft_x_inv_body<T, L, true>(s, b, P);                  \
        else fft_x_inv_body<T, L, false>(s, b, P);                      \
        return;
        EK_FFT_LENGTHS(EK_CASE)
#undef EK_CASE
        default: fft_x_inv_body<T, 0>(s, b, P);
    }
}
// Is group b of a y or z pass a full group of TX columns?
__device__ __forceinline__ bool full_group(int b, int nh, int TX) {
    const int tiles = (nh + TX - 1) / TX;
    return (b % tiles) * TX + TX <= nh;
}
template <typename T, bool INV>
__device__ __forceinline__ void y_any(const Sim<T>& s, int b, int TX) {
    const bool full = full_group(b, s.nxh, TX);
    switch (s.ny) {
#define EK_CASE(L)                                                                   \
    case L:                                                                          \
        if (full && TX == fft_tile_kx(L, sizeof(T)))                                 \
            fft_y_body<T, INV, L, fft_tile_kx(L, sizeof(T))>(s, b, TX);              \
        else                                                                         \
            fft_y_body<T, INV, L, 0>(s, b, TX);                                      \
        return;
        EK_FFT_LENGTHS(EK_CASE)
#undef EK_CASE
        default: fft_y_body<T, INV, 0, 0>(s, b, TX);
    }
}
template <typename T>
__device__ __forceinline__ void z_any(const Sim<T>& s, int b, int TX) {
    const bool full = full_group(b, s.nxh, TX);
    switch (s.nz) {
#define EK_CASE(L)                                                                   \
    case L:                                                                          \
        if (full && TX == fft_tile_kx(L, sizeof(T)))                                 \
            fft_z_green_body<T, L, fft_tile_kx(L, sizeof(T))>(s, b, TX);             \
        else                                                                         \
            fft_z_green_body<T, L, 0>(s, b, TX);                                     \
        return;
        EK_FFT_LENGTHS(EK_CASE)
#undef EK_CASE
        default: fft_z_green_body<T, 0, 0>(s, b, TX);
    }
}

template <typename T>
__global__ __launch_bounds__(FT) void k_fft_x_fwd(Sim<T> s, int P) {
    x_fwd_any<T>(s, blockIdx.x, P);
}
template <typename T>
__global__ __launch_bounds__(FT) void k_fft_x_inv(Sim<T> s, int P) {
    x_inv_any<T>(s, blockIdx.x, P);
}
template <typename T, bool INV>
__global__ __launch_bounds__(FT) void k_fft_y(Sim<T> s, int TX) {
    y_any<T, INV>(s, blockIdx.x, TX);
}
template <typename T>
__global__ __launch_bounds__(FT) void k_fft_z_green(Sim<T> s, int TX) {
    z_any<T>(s, blockIdx.x, TX);
}

template <typename T>
void launch_charge_poisson(const Sim<T>& s, hipStream_t st) {
    const size_t cs = sizeof(cpx<T>);
    Grids<T> g = grids_of<T>(s);
    int P = fft_pencils_x(s.nx);
    size_t shx = ((size_t)P * fft_ld(s.nx) + s.nx) * cs;
    hipLaunchKernelGGL(k_fft_x_fwd<T>, dim3(g.n[KK_FFTX]), dim3(FT), shx, st, s, P);
    int TXy = fft_tile_kx(s.ny, sizeof(T)), TXz = fft_tile_kx(s.nz, sizeof(T));
    size_t shy = ((size_t)TXy * fft_ld(s.ny) + s.ny) * cs;
    hipLaunchKernelGGL((k_fft_y<T, false>), dim3(g.n[KK_FFTY]), dim3(FT), shy, st, s, TXy);
    size_t shz = ((size_t)TXz * fft_ld(s.nz) + s.nz) * cs;
    hipLaunchKernelGGL(k_fft_z_green<T>, dim3(g.n[KK_FFTZ]), dim3(FT), shz, st, s, TXz);
    hipLaunchKernelGGL((k_fft_y<T, true>), dim3(g.n[KK_FFTY]), dim3(FT), shy, st, s, TXy);
    hipLaunchKernelGGL(k_fft_x_inv<T>, dim3(g.n[KK_FFTX]), dim3(FT), shx, st, s, P);
}

// ---------------------------------------------------------------------------
// Batched passes (FP32 tables): P and TX are derived per simulation; the LDS
// size is the largest any allowed edge needs.
// ---------------------------------------------------------------------------
constexpr int BATCH_FFT_BLOCKS = 2048;
constexpr bool FLAT_FFT = true;

static size_t batch_lds_x() {
    size_t m = 0;
    for (int n = 8; n <= MAX_FFT; n += 2) {
        size_t v = ((size_t)fft_pencils_x(n) * fft_ld(n) + n) * sizeof(cpx<float>);
        m = v > m ? v : m;
    }
    return m;
}
static size_t batch_lds_yz() {
    size_t m = 0;
    for (int n = 8; n <= MAX_FFT; n += 2) {
        size_t v = ((size_t)fft_tile_kx(n, 4) * fft_ld(n) + n) * sizeof(cpx<float>);
        m = v > m ? v : m;
    }
    return m;
}

// Flat launches with the same length dispatch as the single-simulation
// passes (compile-time bodies for the listed lengths).
__global__ __launch_bounds__(FT) void kb_fft_x_fwd(const BatchTable* __restrict__ tab) {
    batch_run<KK_FFTX, FLAT_FFT>(tab, [](const Sim<float>& s, int b) { x_fwd_any<float>(s, b, fft_pencils_x(s.nx)); });
}
__global__ __launch_bounds__(FT) void kb_fft_x_inv(const BatchTable* __restrict__ tab) {
    batch_run<KK_FFTX, FLAT_FFT>(tab, [](const Sim<float>& s, int b) { x_inv_any<float>(s, b, fft_pencils_x(s.nx)); });
}
template <bool INV>
__global__ __launch_bounds__(FT) void kb_fft_y(const BatchTable* __restrict__ tab) {
    batch_run<KK_FFTY, FLAT_FFT>(tab, [](const Sim<float>& s, int b) { y_any<float, INV>(s, b, fft_tile_kx(s.ny, 4)); });
}
__global__ __launch_bounds__(FT) void kb_fft_z_green(const BatchTable* __restrict__ tab) {
    batch_run<KK_FFTZ, FLAT_FFT>(tab, [](const Sim<float>& s, int b) { z_any<float>(s, b, fft_tile_kx(s.nz, 4)); });
}

void launch_batch_poisson(const BatchTable* tab, const int* items, hipStream_t st) {
    size_t lx = batch_lds_x(), lyz = batch_lds_yz();
    hipLaunchKernelGGL(kb_fft_x_fwd, dim3(batch_grid(FLAT_FFT, items[KK_FFTX], (const void*)kb_fft_x_fwd, FT, lx, BATCH_FFT_BLOCKS)), dim3(FT), lx, st, tab);
    hipLaunchKernelGGL(kb_fft_y<false>, dim3(batch_grid(FLAT_FFT, items[KK_FFTY], (const void*)kb_fft_y<false>, FT, lyz, BATCH_FFT_BLOCKS)), dim3(FT), lyz, st, tab);
    hipLaunchKernelGGL(kb_fft_z_green, dim3(batch_grid(FLAT_FFT, items[KK_FFTZ], (const void*)kb_fft_z_green, FT, lyz, BATCH_FFT_BLOCKS)), dim3(FT), lyz, st, tab);
    hipLaunchKernelGGL(kb_fft_y<true>, dim3(batch_grid(FLAT_FFT, items[KK_FFTY], (const void*)kb_fft_y<true>, FT, lyz, BATCH_FFT_BLOCKS)), dim3(FT), lyz, st, tab);
    hipLaunchKernelGGL(kb_fft_x_inv, dim3(batch_grid(FLAT_FFT, items[KK_FFTX], (const void*)kb_fft_x_inv, FT, lx, BATCH_FFT_BLOCKS)), dim3(FT), lx, st, tab);
}

template void launch_charge_poisson<float>(const Sim<float>&, hipStream_t);
template void launch_charge_poisson<double>(const Sim<double>&, hipStream_t);

}  // namespace ek
