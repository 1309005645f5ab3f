// ek_fields.hip -- the two full-lattice stencil kernels of a step.
//
// k_ek: Nernst-Planck solute update (Sec. III.C, III.D.2).  For each cell, the
//   flux on each of its 26 links is evaluated (13 directions, both ends), the
//   density changes by the flux divergence, and the coupling force on the fluid
//   is the friction of the diffusive/migrative part (Eq. fluidcoupling).  Both
//   cells of a link evaluate it with identical operands and operation order, so
//   the two evaluations are bitwise equal and solute is conserved link by link.
//   Per link a -> b = a + s (s one of the 13 half-set directions):
//     diffusive + migrative (the 9 D3Q19 links, Eq. flux-pv multiplied out):
//       j = D/(A0|s|) [ rho_a(1-Psi_b) - rho_b(1-Psi_a)
//                       + z/2 (rho_a(1-Psi_b) + rho_b(1-Psi_a)) (phi_a - phi_b + E.s) ]
//     advective (all 13, volume of fluid): rho_a g(s; u_a) - rho_b g(-s; u_b),
//       g(s; u) = prod_d (s_d == 0 ? 1 - |u_d| : (s_d u_d > 0 ? |u_d| : 0))
//     zero if either end is a boundary cell.
//   The staged neighbourhood lives in LDS: a (TX+2) x (TY+2) x 3 window of every
//   input field, marched along z.
//
// k_lb: D3Q19 TRT stream/collide with the Guo force (Sec. III.A), pull form:
//   f_i(r) <- f_i*(r - c_i), or, if r - c_i is a boundary cell, the moving
//   bounce-back f_ibar*(r) + 6 w_i rho0 c_i.v_b (Sec. III.A/B).  Then
//   rho = sum f_i, j = sum f_i c_i, u = j + f/2,
//   f_i* = f_i + le (f_i+ - feq_i+) + lo (f_i- - feq_i-) + Delta_i,
//   feq_i+ = w_i (rho + 9/2 (c.u)^2 - 3/2 u^2),  feq_i- = 3 w_i c.j,
//   Delta_i = 3 w_i [c.f + 3/2 (2+le)((c.u)(c.f) - u.f/3)].
// On the FP32 path populations are stored as f_i - w_i and densities as
// rho_k - mean_k; every formula above is linear in those offsets except the
// explicit mean terms, which are carried exactly.
#include "ek_internal.h"

namespace ek {

constexpr int BT = 256;

template <typename T>
__device__ __forceinline__ long cidx3(const Sim<T>& s, int x, int y, int z) {
    return (long)x + (long)s.nx * ((long)y + (long)s.ny * z);
}

// ---------------------------------------------------------------------------
// EK
// ---------------------------------------------------------------------------
template <typename T, int NS>
struct CellEK {
    T r[NS];
    T psi, phi, ux, uy, uz;
    bool wall;
};

template <typename T, int H>
__device__ __forceinline__ T adv_frac(T ux, T uy, T uz, int sgn) {
    constexpr int sx = hx(H), sy = hy(H), sz = hz(H);
    T g = (T)1;
    T u[3] = {ux, uy, uz};
    int sv[3] = {sx * sgn, sy * sgn, sz * sgn};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T a = fabs(u[d]);
        if (sv[d] == 0) g *= ((T)1 - a);
        else g *= ((sv[d] > 0 && u[d] > (T)0) || (sv[d] < 0 && u[d] < (T)0)) ? a : (T)0;
    }
    return g;
}

template <typename T, bool DEV, int NS, int H>
__device__ __forceinline__ void link_flux(const Sim<T>& s, const CellEK<T, NS>& a, const CellEK<T, NS>& b,
                                          const T (&Es)[13], const T (&coef)[13], T (&jt)[NS], T (&gd)[NS]) {
    if (a.wall || b.wall) {
#pragma unroll
        for (int k = 0; k < NS; ++k) jt[k] = gd[k] = (T)0;
        return;
    }
    T pa = s.pv ? a.psi : (T)0;
    T pb = s.pv ? b.psi : (T)0;
    T oa = (T)1 - pa, ob = (T)1 - pb;
    T dphi = (a.phi - b.phi) + Es[H];
    T ga = adv_frac<T, H>(a.ux, a.uy, a.uz, +1);
    T gb = adv_frac<T, H>(b.ux, b.uy, b.uz, -1);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        T ra = a.r[k], rb = b.r[k];
        T g = (T)0;
        T A = ra * ob - rb * oa;
        T B = ra * ob + rb * oa;
        T adv = ra * ga - rb * gb;
        if constexpr (DEV) {
            T ref = (T)s.rho_ref[k];
            A += ref * (pa - pb);
            B += ref * (oa + ob);
            adv += ref * (ga - gb);
        }
        if constexpr (H < 9) g = (A + (T)0.5 * (T)s.z[k] * B * dphi) * coef[H];
        gd[k] = g;
        jt[k] = (T)s.D[k] * g + adv;
    }
}

// LDS window: a (TXW+2) x (TYW+2) window of every input field for three
// consecutive z-planes (z-1, z, z+1), marched along z.
template <typename T, int NS, int TXW, int TYW>
struct EKShared {
    static constexpr int WX = TXW + 2, WY = TYW + 2, WPL = WX * WY;
    T r[NS][3][WPL];
    float psi[3][WPL];
    T phi[3][WPL];
    T u[3][3][WPL];
    uint8_t fl[3][WPL];
};

template <typename T, int NS, int TXW, int TYW>
__device__ __forceinline__ void ek_load_plane(const Sim<T>& s, EKShared<T, NS, TXW, TYW>& sh, int slot, int x0,
                                              int y0, int z, const T* __restrict__ rin) {
    using SH = EKShared<T, NS, TXW, TYW>;
    int zz = wrapi(z, s.nz);
    for (int t = threadIdx.x; t < SH::WPL; t += TXW * TYW) {
        int i = t % SH::WX, j = t / SH::WX;
        int x = wrapi(x0 + i - 1, s.nx), y = wrapi(y0 + j - 1, s.ny);
        long c = cidx3(s, x, y, zz);
#pragma unroll
        for (int k = 0; k < NS; ++k) sh.r[k][slot][t] = rin[(long)k * s.N + c];
        sh.psi[slot][t] = s.psi[c];
        sh.phi[slot][t] = s.phi[c];
        sh.u[0][slot][t] = s.u[c];
        sh.u[1][slot][t] = s.u[s.N + c];
        sh.u[2][slot][t] = s.u[2 * s.N + c];
        sh.fl[slot][t] = s.flag[c];
    }
}

template <typename T, int NS, int TXW, int TYW>
__device__ __forceinline__ CellEK<T, NS> ek_cell(const EKShared<T, NS, TXW, TYW>& sh, int slot, int t) {
    CellEK<T, NS> c;
#pragma unroll
    for (int k = 0; k < NS; ++k) c.r[k] = sh.r[k][slot][t];
    c.psi = (T)sh.psi[slot][t];
    c.phi = sh.phi[slot][t];
    c.ux = sh.u[0][slot][t];
    c.uy = sh.u[1][slot][t];
    c.uz = sh.u[2][slot][t];
    c.wall = (sh.fl[slot][t] & F_CUR) != 0;
    return c;
}

// Grid: ceil(nx/TXW) x ceil(ny/TYW) x z-chunks; each workgroup marches ZC planes.
template <typename T, bool DEV, int NS, int TXW, int TYW>
__global__ __launch_bounds__(TXW* TYW) void k_ek(Sim<T> s, int ZC) {
    using SH = EKShared<T, NS, TXW, TYW>;
    __shared__ SH sh;
    const int x0 = blockIdx.x * TXW, y0 = blockIdx.y * TYW, zbeg = blockIdx.z * ZC;
    const T* __restrict__ rin = s.rho[s.cur];
    T* __restrict__ rout = s.rho[s.cur ^ 1];
    T Es[13], coef[13];
    sfor<13>([&](auto HH) {
        constexpr int h = HH;
        Es[h] = (T)(s.E[0] * hx(h) + s.E[1] * hy(h) + s.E[2] * hz(h));
        coef[h] = (T)(1.0 / ((1.0 + 2.0 * 1.4142135623730950488) * hlen(h)));
    });
    const T half_kT = (T)(0.5 * s.kT);
    ek_load_plane<T, NS, TXW, TYW>(s, sh, (zbeg + 2) % 3, x0, y0, zbeg - 1, rin);
    ek_load_plane<T, NS, TXW, TYW>(s, sh, zbeg % 3, x0, y0, zbeg, rin);
    const int tx = threadIdx.x % TXW, ty = threadIdx.x / TXW;
    const int x = x0 + tx, y = y0 + ty;
    const bool valid = x < s.nx && y < s.ny;
    const int zend = zbeg + ZC < s.nz ? zbeg + ZC : s.nz;
    for (int z = zbeg; z < zend; ++z) {
        ek_load_plane<T, NS, TXW, TYW>(s, sh, (z + 1) % 3, x0, y0, z + 1, rin);
        __syncthreads();
        if (valid) {
            const int sm = (z + 2) % 3, s0 = z % 3, sp = (z + 1) % 3;
            const int ctr = (ty + 1) * SH::WX + (tx + 1);
            long c = cidx3(s, x, y, z);
            CellEK<T, NS> me = ek_cell<T, NS, TXW, TYW>(sh, s0, ctr);
            T dr[NS];
            T fe[3] = {(T)0, (T)0, (T)0};
#pragma unroll
            for (int k = 0; k < NS; ++k) dr[k] = (T)0;
            if (!me.wall) {
                sfor<13>([&](auto HH) {
                    constexpr int h = HH;
                    constexpr int ox = hx(h), oy = hy(h), oz = hz(h);
                    const int up = ctr + oy * SH::WX + ox, dn = ctr - oy * SH::WX - ox;
                    const int sup = oz == 0 ? s0 : (oz > 0 ? sp : sm);
                    const int sdn = oz == 0 ? s0 : (oz > 0 ? sm : sp);
                    CellEK<T, NS> cu = ek_cell<T, NS, TXW, TYW>(sh, sup, up);
                    CellEK<T, NS> cd = ek_cell<T, NS, TXW, TYW>(sh, sdn, dn);
                    T jt1[NS], gd1[NS], jt2[NS], gd2[NS];
                    link_flux<T, DEV, NS, h>(s, me, cu, Es, coef, jt1, gd1);
                    link_flux<T, DEV, NS, h>(s, cd, me, Es, coef, jt2, gd2);
#pragma unroll
                    for (int k = 0; k < NS; ++k) {
                        dr[k] += -jt1[k] + jt2[k];
                        if constexpr (h < 9) {
                            T g = half_kT * (gd1[k] + gd2[k]);
                            if constexpr (ox != 0) fe[0] += g * (T)ox;
                            if constexpr (oy != 0) fe[1] += g * (T)oy;
                            if constexpr (oz != 0) fe[2] += g * (T)oz;
                        }
                    }
                });
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                T out;
                if (me.wall) out = DEV ? (T)(-s.rho_ref[k]) : (T)0;
                else out = me.r[k] + dr[k];
                rout[(long)k * s.N + c] = out;
            }
            s.fext[c] = fe[0];
            s.fext[s.N + c] = fe[1];
            s.fext[2 * s.N + c] = fe[2];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// LB
// ---------------------------------------------------------------------------
template <typename T, bool DEV>
__global__ __launch_bounds__(BT) void k_lb(Sim<T> s) {
    long c = (long)blockIdx.x * BT + threadIdx.x;
    if (c >= s.N) return;
    const int nx = s.nx, ny = s.ny, nz = s.nz;
    int x = (int)(c % nx);
    int y = (int)((c / nx) % ny);
    int z = (int)(c / ((long)nx * ny));
    const uint8_t fl = s.flag[c];
    if (fl & F_CUR) {
        s.u[c] = s.u[s.N + c] = s.u[2 * s.N + c] = (T)0;
        return;
    }
    const T* __restrict__ fs = s.f[s.cur];
    T* __restrict__ fd = s.f[s.cur ^ 1];
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
    // Pull every population from its source r - c_i first (independent loads),
    // then replace those whose source is a boundary cell (rare).
    T fi[19];
    long src[19];
    sfor<19>([&](auto I) {
        constexpr int i = I;
        const int sx = q19x(i) > 0 ? xm : (q19x(i) < 0 ? xp : x);
        const int sy = q19y(i) > 0 ? ym : (q19y(i) < 0 ? yp : y);
        const int sz = q19z(i) > 0 ? zm : (q19z(i) < 0 ? zp : z);
        src[i] = cidx3(s, sx, sy, sz);
        fi[i] = fs[(long)i * s.N + src[i]];
    });
    const T fx = s.fext[c], fy = s.fext[s.N + c], fz = s.fext[2 * s.N + c];
    unsigned bmask = 0;
    sfor<19>([&](auto I) {
        constexpr int i = I;
        if constexpr (i > 0) bmask |= (unsigned)(s.flag[src[i]] & F_CUR) << i;
    });
    if (bmask) {
        sfor<19>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) {
                if (bmask & (1u << i)) {
                    // moving bounce-back from the boundary cell src
                    const long b = src[i];
                    double vb[3] = {0.0, 0.0, 0.0};
                    uint16_t ow = s.owner[b];
                    if (ow != NO_OWNER) {
                        const PState& q = s.parts[ow];
                        const int bx = (int)(b % nx), by = (int)((b / nx) % ny), bz = (int)(b / ((long)nx * ny));
                        double r[3] = {min_image((double)bx + 0.5, q.x[0], (double)nx),
                                       min_image((double)by + 0.5, q.x[1], (double)ny),
                                       min_image((double)bz + 0.5, q.x[2], (double)nz)};
                        vb[0] = q.v[0] + (q.w[1] * r[2] - q.w[2] * r[1]);
                        vb[1] = q.v[1] + (q.w[2] * r[0] - q.w[0] * r[2]);
                        vb[2] = q.v[2] + (q.w[0] * r[1] - q.w[1] * r[0]);
                    }
                    double cv = q19x(i) * vb[0] + q19y(i) * vb[1] + q19z(i) * vb[2];
                    fi[i] = fs[(long)q19opp(i) * s.N + c] + (T)(6.0 * q19w(i) * cv);
                }
            }
        });
    }
    T rho = (T)0, jx = (T)0, jy = (T)0, jz = (T)0;
    sfor<19>([&](auto I) {
        constexpr int i = I;
        rho += fi[i];
        if constexpr (q19x(i) != 0) jx += (T)q19x(i) * fi[i];
        if constexpr (q19y(i) != 0) jy += (T)q19y(i) * fi[i];
        if constexpr (q19z(i) != 0) jz += (T)q19z(i) * fi[i];
    });
    const T ux = jx + (T)0.5 * fx, uy = jy + (T)0.5 * fy, uz = jz + (T)0.5 * fz;
    const T usq = ux * ux + uy * uy + uz * uz;
    const T uf = ux * fx + uy * fy + uz * fz;
    const T le = s.lam_e, lo = s.lam_o;
    const T g2 = (T)2 + le;
    sfor<19>([&](auto I) {
        constexpr int i = I;
        constexpr int o = q19opp(i);
        const T w = (T)q19w(i);
        const T cu = (T)q19x(i) * ux + (T)q19y(i) * uy + (T)q19z(i) * uz;
        const T cj = (T)q19x(i) * jx + (T)q19y(i) * jy + (T)q19z(i) * jz;
        const T cf = (T)q19x(i) * fx + (T)q19y(i) * fy + (T)q19z(i) * fz;
        const T feq_e = w * (rho + (T)4.5 * cu * cu - (T)1.5 * usq);
        const T feq_o = w * (T)3 * cj;
        const T fp = (T)0.5 * (fi[i] + fi[o]);
        const T fm = (T)0.5 * (fi[i] - fi[o]);
        const T delta = (T)3 * w * (cf + (T)1.5 * (g2 * cu * cf - g2 * uf / (T)3));
        __builtin_nontemporal_store(fi[i] + le * (fp - feq_e) + lo * (fm - feq_o) + delta, &fd[(long)i * s.N + c]);
    });
    __builtin_nontemporal_store(ux, &s.u[c]);
    __builtin_nontemporal_store(uy, &s.u[s.N + c]);
    __builtin_nontemporal_store(uz, &s.u[2 * s.N + c]);
}

// ---------------------------------------------------------------------------
template <typename T, bool DEV, int NS>
static void launch_ek_ns(const Sim<T>& s, hipStream_t st) {
    constexpr int TXW = sizeof(T) == 4 ? 32 : 16, TYW = 8;
    int gx = (s.nx + TXW - 1) / TXW, gy = (s.ny + TYW - 1) / TYW;
    int ZC = 8;
    int gz = (s.nz + ZC - 1) / ZC;
    hipLaunchKernelGGL((k_ek<T, DEV, NS, TXW, TYW>), dim3(gx, gy, gz), dim3(TXW * TYW), 0, st, s, ZC);
}

template <typename T>
void launch_ek(const Sim<T>& s, hipStream_t st) {
    constexpr bool DEV = sizeof(T) == 4;
    switch (s.ns) {
        case 1: launch_ek_ns<T, DEV, 1>(s, st); break;
        case 2: launch_ek_ns<T, DEV, 2>(s, st); break;
        case 3: launch_ek_ns<T, DEV, 3>(s, st); break;
        default: launch_ek_ns<T, DEV, 4>(s, st); break;
    }
}

template <typename T>
void launch_lb(const Sim<T>& s, hipStream_t st) {
    constexpr bool DEV = sizeof(T) == 4;
    hipLaunchKernelGGL((k_lb<T, DEV>), dim3((unsigned)((s.N + BT - 1) / BT)), dim3(BT), 0, st, s);
}

template void launch_ek<float>(const Sim<float>&, hipStream_t);
template void launch_ek<double>(const Sim<double>&, hipStream_t);
template void launch_lb<float>(const Sim<float>&, hipStream_t);
template void launch_lb<double>(const Sim<double>&, hipStream_t);

}  // namespace ek
