// ek_lb.h -- D3Q19 TRT stream/collide of one cell (Sec. III.A, III.B), shared
// by the stand-alone LB kernel (ek_lb.hip) and the fused EK+LB pass
// (ek_fields.hip).
//
// Pull form: f_i(r) <- f_i*(r - c_i), or, if r - c_i is a boundary cell, the
// moving bounce-back f_ibar*(r) + 6 w_i rho0 c_i.v_b.  Then rho = sum f_i,
// j = sum f_i c_i, u = j + f/2,
//   f_i* = f_i + le (f_i+ - feq_i+) + lo (f_i- - feq_i-) + Delta_i,
//   feq_i+ = w_i (rho + 9/2 (c.u)^2 - 3/2 u^2),  feq_i- = 3 w_i c.j,
//   Delta_i = 3 w_i [c.f + 3/2 (2+le)((c.u)(c.f) - u.f/3)].
// On the FP32 path populations are stored as f_i - w_i; every formula above is
// linear in those offsets except the explicit mean terms, carried exactly.
#pragma once
#include "ek_internal.h"

namespace ek {

constexpr int BT = 256;  // threads per LB workgroup

template <typename T>
__device__ __forceinline__ long cidx3(const Sim<T>& s, int x, int y, int z) {
    return (long)x + (long)s.nx * ((long)y + (long)s.ny * z);
}

// 32-bit cell index and element access with a uniform base pointer: every
// allowed lattice has N * sizeof(T) < 2^32, so the byte offset of a cell fits
// a 32-bit register and the load/store can use the scalar-base addressing mode.
template <typename T>
__device__ __forceinline__ uint32_t cidx32(const Sim<T>& s, int x, int y, int z) {
    return (uint32_t)x + (uint32_t)s.nx * ((uint32_t)y + (uint32_t)s.ny * (uint32_t)z);
}
template <typename T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, uint32_t e) {
    return gld((const T*)((const char*)base + (uint32_t)(e * (uint32_t)sizeof(T))));
}
template <typename T>
__device__ __forceinline__ void st32_nt(T* __restrict__ base, uint32_t e, T v) {
    gst_nt((T*)((char*)base + (uint32_t)(e * (uint32_t)sizeof(T))), v);
}

// ---------------------------------------------------------------------------
// LB cell update (used by the fused EK+LB kernel and the unfused LB kernel)
// ---------------------------------------------------------------------------
// Periodic neighbour coordinates of one cell.
struct Nbr {
    int x, y, z, xm, xp, ym, yp, zm, zp;
    // index of the cell and the index offsets of its periodic neighbours
    uint32_t c;
    int dxm, dxp, dym, dyp, dzm, dzp;
    __device__ __forceinline__ Nbr(int x_, int y_, int z_, int nx, int ny, int nz) : x(x_), y(y_), z(z_) {
        xm = x == 0 ? nx - 1 : x - 1;
        xp = x == nx - 1 ? 0 : x + 1;
        ym = y == 0 ? ny - 1 : y - 1;
        yp = y == ny - 1 ? 0 : y + 1;
        zm = z == 0 ? nz - 1 : z - 1;
        zp = z == nz - 1 ? 0 : z + 1;
        const int P = nx * ny;
        c = (uint32_t)x + (uint32_t)nx * ((uint32_t)y + (uint32_t)ny * (uint32_t)z);
        dxm = xm - x;
        dxp = xp - x;
        dym = (ym - y) * nx;
        dyp = (yp - y) * nx;
        dzm = (zm - z) * P;
        dzp = (zp - z) * P;
    }
    // source cell r - c_i of population i
    __device__ __forceinline__ int sx(int i) const { return q19x(i) > 0 ? xm : (q19x(i) < 0 ? xp : x); }
    __device__ __forceinline__ int sy(int i) const { return q19y(i) > 0 ? ym : (q19y(i) < 0 ? yp : y); }
    __device__ __forceinline__ int sz(int i) const { return q19z(i) > 0 ? zm : (q19z(i) < 0 ? zp : z); }
    // its index: c plus the offsets of the axes along which c_i is non-zero
    __device__ __forceinline__ uint32_t src32(int i) const {
        int d = 0;
        if (q19x(i) > 0) d += dxm;
        if (q19x(i) < 0) d += dxp;
        if (q19y(i) > 0) d += dym;
        if (q19y(i) < 0) d += dyp;
        if (q19z(i) > 0) d += dzm;
        if (q19z(i) < 0) d += dzp;
        return c + (uint32_t)d;
    }
};

// Pull every population from its source r - c_i (independent loads).
template <typename T>
__device__ __forceinline__ void lb_pull(const Sim<T>& s, const Nbr& nb, T (&fi)[19]) {
    const T* __restrict__ fs = s.f[s.cur];
    sfor<19>([&](auto I) {
        constexpr int i = I;
        fi[i] = gld(fs + fidx(i, nb.src32(i)));
    });
}

// Boundary-cell sources (bit i of bmask: r - c_i is a boundary cell).
template <typename T>
__device__ __forceinline__ unsigned lb_bmask_global(const Sim<T>& s, const Nbr& nb) {
    unsigned bmask = 0;
    sfor<19>([&](auto I) {
        constexpr int i = I;
        if constexpr (i > 0) bmask |= (unsigned)(ld32(s.flag, nb.src32(i)) & F_CUR) << i;
    });
    return bmask;
}

// Stream/collide of fluid cell c with pulled populations fi, force density
// (fx, fy, fz) and boundary-source mask bmask; writes f* and u.
template <typename T, bool DEV>
__device__ __forceinline__ void lb_collide(const Sim<T>& s, uint32_t c, const Nbr& nb, T (&fi)[19], unsigned bmask,
                                           T fx, T fy, T fz) {
    const T* __restrict__ fs = s.f[s.cur];
    T* __restrict__ fd = s.f[s.cur ^ 1];
    T* __restrict__ uo = s.u[s.cur ^ 1];
    if (bmask) {
        const int nx = s.nx, ny = s.ny, nz = s.nz;
        sfor<19>([&](auto I) {
            constexpr int i = I;
            if constexpr (i > 0) {
                if (bmask & (1u << i)) {
                    // moving bounce-back from the boundary cell b = r - c_i
                    const int bx = nb.sx(i), by = nb.sy(i), bz = nb.sz(i);
                    double vb[3] = {0.0, 0.0, 0.0};
                    uint16_t ow = ld32(s.owner, nb.src32(i));
                    if (ow != NO_OWNER) {
                        const gmem<PState>& q = *(const gmem<PState>*)(s.parts + ow);
                        double r[3] = {min_image((double)bx + 0.5, q.x[0], (double)nx),
                                       min_image((double)by + 0.5, q.x[1], (double)ny),
                                       min_image((double)bz + 0.5, q.x[2], (double)nz)};
                        vb[0] = q.v[0] + (q.w[1] * r[2] - q.w[2] * r[1]);
                        vb[1] = q.v[1] + (q.w[2] * r[0] - q.w[0] * r[2]);
                        vb[2] = q.v[2] + (q.w[0] * r[1] - q.w[1] * r[0]);
                    }
                    double cv = q19x(i) * vb[0] + q19y(i) * vb[1] + q19z(i) * vb[2];
                    fi[i] = gld(fs + fidx(q19opp(i), c)) + (T)(6.0 * q19w(i) * cv);
                }
            }
        });
    }
    // Moments from the pair sums and differences of (i, ibar) (i odd, ibar = i + 1).
    T rho = fi[0], jx = (T)0, jy = (T)0, jz = (T)0;
    T ps[19], pd[19];
    sfor<9>([&](auto P) {
        constexpr int i = 2 * P + 1, o = i + 1;
        ps[i] = fi[i] + fi[o];
        pd[i] = fi[i] - fi[o];
        rho += ps[i];
        if constexpr (q19x(i) != 0) jx += (T)q19x(i) * pd[i];
        if constexpr (q19y(i) != 0) jy += (T)q19y(i) * pd[i];
        if constexpr (q19z(i) != 0) jz += (T)q19z(i) * pd[i];
    });
    const T ux = jx + (T)0.5 * fx, uy = jy + (T)0.5 * fy, uz = jz + (T)0.5 * fz;
    if (const uint32_t bad = velocity_status(ux, uy, uz)) latch_status(s.status, bad);
    const T usq = ux * ux + uy * uy + uz * uz;
    const T uf = ux * fx + uy * fy + uz * fz;
    const T le = s.lam_e, lo = s.lam_o;
    const T g2 = (T)2 + le;
    const T uf3 = uf / (T)3;
    T* __restrict__ fc = fd + fidx(0, c);  // population i of cell c at fc[i * FB]
    {  // rest population: even part only
        const T w = (T)q19w(0);
        const T feq_e = w * (rho - (T)1.5 * usq);
        gst_nt(fc, fi[0] + le * (fi[0] - feq_e) + (T)4.5 * w * g2 * (-uf3));
    }
    // TRT per pair: the even part (symmetric relaxation and the even forcing
    // term) is shared by i and ibar, the odd part changes sign.
    sfor<9>([&](auto P) {
        constexpr int i = 2 * P + 1, o = i + 1;
        const T w = (T)q19w(i);
        const T cu = (T)q19x(i) * ux + (T)q19y(i) * uy + (T)q19z(i) * uz;
        const T cj = (T)q19x(i) * jx + (T)q19y(i) * jy + (T)q19z(i) * jz;
        const T cf = (T)q19x(i) * fx + (T)q19y(i) * fy + (T)q19z(i) * fz;
        const T feq_e = w * (rho + (T)4.5 * cu * cu - (T)1.5 * usq);
        const T ev = le * ((T)0.5 * ps[i] - feq_e) + (T)4.5 * w * g2 * (cu * cf - uf3);
        const T od = lo * ((T)0.5 * pd[i] - (T)3 * w * cj) + (T)3 * w * cf;
        gst_nt(fc + i * FB, fi[i] + ev + od);
        gst_nt(fc + o * FB, fi[o] + ev - od);
    });
    T* uc = uo + vidx(0, c);
    gst_nt(uc, ux);
    gst_nt(uc + FB, uy);
    gst_nt(uc + 2 * FB, uz);
}

// Velocity of a boundary cell (no populations are streamed there).
template <typename T>
__device__ __forceinline__ void lb_wall(const Sim<T>& s, uint32_t c) {
    T* __restrict__ uc = s.u[s.cur ^ 1] + vidx(0, c);
    gst_nt(uc, (T)0);
    gst_nt(uc + FB, (T)0);
    gst_nt(uc + 2 * FB, (T)0);
}

// Launch geometry of the stand-alone LB kernel: workgroup b covers cells
// [256 (b mod nbp), 256 (b mod nbp) + 256) of plane z = b div nbp,
// nbp = ceil(nx ny / 256) (the grid size is grids_of(...).n[KK_LB]).
template <typename T> void launch_lb(const Sim<T>& s, hipStream_t st);
void launch_batch_lb(const BatchTable* tab, const int* items, hipStream_t st);

}  // namespace ek
