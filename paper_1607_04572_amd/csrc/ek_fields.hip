// ek_fields.hip -- the EK solute update of a step, alone (FP32 path; the LB
// stream/collide then runs as its own kernel, ek_lb.hip) or fused with the LB
// cell update of ek_lb.h (FP64 path).
//
// k_ek: Nernst-Planck solute update (Sec. III.C, III.D.2).  For each cell, the
//   flux on each of its 26 links is evaluated (13 directions, both ends), the
//   density changes by the flux divergence, and the coupling force on the fluid
//   is the friction of the diffusive/migrative part (Eq. fluidcoupling).  In
//   the general form (ek_cell_update: windows holding a boundary cell or a
//   partial volume) both cells of a link evaluate it with identical operands
//   and operation order, so the two evaluations are bitwise equal and solute
//   is conserved link by link; windows free of both gather the same fluxes
//   per neighbour in fewer operations (ek_cell_update_gather), conserving
//   solute to the rounding of each cell's sums.
//   Per link a -> b = a + s (s one of the 13 half-set directions):
//     diffusive + migrative (the 9 D3Q19 links, Eq. flux-pv multiplied out):
//       j = D/(A0|s|) [ rho_a(1-Psi_b) - rho_b(1-Psi_a)
//                       + z/2 (rho_a(1-Psi_b) + rho_b(1-Psi_a)) (phi_a - phi_b + E.s) ]
//     advective (all 13, volume of fluid): rho_a g(s; u_a) - rho_b g(-s; u_b),
//       g(s; u) = prod_d (s_d == 0 ? 1 - |u_d| : (s_d u_d > 0 ? |u_d| : 0))
//     zero if either end is a boundary cell.
//   The staged neighbourhood lives in LDS: a (TX+2) x (TY+2) x 3 window of every
//   input field, marched along z.
// k_ek32: the FP32 pass, with the loads of the window's next plane in flight
//   while the current one is computed (ek_body_pipe).
// k_ek<..., FUSE>: EK and LB in one pass: each thread finishes its cell's EK
//   update and then streams/collides the same cell with the coupling force
//   still in registers.  The velocity is double-buffered (EK reads u[cur], LB
//   writes u[cur^1]) so that the two can interleave across workgroups.
// On the FP32 path densities are stored as rho_k - mean_k; every formula above
// is linear in those offsets except the explicit mean terms, which are carried
// exactly.
#include "ek_lb.h"

namespace ek {

// ---------------------------------------------------------------------------
// EK
// ---------------------------------------------------------------------------
// One LDS record per cell: NS densities, potential, Psi, velocity, boundary
// flag, padded to a multiple of 4 elements (vector LDS reads).
template <typename T, int NS>
struct alignas(16) RecEK {
    static constexpr int NV = ((NS + 6) + 3) / 4 * 4;
    T v[NV];
    __device__ __forceinline__ T r(int k) const { return v[k]; }
    __device__ __forceinline__ T phi() const { return v[NS]; }
    __device__ __forceinline__ T psi() const { return v[NS + 1]; }
    __device__ __forceinline__ T ux() const { return v[NS + 2]; }
    __device__ __forceinline__ T uy() const { return v[NS + 3]; }
    __device__ __forceinline__ T uz() const { return v[NS + 4]; }
    __device__ __forceinline__ bool wall() const { return v[NS + 5] != (T)0; }
};

// Per-species constants of the link flux, hoisted out of the cell loop.
// Dc[k][0/1] = D_k / (A0 |s|) for |s| = 1 and sqrt 2 (the link-length
// factor of the diffusive/migrative flux).
template <typename T, int NS>
struct EKConst {
    T D[NS], hz[NS], ref[NS];
    T Es[13], Dc[NS][2];
};

// 1 / (A0 |s|) of half-direction h (A0 = 1 + 2 sqrt 2).
template <int H>
constexpr double link_coef() { return 1.0 / ((1.0 + 2.0 * 1.4142135623730950488) * hlen(H)); }

template <typename T, int NS>
__device__ __forceinline__ EKConst<T, NS> ek_consts(const Sim<T>& s) {
    EKConst<T, NS> K;
    sfor<13>([&](auto HH) {
        constexpr int h = HH;
        K.Es[h] = (T)(s.E[0] * hx(h) + s.E[1] * hy(h) + s.E[2] * hz(h));
    });
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        K.Dc[k][0] = (T)(s.D[k] * link_coef<0>());
        K.Dc[k][1] = (T)(s.D[k] * link_coef<3>());
        K.D[k] = (T)s.D[k];
        K.hz[k] = (T)(0.5 * s.z[k]);
        K.ref[k] = (T)s.rho_ref[k];
    }
    return K;
}

// Fraction of a cell moving with velocity u that lands in the neighbour at
// offset s along one axis: |u| if s has the sign of u, 1 - |u| if s = 0, else 0.
// In FP32 max(+-u, 0) is one median-of-three instruction, med3(+-u, 0, 1e30)
// (the plain select or max costs a compare or a NaN-quieting step more; a
// lattice velocity is far below the bound); the result differs at most in the
// sign of a zero fraction, which no sum can turn into a value.
template <typename T, int SX>
__device__ __forceinline__ T vof_axis(T u) {
    if constexpr (sizeof(T) == 4 && SX != 0) {
        return __builtin_amdgcn_fmed3f(SX > 0 ? u : -u, 0.0f, 1.0e30f);
    } else {
        if constexpr (SX > 0) return u > (T)0 ? u : (T)0;
        else if constexpr (SX < 0) return u < (T)0 ? -u : (T)0;
        else return (T)1 - fabs(u);
    }
}

// g(s; u) = product over the axes, in axis order.
template <typename T, int SX, int SY, int SZ>
__device__ __forceinline__ T vof_frac(T ux, T uy, T uz) {
    return (vof_axis<T, SX>(ux) * vof_axis<T, SY>(uy)) * vof_axis<T, SZ>(uz);
}

// Fused multiply-add of the element type.
__device__ __forceinline__ float fmt(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmt(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Flux on the link a -> b along half-direction H: total flux jt[k] and the
// diffusive/migrative part divided by D, summed over species, in gsum (the
// general form: boundary cells and partial volumes; both cells of a link
// evaluate it, from the same operands in the same order).
// The advective fractions of one cell for every direction, from its nine
// axis factors and their x-y pair products: g(s; u) = (f_x f_y) f_z, the same
// operations in the same order as vof_frac, so both ends of a link still
// evaluate it bit for bit alike.
template <typename T>
struct VofCell {
    T fz[3], pxy[3][3];
    __device__ __forceinline__ VofCell(T ux, T uy, T uz) {
        const T fx[3] = {vof_axis<T, -1>(ux), vof_axis<T, 0>(ux), vof_axis<T, 1>(ux)};
        const T fy[3] = {vof_axis<T, -1>(uy), vof_axis<T, 0>(uy), vof_axis<T, 1>(uy)};
        fz[0] = vof_axis<T, -1>(uz);
        fz[1] = vof_axis<T, 0>(uz);
        fz[2] = vof_axis<T, 1>(uz);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) pxy[i][j] = fx[i] * fy[j];
    }
    template <int SX, int SY, int SZ>
    __device__ __forceinline__ T frac() const { return pxy[SX + 1][SY + 1] * fz[SZ + 1]; }
};

// ga = g(s; u_a), gb = g(-s; u_b) are passed in (one end's fractions come
// from its VofCell).
template <typename T, bool DEV, int NS, int H>
__device__ __forceinline__ void link_flux(const Sim<T>& s, const RecEK<T, NS>& a, const RecEK<T, NS>& b,
                                          const EKConst<T, NS>& K, const T ga, const T gb, T (&jt)[NS], T& gsum) {
    // Fused multiply-adds written out, none left to contraction: which
    // product of x y - z w the compiler would fuse depends on the code around
    // each inlined call, and the two cells of a link must round its flux alike.
#pragma clang fp contract(off)
    if (a.wall() || b.wall()) {
#pragma unroll
        for (int k = 0; k < NS; ++k) jt[k] = (T)0;
        gsum = (T)0;
        return;
    }
    const T dphi = (a.phi() - b.phi()) + K.Es[H];
    const T pa = s.pv ? a.psi() : (T)0, pb = s.pv ? b.psi() : (T)0;
    const T oa = (T)1 - pa, ob = (T)1 - pb;
    const T dg = ga - gb;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const T ra = a.r(k), rb = b.r(k);
        const T rbo = rb * oa;
        T A = fmt(ra, ob, -rbo);
        const T B = fmt(ra, ob, rbo);
        if constexpr (DEV) A = fmt(K.ref[k], pa - pb, A);
        T adv = fmt(ra, ga, -(rb * gb));
        T mig = K.hz[k] * B;
        if constexpr (DEV) {
            // reference density terms: B += ref (oa + ob)
            mig = fmt(K.hz[k], K.ref[k] * (oa + ob), mig);
            adv = fmt(K.ref[k], dg, adv);
        }
        if constexpr (H < 9) {
            // g = (A + mig dphi): the flux over D/(A0|s|); gsum collects it for
            // the friction, which the caller scales by 1/(A0|s|)
            const T g = fmt(mig, dphi, A);
            gsum = k == 0 ? g : gsum + g;
            jt[k] = fmt(K.Dc[k][hlen(H) > 1.0 ? 1 : 0], g, adv);
        } else {
            jt[k] = adv;
            gsum = (T)0;
        }
    }
}

// LDS window: (TXW+2) x (TYW+2) records for three consecutive z-planes
// (z-1, z, z+1), marched along z.  A record is stored as NCH 16-byte chunks,
// chunk-major (ch[slot][j][cell]): the lanes of a wavefront reading the same
// chunk of consecutive cells touch consecutive 16-byte words, free of bank
// conflicts, where whole records side by side would be read at a stride.
template <typename T, int NS, int TXW, int TYW>
struct EKShared {
    static constexpr int WX = TXW + 2, WY = TYW + 2, WPL = WX * WY;
    static constexpr int PER = 16 / sizeof(T);                 // elements per chunk
    static constexpr int NCH = RecEK<T, NS>::NV / PER;         // chunks per record
    struct alignas(16) Chunk { T v[PER]; };
    Chunk ch[3][NCH][WPL];
    int dirty[3];
    __device__ __forceinline__ RecEK<T, NS> get(int slot, int i) const {
        RecEK<T, NS> r;
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            const Chunk c = ch[slot][j][i];
#pragma unroll
            for (int e = 0; e < PER; ++e) r.v[j * PER + e] = c.v[e];
        }
        return r;
    }
    __device__ __forceinline__ void put(int slot, int i, const RecEK<T, NS>& r) {
#pragma unroll
        for (int j = 0; j < NCH; ++j) {
            Chunk c;
#pragma unroll
            for (int e = 0; e < PER; ++e) c.v[e] = r.v[j * PER + e];
            ch[slot][j][i] = c;
        }
    }
    // one element of a record (reads only its chunk)
    __device__ __forceinline__ T elem(int slot, int i, int k) const { return ch[slot][k / PER][i].v[k % PER]; }
    __device__ __forceinline__ bool wall(int slot, int i) const { return elem(slot, i, NS + 5) != (T)0; }
};

// In-plane part x + nx y of the cell index of each window record this thread
// loads (records t = threadIdx.x + r TXW TYW); it is the same for every plane.
// Records up to one past the tile's last valid cell wrap periodically; those
// beyond (tiles wider than a small domain) serve no valid cell and are clamped
// into range.
// (FP32 only: the FP64 fused kernel has no registers to spare for them and
// recomputes the offsets per plane.)
template <typename T, int NS, int TXW, int TYW>
struct PlaneMap {
    using SH = EKShared<T, NS, TXW, TYW>;
    static constexpr int NT = TXW * TYW, NR = (SH::WPL + NT - 1) / NT;
    static constexpr bool KEEP = sizeof(T) == 4;
    uint32_t cxy[KEEP ? NR : 1];
    int x0, y0;
    __device__ __forceinline__ static uint32_t offset(const Sim<T>& s, int x0, int y0, int t) {
        const int i = t % SH::WX, j = t / SH::WX;
        int x = wrap1(x0 + i - 1, s.nx), y = wrap1(y0 + j - 1, s.ny);
        x = x < s.nx ? x : s.nx - 1;
        y = y < s.ny ? y : s.ny - 1;
        return (uint32_t)x + (uint32_t)s.nx * (uint32_t)y;
    }
    __device__ __forceinline__ PlaneMap(const Sim<T>& s, int x0_, int y0_) : x0(x0_), y0(y0_) {
        if constexpr (KEEP) {
#pragma unroll
            for (int r = 0; r < NR; ++r) cxy[r] = offset(s, x0, y0, threadIdx.x + r * NT);
        }
    }
    __device__ __forceinline__ uint32_t at(const Sim<T>& s, int r) const {
        if constexpr (KEEP) return cxy[r];
        else return offset(s, x0, y0, threadIdx.x + r * NT);
    }
};

// Load one plane; returns whether it holds a boundary cell or a partial volume.
template <typename T, int NS, int TXW, int TYW>
__device__ __forceinline__ bool ek_load_plane(const Sim<T>& s, EKShared<T, NS, TXW, TYW>& sh, int slot,
                                              const PlaneMap<T, NS, TXW, TYW>& pm, int z,
                                              const T* __restrict__ rin) {
    using SH = EKShared<T, NS, TXW, TYW>;
    using PM = PlaneMap<T, NS, TXW, TYW>;
    const uint32_t zoff = (uint32_t)wrap1(z, s.nz) * ((uint32_t)s.nx * (uint32_t)s.ny);  // z in [-1, nz]
    const T* __restrict__ ui = s.u[s.cur];
    bool dirty = false;
    auto one = [&](int rr) {
        const int t = threadIdx.x + rr * PM::NT;
        const uint32_t c = pm.at(s, rr) + zoff;
        RecEK<T, NS> r;
#pragma unroll
        for (int k = 0; k < NS; ++k) r.v[k] = ld32(rin + (long)k * s.N, c);
        float psi = ld32(s.psi, c);
        uint8_t fl = ld32(s.flag, c);
        r.v[NS] = ld32(s.phi, c);
        r.v[NS + 1] = (T)psi;
        const T* uc = ui + vidx(0, c);
        r.v[NS + 2] = gld(uc);
        r.v[NS + 3] = gld(uc + FB);
        r.v[NS + 4] = gld(uc + 2 * FB);
        r.v[NS + 5] = (fl & F_CUR) ? (T)1 : (T)0;
#pragma unroll
        for (int k = NS + 6; k < RecEK<T, NS>::NV; ++k) r.v[k] = (T)0;
        sh.put(slot, t, r);
        dirty |= (psi != 0.0f) || (fl & F_CUR);
    };
    if constexpr (PM::KEEP) {
#pragma unroll
        for (int rr = 0; rr < PM::NR; ++rr)
            if (threadIdx.x + rr * PM::NT < SH::WPL) one(rr);
    } else {
        // one record at a time (two in flight would not fit the FP64 budget)
#pragma nounroll
        for (int rr = 0; rr < PM::NR; ++rr)
            if (threadIdx.x + rr * PM::NT < SH::WPL) one(rr);
    }
    return dirty;
}

// Block -> tile map that keeps neighbouring tiles on one XCD: workgroups are
// dispatched round-robin over the 8 XCDs (each with its own L2), so tile
// (bid mod 8) * (n / 8) + bid / 8 puts consecutive tiles, whose halo cache
// lines overlap, on the same L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
    constexpr int NXCD = 8;
    if (n % NXCD) return bid;
    return (bid % NXCD) * (n / NXCD) + bid / NXCD;
}

template <typename T, bool DEV, int NS, typename SH>
__device__ __forceinline__ void ek_cell_update(const Sim<T>& s, const SH& sh, int s0, int sm, int sp, int ctr,
                                               const EKConst<T, NS>& K, T (&dr)[NS], T (&fe)[3]) {
    const RecEK<T, NS> me = sh.get(s0, ctr);
    const VofCell<T> mv(me.ux(), me.uy(), me.uz());
    sfor<13>([&](auto HH) {
        constexpr int h = HH;
        constexpr int ox = hx(h), oy = hy(h), oz = hz(h);
        const int up = ctr + oy * SH::WX + ox, dn = ctr - oy * SH::WX - ox;
        const int sup = oz == 0 ? s0 : (oz > 0 ? sp : sm);
        const int sdn = oz == 0 ? s0 : (oz > 0 ? sm : sp);
        const RecEK<T, NS> cu = sh.get(sup, up);
        const RecEK<T, NS> cd = sh.get(sdn, dn);
        T jt1[NS], jt2[NS], g1, g2;
        link_flux<T, DEV, NS, h>(s, me, cu, K, mv.template frac<ox, oy, oz>(),
                                        vof_frac<T, -ox, -oy, -oz>(cu.ux(), cu.uy(), cu.uz()), jt1, g1);
        link_flux<T, DEV, NS, h>(s, cd, me, K, vof_frac<T, ox, oy, oz>(cd.ux(), cd.uy(), cd.uz()),
                                        mv.template frac<-ox, -oy, -oz>(), jt2, g2);
        // the first term of each sum is assigned (an added 0 is an instruction)
#pragma unroll
        for (int k = 0; k < NS; ++k) dr[k] = h == 0 ? jt2[k] - jt1[k] : dr[k] + (jt2[k] - jt1[k]);
        if constexpr (h < 9) {
            // each link's friction is shared by its two cells (scaled by kT/2
            // below); directions 0, 1, 2 are the unit vectors x, y, z
            const T g = (g1 + g2) * (T)link_coef<h>();
            if constexpr (h < 3) fe[h] = g;
            else {
                if constexpr (ox > 0) fe[0] += g;
                if constexpr (ox < 0) fe[0] -= g;
                if constexpr (oy > 0) fe[1] += g;
                if constexpr (oy < 0) fe[1] -= g;
                if constexpr (oz > 0) fe[2] += g;
                if constexpr (oz < 0) fe[2] -= g;
            }
        }
    });
}

// Clean-window update gathered per neighbour.  The same fluxes as
// ek_cell_update, summed in another order: for the neighbours n = a + d of
// cell a (26 of them), with R the full density (r + mean when DEV stores
// deviations r from the mean, r itself otherwise),
//   advective: the outgoing part, sum_d R_a g(d; u_a), is R_a (1 - g(0; u_a))
//     (a cell's fractions over its 27 destinations add up to one), so only
//     the incoming parts R_n g(-d; u_n) are gathered;
//   diffusive/migrative (D3Q19 d): g_k = (r_a - r_n) + z_k/2 (R_a + R_n)
//     (phi_a - phi_n + E.d) is summed per link length, whose factor
//     D_k/(A0|d|) is applied once;
//   friction: sum_d d sum_k g_k, per link length.
// Each link's flux is then not rounded on its own, so the two cells of a link
// no longer hand over bitwise equal amounts: the species totals move by the
// rounding of each cell's sums, ~1e-7 of that cell's fluxes.
template <typename T, bool DEV, int NS, typename SH>
__device__ __forceinline__ void ek_cell_update_gather(const SH& sh, int s0, int sm, int sp, int ctr,
                                                      const EKConst<T, NS>& K, T (&dr)[NS], T (&fe)[3]) {
    const RecEK<T, NS> me = sh.get(s0, ctr);
    T G[NS][2], adv[NS], hzC[NS], F[2][3] = {{(T)0, (T)0, (T)0}, {(T)0, (T)0, (T)0}}, gin = (T)0;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        G[k][0] = G[k][1] = adv[k] = (T)0;
        // the cell's share of z/2 (R_a + R_n): z/2 (r_a + 2 mean) for deviations
        hzC[k] = DEV ? K.hz[k] * (me.r(k) + K.ref[k] * (T)2) : K.hz[k] * me.r(k);
    }
    sfor<13>([&](auto HH) {
        constexpr int h = HH;
        constexpr int c = hlen(h) > 1.0 ? 1 : 0;
        auto one = [&](auto SG) {
            constexpr int sg = SG;
            constexpr int dx = sg * hx(h), dy = sg * hy(h), dz = sg * hz(h);
            const int slot = dz == 0 ? s0 : (dz > 0 ? sp : sm);
            const RecEK<T, NS> n = sh.get(slot, ctr + dy * SH::WX + dx);
            const T gn = vof_frac<T, -dx, -dy, -dz>(n.ux(), n.uy(), n.uz());
            gin += gn;
#pragma unroll
            for (int k = 0; k < NS; ++k) adv[k] = fmt(n.r(k), gn, adv[k]);
            if constexpr (h < 9) {
                const T dphi = (me.phi() - n.phi()) + (sg > 0 ? K.Es[h] : -K.Es[h]);
                T gs = (T)0;
#pragma unroll
                for (int k = 0; k < NS; ++k) {
                    const T m = fmt(K.hz[k], n.r(k), hzC[k]);
                    const T g = fmt(m, dphi, me.r(k) - n.r(k));
                    G[k][c] += g;
                    gs = k == 0 ? g : gs + g;
                }
                if constexpr (dx > 0) F[c][0] += gs;
                if constexpr (dx < 0) F[c][0] -= gs;
                if constexpr (dy > 0) F[c][1] += gs;
                if constexpr (dy < 0) F[c][1] -= gs;
                if constexpr (dz > 0) F[c][2] += gs;
                if constexpr (dz < 0) F[c][2] -= gs;
            }
        };
        one(std::integral_constant<int, 1>{});
        one(std::integral_constant<int, -1>{});
    });
    // Leaving fraction: the sum of the 26 fractions g(d; u_a) that the
    // neighbours gather, with a_i = |u_i| and b_i = 1 - |u_i| rounded as
    // there: a_x (a_y + b_y)(a_z + b_z) + b_x (a_y (a_z + b_z) + b_y a_z).
    // (1 - b_x b_y b_z would carry the rounding of each b_i, ~1e-8 absolute,
    // into every step's solute balance.)
    const T ax = fabs(me.ux()), ay = fabs(me.uy()), az = fabs(me.uz());
    const T bx = vof_axis<T, 0>(me.ux()), by = vof_axis<T, 0>(me.uy()), bz = vof_axis<T, 0>(me.uz());
    const T sz = az + bz;
    const T out = fmt(ax, (ay + by) * sz, bx * fmt(ay, sz, by * az));
    const T dg = gin - out;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        T d = fmt(-me.r(k), out, adv[k]);
        if constexpr (DEV) d = fmt(K.ref[k], dg, d);  // mean * (in - out)
        d = fmt(-K.Dc[k][1], G[k][1], d);
        dr[k] = fmt(-K.Dc[k][0], G[k][0], d);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) fe[d] = fmt((T)link_coef<3>(), F[1][d], (T)link_coef<0>() * F[0][d]);
}

// Boundary-cell sources of one cell's populations from the staged flags.
template <typename T, int NS, int TXW, int TYW>
__device__ __forceinline__ unsigned lb_bmask_lds(const EKShared<T, NS, TXW, TYW>& sh, int ctr, int s0, int sm,
                                                 int sp) {
    using SH = EKShared<T, NS, TXW, TYW>;
    unsigned m = 0;
    sfor<19>([&](auto I) {
        constexpr int i = I;
        if constexpr (i > 0) {
            constexpr int cx = q19x(i), cy = q19y(i), cz = q19z(i);
            const int slot = cz > 0 ? sm : (cz < 0 ? sp : s0);
            m |= (unsigned)sh.wall(slot, ctr - cy * SH::WX - cx) << i;
        }
    });
    return m;
}

// Block-wide OR of a predicate through one LDS word per wave.  (The runtime's
// __syncthreads_or reads the block size from memory and so waits for every
// outstanding vector memory operation, the stores of the plane just finished
// and the loads of the plane being fetched among them.)  w must not be
// written again before every wave has read it: callers alternate between
// arrays separated by other barriers.
template <int NW>
__device__ __forceinline__ bool block_any(int (&w)[NW], bool p) {
    const int wave_any = __any(p);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = wave_any;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) r |= w[i];
    return r != 0;
}

// Grid: tiles of TXW x TYW cells in x-y times z-chunks of ZC planes, flattened
// and mapped with xcd_tile; each workgroup marches its ZC planes.
// FUSE: the cell's LB stream/collide follows its EK update in the same thread,
// with the coupling force taken from registers (the force field is still
// written for readers of the state).  The velocity the EK advection reads
// (u[cur]) and the one LB writes (u[cur^1]) are different buffers, so the
// order of cells across workgroups does not matter.  The populations of a
// cell are requested at the start of its z-iteration, before the next plane
// is staged, so that their latency overlaps the staging and the flux work
// (PREFETCH), or after the flux work (fewer registers live across it).
template <typename T, bool DEV, int NS, int TXW, int TYW, bool FUSE, bool PREFETCH = true>
__device__ __forceinline__ void ek_body(const Sim<T>& s, int bx_, int by_, int gx_, int ZC, int gx, int gy, int ntiles) {
    using SH = EKShared<T, NS, TXW, TYW>;
    constexpr int NW = TXW * TYW / 64;
    __shared__ SH sh;
    __shared__ int wany[3][NW];  // per slot, for block_any
    const int tile = xcd_tile(bx_, ntiles);
    const int bx = tile % gx, by = (tile / gx) % gy, bz = tile / (gx * gy);
    const int x0 = bx * TXW, y0 = by * TYW, zbeg = bz * ZC;
    const T* __restrict__ rin = s.rho[s.cur];
    T* __restrict__ rout = s.rho[s.cur ^ 1];
    const EKConst<T, NS> K = ek_consts<T, NS>(s);
    const T half_kT = (T)(0.5 * s.kT);
    const PlaneMap<T, NS, TXW, TYW> pm(s, x0, y0);
    {
        bool d0 = ek_load_plane<T, NS, TXW, TYW>(s, sh, (zbeg + 2) % 3, pm, zbeg - 1, rin);
        bool d1 = ek_load_plane<T, NS, TXW, TYW>(s, sh, zbeg % 3, pm, zbeg, rin);
        const int a0 = block_any<NW>(wany[(zbeg + 2) % 3], d0), a1 = block_any<NW>(wany[zbeg % 3], d1);
        if (threadIdx.x == 0) {
            sh.dirty[(zbeg + 2) % 3] = a0;
            sh.dirty[zbeg % 3] = a1;
        }
    }
    const int tx = threadIdx.x % TXW, ty = threadIdx.x / TXW;
    const int x = x0 + tx, y = y0 + ty;
    const bool valid = x < s.nx && y < s.ny;
    const int ctr = (ty + 1) * SH::WX + (tx + 1);
    const int zend = zbeg + ZC < s.nz ? zbeg + ZC : s.nz;
    for (int z = zbeg; z < zend; ++z) {
        const int sm = (z + 2) % 3, s0 = z % 3, sp = (z + 1) % 3;
        // plane z is staged since the previous iteration
        const bool wall = valid && sh.wall(s0, ctr);
        T fi[FUSE ? 19 : 1];
        if constexpr (FUSE && PREFETCH) {
            if (valid && !wall) lb_pull(s, Nbr(x, y, z, s.nx, s.ny, s.nz), fi);
        }
        bool dn = ek_load_plane<T, NS, TXW, TYW>(s, sh, sp, pm, z + 1, rin);
        const int an = block_any<NW>(wany[sp], dn);
        if (threadIdx.x == 0) sh.dirty[sp] = an;
        __syncthreads();
        const bool clean = !(sh.dirty[0] | sh.dirty[1] | sh.dirty[2]);
        if (valid) {
            const uint32_t c = cidx32(s, x, y, z);
            T dr[NS];
            T fe[3] = {(T)0, (T)0, (T)0};
#pragma unroll
            for (int k = 0; k < NS; ++k) dr[k] = (T)0;
            if (clean)
                ek_cell_update_gather<T, DEV, NS>(sh, s0, sm, sp, ctr, K, dr, fe);
            else if (!wall)
                ek_cell_update<T, DEV, NS>(s, sh, s0, sm, sp, ctr, K, dr, fe);
            fe[0] *= half_kT;
            fe[1] *= half_kT;
            fe[2] *= half_kT;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                T out;
                if (wall) out = DEV ? (T)(-s.rho_ref[k]) : (T)0;
                else out = sh.elem(s0, ctr, k) + dr[k];
                st32_nt(rout + (long)k * s.N, c, out);
            }
            T* fc = s.fext + vidx(0, c);
            gst_nt(fc, fe[0]);
            gst_nt(fc + FB, fe[1]);
            gst_nt(fc + 2 * FB, fe[2]);
            if constexpr (FUSE) {
                if (wall) {
                    lb_wall(s, c);
                } else {
                    const Nbr nb(x, y, z, s.nx, s.ny, s.nz);
                    if constexpr (!PREFETCH) lb_pull(s, nb, fi);
                    const unsigned bmask = clean ? 0u : lb_bmask_lds<T, NS, TXW, TYW>(sh, ctr, s0, sm, sp);
                    lb_collide<T, DEV>(s, c, nb, fi, bmask, fe[0], fe[1], fe[2]);
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// FP32 EK pass with the staging of the window pipelined: the loads of plane
// z + 2 are issued into registers before plane z is computed and written to
// LDS after it (into the slot of plane z - 1), so their latency hides behind
// the flux work of the same workgroup.  Every thread holds the dirty mask of
// the three staged planes (the result of the block-wide OR), so a plane costs
// two barriers.
// ---------------------------------------------------------------------------
template <int NS, int TXW, int TYW>
struct PlaneRegs {
    static constexpr int NR = PlaneMap<float, NS, TXW, TYW>::NR;
    float v[NR][NS + 5];  // densities, potential, Psi, velocity
    uint8_t fl[NR];
};

template <int NS, int TXW, int TYW>
__device__ __forceinline__ void plane_issue(const Sim<float>& s, const PlaneMap<float, NS, TXW, TYW>& pm, int z,
                                            const float* __restrict__ rin, PlaneRegs<NS, TXW, TYW>& pr) {
    using PM = PlaneMap<float, NS, TXW, TYW>;
    using SH = EKShared<float, NS, TXW, TYW>;
    const uint32_t zoff = (uint32_t)wrap1(z, s.nz) * ((uint32_t)s.nx * (uint32_t)s.ny);  // z in [-1, nz]
    const float* __restrict__ ui = s.u[s.cur];
#pragma unroll
    for (int rr = 0; rr < PM::NR; ++rr) {
        if ((rr + 1) * PM::NT > SH::WPL && threadIdx.x + rr * PM::NT >= SH::WPL) continue;
        const uint32_t c = pm.at(s, rr) + zoff;
#pragma unroll
        for (int k = 0; k < NS; ++k) pr.v[rr][k] = ld32(rin + (long)k * s.N, c);
        pr.v[rr][NS] = ld32(s.phi, c);
        pr.v[rr][NS + 1] = ld32(s.psi, c);
        const float* uc = ui + vidx(0, c);
        pr.v[rr][NS + 2] = gld(uc);
        pr.v[rr][NS + 3] = gld(uc + FB);
        pr.v[rr][NS + 4] = gld(uc + 2 * FB);
        pr.fl[rr] = ld32(s.flag, c);
    }
}

// Stage the loaded records; returns whether they hold a boundary cell or a
// partial volume.
template <int NS, int TXW, int TYW>
__device__ __forceinline__ bool plane_commit(EKShared<float, NS, TXW, TYW>& sh, int slot,
                                             const PlaneRegs<NS, TXW, TYW>& pr) {
    using PM = PlaneMap<float, NS, TXW, TYW>;
    using SH = EKShared<float, NS, TXW, TYW>;
    // Every load of the plane has landed, on every path: without this wait
    // (s_waitcnt vmcnt(0)) here, the compiler would see loads possibly in
    // flight at the next plane's loads into the same registers and wait
    // there, after this plane's stores.
    __builtin_amdgcn_s_waitcnt(0x0F70);
    bool dirty = false;
#pragma unroll
    for (int rr = 0; rr < PM::NR; ++rr) {
        const int t = threadIdx.x + rr * PM::NT;
        if ((rr + 1) * PM::NT > SH::WPL && t >= SH::WPL) continue;
        RecEK<float, NS> r;
#pragma unroll
        for (int k = 0; k < NS + 5; ++k) r.v[k] = pr.v[rr][k];
        const bool wall = (pr.fl[rr] & F_CUR) != 0;
        r.v[NS + 5] = wall ? 1.0f : 0.0f;
#pragma unroll
        for (int k = NS + 6; k < RecEK<float, NS>::NV; ++k) r.v[k] = 0.0f;
        sh.put(slot, t, r);
        dirty |= (pr.v[rr][NS + 1] != 0.0f) || wall;
    }
    return dirty;
}


template <int NS, int TXW, int TYW>
__device__ __forceinline__ void ek_body_pipe(const Sim<float>& s, int bx_, int ZC, int gx, int gy, int ntiles) {
    using SH = EKShared<float, NS, TXW, TYW>;
    constexpr int NW = TXW * TYW / 64;
    __shared__ SH sh;
    __shared__ int wany[3][NW];  // per slot, for block_any
    const int tile = xcd_tile(bx_, ntiles);
    const int bx = tile % gx, by = (tile / gx) % gy, bz = tile / (gx * gy);
    const int x0 = bx * TXW, y0 = by * TYW, zbeg = bz * ZC;
    const int zend = zbeg + ZC < s.nz ? zbeg + ZC : s.nz;
    const float* __restrict__ rin = s.rho[s.cur];
    float* __restrict__ rout = s.rho[s.cur ^ 1];
    const EKConst<float, NS> K = ek_consts<float, NS>(s);
    const float half_kT = (float)(0.5 * s.kT);
    const PlaneMap<float, NS, TXW, TYW> pm(s, x0, y0);
    PlaneRegs<NS, TXW, TYW> pr;
    // planes zbeg - 1, zbeg, zbeg + 1 in slots (z + 3) mod 3
    unsigned dm = 0;
    for (int i = -1; i <= 1; ++i) {
        plane_issue<NS, TXW, TYW>(s, pm, zbeg + i, rin, pr);
        const int slot = (zbeg + i + 3) % 3;
        dm |= (unsigned)block_any<NW>(wany[slot], plane_commit<NS, TXW, TYW>(sh, slot, pr)) << slot;
    }
    const int tx = threadIdx.x % TXW, ty = threadIdx.x / TXW;
    const int x = x0 + tx, y = y0 + ty;
    const bool valid = x < s.nx && y < s.ny;
    const int ctr = (ty + 1) * SH::WX + (tx + 1);
    // One plane; MORE: a plane follows (stage plane z + 2).  The last plane is
    // peeled off, so that on every path into the next plane's loads those of
    // this plane have been waited for (else the wait before them would also
    // cover this plane's stores).
    auto plane = [&](int z, auto MORE) {
        constexpr bool more = decltype(MORE)::value;
        const int sm = (z + 2) % 3, s0 = z % 3, sp = (z + 1) % 3;
        if constexpr (more) plane_issue<NS, TXW, TYW>(s, pm, z + 2, rin, pr);
        float out[NS], fe[3] = {0.0f, 0.0f, 0.0f};
        if (valid) {
            const bool wall = sh.wall(s0, ctr);
            float dr[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) dr[k] = 0.0f;
            if (dm == 0)
                ek_cell_update_gather<float, true, NS>(sh, s0, sm, sp, ctr, K, dr, fe);
            else if (!wall)
                ek_cell_update<float, true, NS>(s, sh, s0, sm, sp, ctr, K, dr, fe);
#pragma unroll
            for (int k = 0; k < NS; ++k) out[k] = wall ? -K.ref[k] : sh.elem(s0, ctr, k) + dr[k];
        }
        // stage plane z + 2 over plane z - 1, then store this plane's results
        // (issued after the wait for the staged loads, so that wait does not
        // also cover these stores)
        bool dnew = false;
        if constexpr (more) {
            __syncthreads();  // plane z - 1 (slot sm) is read no more
            dnew = plane_commit<NS, TXW, TYW>(sh, sm, pr);
        }
        if (valid) {
            const uint32_t c = cidx32(s, x, y, z);
#pragma unroll
            for (int k = 0; k < NS; ++k) st32_nt(rout + (long)k * s.N, c, out[k]);
            float* fc = s.fext + vidx(0, c);
            gst_nt(fc, fe[0] * half_kT);
            gst_nt(fc + FB, fe[1] * half_kT);
            gst_nt(fc + 2 * FB, fe[2] * half_kT);
        }
        if constexpr (more) dm = (dm & ~(1u << sm)) | ((unsigned)block_any<NW>(wany[sm], dnew) << sm);
    };
    for (int z = zbeg; z + 1 < zend; ++z) plane(z, std::true_type{});
    plane(zend - 1, std::false_type{});
}

// At least two waves per SIMD: keeps the FP64 fused kernel from spilling into
// accumulation registers past the 256-register budget of that occupancy.
template <typename T, bool DEV, int NS, int TXW, int TYW, bool FUSE, bool PREFETCH>
__global__ __launch_bounds__(TXW* TYW) __attribute__((amdgpu_waves_per_eu(2))) void k_ek(Sim<T> s, int ZC, int gx,
                                                                                          int gy, int ntiles) {
    ek_body<T, DEV, NS, TXW, TYW, FUSE, PREFETCH>(s, blockIdx.x, blockIdx.y, gridDim.x, ZC, gx, gy, ntiles);
}

// FP32.  (Capping it at 128 registers for a fourth wave per SIMD spills and
// runs slower.)
template <int NS, int TXW, int TYW>
__global__ __launch_bounds__(TXW* TYW) void k_ek32(
    Sim<float> s, int ZC, int gx, int gy, int ntiles) {
    ek_body_pipe<NS, TXW, TYW>(s, blockIdx.x, ZC, gx, gy, ntiles);
}

// ---------------------------------------------------------------------------
// Launchers.  FP64 runs the fused EK+LB kernel (populations pulled after the
// flux work): the flux work is ALU-bound and the stream/collide HBM-bound, and
// at FP64 register counts the interleaving pays (about 15 % over two
// kernels).  In FP32 two kernels are faster: the stand-alone LB kernel streams
// whole 1 KB rows per population at higher occupancy than the tiled fused pass.
// ---------------------------------------------------------------------------
template <typename T> constexpr bool kFuseFields = sizeof(T) == 8;
template <typename T> constexpr bool kPrefetch = false;

// Planes per workgroup of the FP32 EK pass: the tile columns are cut into as
// many z-ranges as make the grid one full round of the workgroups the device
// holds at once (a partial last round idles the rest of the chip, and each
// range pays its three-plane prologue once), with at least MIN_ZC planes per
// range.  Workgroups per CU and the CU count are queried once per process.
template <int NS>
static int ek32_planes(int columns, int nz) {
    constexpr int TXW = EKTile<float>::TXW, TYW = EKTile<float>::TYW, MIN_ZC = 4;
    static int slots = 0;
    if (slots == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ek32<NS, TXW, TYW>, TXW * TYW, 0) != hipSuccess ||
            cus <= 0 || per_cu <= 0)
            return EKTile<float>::ZC;
        slots = cus * per_cu;
    }
    int k = (slots + columns / 2) / columns;  // z-ranges per column
    const int kmax = (nz + MIN_ZC - 1) / MIN_ZC;
    k = k < 1 ? 1 : (k > kmax ? kmax : k);
    return (nz + k - 1) / k;
}

template <typename T, bool DEV, int NS, bool FUSE>
static void launch_ek_ns(const Sim<T>& s, hipStream_t st) {
    constexpr int TXW = EKTile<T>::TXW, TYW = EKTile<T>::TYW;
    Grids<T> g = grids_of<T>(s);
    if constexpr (sizeof(T) == 4 && DEV && !FUSE) {
        const int zc = ek32_planes<NS>(g.ek_gx * g.ek_gy, s.nz);
        const int nt = g.ek_gx * g.ek_gy * ((s.nz + zc - 1) / zc);
        hipLaunchKernelGGL((k_ek32<NS, TXW, TYW>), dim3(nt), dim3(TXW * TYW), 0, st, s, zc, g.ek_gx, g.ek_gy, nt);
    } else {
        const int nt = g.n[KK_EK];
        hipLaunchKernelGGL((k_ek<T, DEV, NS, TXW, TYW, FUSE, kPrefetch<T>>), dim3(nt), dim3(TXW * TYW), 0, st, s,
                           EKTile<T>::ZC, g.ek_gx, g.ek_gy, nt);
    }
}

template <typename T, bool FUSE>
static void launch_ek(const Sim<T>& s, hipStream_t st) {
    constexpr bool DEV = sizeof(T) == 4;
    switch (s.ns) {
        case 1: launch_ek_ns<T, DEV, 1, FUSE>(s, st); break;
        case 2: launch_ek_ns<T, DEV, 2, FUSE>(s, st); break;
        case 3: launch_ek_ns<T, DEV, 3, FUSE>(s, st); break;
        default: launch_ek_ns<T, DEV, 4, FUSE>(s, st); break;
    }
}

template <typename T>
void launch_fields(const Sim<T>& s, hipStream_t st, hipEvent_t mid) {
    constexpr bool DEV = sizeof(T) == 4;
    launch_ek<T, kFuseFields<T>>(s, st);
    if (mid) (void)hipEventRecord(mid, st);
    if constexpr (!kFuseFields<T>) launch_lb(s, st);
}

// ---------------------------------------------------------------------------
// Batched EK and LB (FP32 tables), same split as the single-simulation path.
// ---------------------------------------------------------------------------
constexpr int BATCH_FIELD_BLOCKS = 2048;
constexpr bool FLAT_EK = false;

// (Four waves per SIMD with a few registers spilled served about 3.5 % more
// cells per second before the staging was pipelined; with the loads of the
// next plane in flight, a spill reload waits for them, so the compiler's
// choice stands.)
template <int NS>
__global__ __launch_bounds__(EKTile<float>::TXW* EKTile<float>::TYW) void kb_ek(const BatchTable* __restrict__ tab) {
    constexpr int TXW = EKTile<float>::TXW, TYW = EKTile<float>::TYW, ZC = EKTile<float>::ZC;
    batch_run<KK_EK, FLAT_EK>(tab, [](const Sim<float>& s, int b) {
        const int gx = (s.nx + TXW - 1) / TXW, gy = (s.ny + TYW - 1) / TYW;
        const int nt = gx * gy * ((s.nz + ZC - 1) / ZC);
        ek_body_pipe<NS, TXW, TYW>(s, b, ZC, gx, gy, nt);
    });
}

void launch_batch_fields(const BatchTable* tab, const int* items, int ns, hipStream_t st) {
    constexpr int NT = EKTile<float>::TXW * EKTile<float>::TYW;
    switch (ns) {
        case 1: hipLaunchKernelGGL(kb_ek<1>, dim3(batch_grid(FLAT_EK, items[KK_EK], (const void*)kb_ek<1>, NT, 0, BATCH_FIELD_BLOCKS)), dim3(NT), 0, st, tab); break;
        case 2: hipLaunchKernelGGL(kb_ek<2>, dim3(batch_grid(FLAT_EK, items[KK_EK], (const void*)kb_ek<2>, NT, 0, BATCH_FIELD_BLOCKS)), dim3(NT), 0, st, tab); break;
        case 3: hipLaunchKernelGGL(kb_ek<3>, dim3(batch_grid(FLAT_EK, items[KK_EK], (const void*)kb_ek<3>, NT, 0, BATCH_FIELD_BLOCKS)), dim3(NT), 0, st, tab); break;
        default: hipLaunchKernelGGL(kb_ek<4>, dim3(batch_grid(FLAT_EK, items[KK_EK], (const void*)kb_ek<4>, NT, 0, BATCH_FIELD_BLOCKS)), dim3(NT), 0, st, tab); break;
    }
    if constexpr (!kFuseFields<float>) launch_batch_lb(tab, items, st);
}

template void launch_fields<float>(const Sim<float>&, hipStream_t, hipEvent_t);
template void launch_fields<double>(const Sim<double>&, hipStream_t, hipEvent_t);

}  // namespace ek
