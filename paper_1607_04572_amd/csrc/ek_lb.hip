// ek_lb.hip -- the stand-alone LB stream/collide kernel (FP32 path) and its
// batched form; the cell update itself is in ek_lb.h.
#include "ek_lb.h"

namespace ek {

// Workgroup b covers cells [256 (b mod nbp), 256 (b mod nbp) + 256) of plane
// z = b div nbp, nbp = ceil(nx ny / 256); the in-plane division by nx is
// exact by multiply-high (nx ny nx < 2^27).
template <typename T, bool DEV>
__device__ __forceinline__ void lb_body(const Sim<T>& s, int bx_, int by_, int gx_) {
    const int nx = s.nx, ny = s.ny, P = nx * ny;
    const int nbp = (P + BT - 1) / BT;
    const int z = bx_ / nbp;
    const int cp = (bx_ - z * nbp) * BT + threadIdx.x;
    if (cp >= P) return;
    const int y = FDiv(nx).div(cp);
    const uint32_t c = (uint32_t)z * (uint32_t)P + (uint32_t)cp;
    const Nbr nb(cp - y * nx, y, z, nx, ny, s.nz);
    // all loads first (a boundary cell's pulls are wasted, but harmless),
    // boundary fix-ups (rare) afterwards
    T fi[19];
    lb_pull(s, nb, fi);
    const uint8_t fl = ld32(s.flag, c);
    const T* fc = s.fext + vidx(0, c);
    const T fx = gld(fc), fy = gld(fc + FB), fz = gld(fc + 2 * FB);
    if (fl & F_CUR) {
        lb_wall(s, c);
        return;
    }
    lb_collide<T, DEV>(s, c, nb, fi, lb_bmask_global(s, nb), fx, fy, fz);
}

template <typename T, bool DEV>
__global__ __launch_bounds__(BT) void k_lb(Sim<T> s) {
    lb_body<T, DEV>(s, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
void launch_lb(const Sim<T>& s, hipStream_t st) {
    constexpr bool DEV = sizeof(T) == 4;
    hipLaunchKernelGGL((k_lb<T, DEV>), dim3((unsigned)grids_of<T>(s).n[KK_LB]), dim3(BT), 0, st, s);
}

constexpr int BATCH_LB_BLOCKS = 2048;
// One workgroup per 256-cell chunk: a persistent grid walking the chunks
// streams about 20 % slower (601 against 494 us on one 256^3 box).
constexpr bool FLAT_LB = true;

__global__ __launch_bounds__(BT) void kb_lb(const BatchTable* __restrict__ tab) {
    batch_run<KK_LB, FLAT_LB>(tab, [](const Sim<float>& s, int b) { lb_body<float, true>(s, b, 0, 0); });
}

void launch_batch_lb(const BatchTable* tab, const int* items, hipStream_t st) {
    const int grid = batch_grid(FLAT_LB, items[KK_LB], (const void*)kb_lb, BT, 0, BATCH_LB_BLOCKS);
    hipLaunchKernelGGL(kb_lb, dim3(grid), dim3(BT), 0, st, tab);
}

template void launch_lb<float>(const Sim<float>&, hipStream_t);
template void launch_lb<double>(const Sim<double>&, hipStream_t);

}  // namespace ek
