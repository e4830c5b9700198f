// k_batched.hip -- one launch advances every resident request of the serving
// engine by one lattice update (two-lattice tiled pull, the same per-node code
// as a single simulation, so a request's result does not depend on what else
// is resident).
//
// The grid is persistent (fixed at graph capture): blocks walk a work list of
// (slot, tile) items that the host rewrites between bundles, so one captured
// graph serves any membership.  Launch k of a bundle advances a slot only
// while k < its remaining updates, which stops every request at exactly its
// requested step count.
#include "lbm_batched.hpp"
#include "lbm_device.hpp"

namespace lbm {

template <int L, class T>
__global__ void __launch_bounds__(256) k_batched(const SlotDesc* __restrict__ slots, const WorkItem* __restrict__ work,
                                                 const int32_t* __restrict__ n_work, int k)
{
    const int32_t nw = *n_work;
    for (int32_t w = blockIdx.x; w < nw; w += gridDim.x) {
        const WorkItem it = work[w];
        const SlotDesc& d = slots[it.slot];
        if (k >= d.steps_left) continue; // uniform per block
        KParams p;
        p.g = d.g;
        p.ph = d.ph;
        p.types = d.types;
        p.links = d.links;
        const int parity = (int)((d.steps_done + k) & 1);
        p.rin = d.rin2 ? d.rin2 + parity * p.g.ny : nullptr;
        p.rout = d.rin2 ? d.rin2 + (parity ^ 1) * p.g.ny : nullptr;
        const T* src = (const T*)d.lat[parity];
        T* dst = (T*)d.lat[parity ^ 1];
        const int x = it.x0 + (int)threadIdx.x;
        const int y = it.y0 + (int)threadIdx.y;
        if (x >= p.g.nx || y >= p.g.ny) continue;
        const int64_t n = (int64_t)y * p.g.px + x;
        if (!(p.types[n] & IRREGULAR)) {
            float f[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int cx = dir_cx(i), cy = dir_cy(i);
                f[i] = ld(src[lat_at<L>(i, n - cx - cy * p.g.px, p.g.P)]);
            }
            collide(f, p.ph.omc, p.ph.F);
            const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
            for (int i = 0; i < 9; ++i) dst[lat_at<L>(i, n, p.g.P)] = enc<T>(f[i], rng.draw(i));
        } else if (updated(p.types[n])) {
            float f[9];
            const uint32_t lk = p.links[n];
            if (lk & LINK_GENERAL)
                gather_pull<L, ST_PULL>(p, src, x, y, n, f);
            else
                gather_linked<L, ST_PULL>(p, src, x, y, n, lk, f);
            record_inlet_density(p, x, y, f);
            collide(f, p.ph.omc, p.ph.F);
            const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
            for (int i = 0; i < 9; ++i) dst[lat_at<L>(i, n, p.g.P)] = enc<T>(f[i], rng.draw(i));
        }
    }
}

hipError_t launch_batched(int layout, int prec, const SlotDesc* slots, const WorkItem* work, const int32_t* n_work,
                          int k, int blocks, hipStream_t s)
{
    const dim3 blk(BATCH_TILE_X, BATCH_TILE_Y);
    return with_layout_storage(layout, prec, [&](auto L, auto TT) {
        hipLaunchKernelGGL((k_batched<decltype(L)::value, typename decltype(TT)::type>), dim3(blocks), blk, 0, s,
                           slots, work, n_work, k);
        return hipGetLastError();
    });
}

int batched_blocks(int layout, int prec)
{
    int dev = 0, cus = 0, per = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    const int threads = BATCH_TILE_X * BATCH_TILE_Y;
    const hipError_t e = with_layout_storage(layout, prec, [&](auto L, auto TT) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per, k_batched<decltype(L)::value, typename decltype(TT)::type>, threads, 0);
    });
    (void)hipGetLastError();
    if (e != hipSuccess || per <= 0) per = 4;
    return cus * per;
}

} // namespace lbm
