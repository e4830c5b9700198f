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
//
// Per work item the chain of dependent memory accesses is kept short: the
// 256-byte descriptor of the next item is fetched with one vector load (a
// dword per lane) while the current item runs, and its fields are read from
// the lanes; the work list is read two items ahead; the node type and the
// nine populations are loaded together (the guard zones around every
// request's lattices keep the plain-neighbour loads of an in-domain node
// inside its memory).  Each XCD (blocks are dealt to the 8 XCDs round robin)
// takes a contiguous band of the work list, so the tiles it runs side by
// side share their halo lines in its L2.  On one 4096 x 1024 request this
// runs 1.15x, on sixteen 1024 x 512 requests 1.46x the first form of the
// kernel (one scalar descriptor read chain per item, list order).
#include <cstddef>

#include "lbm_batched.hpp"
#include "lbm_device.hpp"
#include "lbm_edges.hpp"

namespace lbm {

// The descriptor's pointers are generic (loaded from memory, not kernel
// arguments); these views let the regular path use global-memory
// instructions instead of flat ones.
template <class T> using gptr = T __attribute__((address_space(1)))*;
template <class T> __device__ __forceinline__ gptr<const T> as_global(const T* q) { return (gptr<const T>)q; }
template <class T> __device__ __forceinline__ gptr<T> as_global(T* q) { return (gptr<T>)q; }

// Field F of a descriptor held one dword per lane (dv), at byte offset OFF:
// its dwords are read from their lanes (wavefront-uniform results).
template <class F, size_t OFF> __device__ __forceinline__ F from_lanes(uint32_t dv)
{
    static_assert(sizeof(F) % 4 == 0 && OFF % 4 == 0 && OFF + sizeof(F) <= 256, "dword-aligned descriptor field");
    struct Words {
        uint32_t u[sizeof(F) / 4];
    } w;
#pragma unroll
    for (int j = 0; j < (int)(sizeof(F) / 4); ++j) w.u[j] = __builtin_amdgcn_readlane(dv, (int)(OFF / 4) + j);
    return __builtin_bit_cast(F, w);
}

template <int L, class T>
__global__ void __launch_bounds__(256) k_batched(const SlotDesc* __restrict__ slots, const WorkItem* __restrict__ work,
                                                 const int32_t* __restrict__ n_work, int k)
{
    static_assert(sizeof(SlotDesc) == 256 && BATCH_TILE_X == 64, "one descriptor dword per lane of a wavefront");
    const int32_t nw = *n_work;
    const int32_t G = (int32_t)gridDim.x;
    int32_t w = blockIdx.x;
    if (w >= nw) return;
    const int lane = (int)threadIdx.x;
    const uint32_t unw = (uint32_t)nw;
    WorkItem cur = work[xcd_tile((uint32_t)w, unw)];
    WorkItem ahead = work[xcd_tile((uint32_t)min(w + G, nw - 1), unw)]; // always a valid entry
    uint32_t dv = reinterpret_cast<const uint32_t*>(slots + cur.slot)[lane];
    for (; w < nw; w += G) {
        const WorkItem it = cur;
        const uint32_t mine = dv;
        cur = ahead;
        dv = reinterpret_cast<const uint32_t*>(slots + cur.slot)[lane];
        ahead = work[xcd_tile((uint32_t)min(w + 2 * G, nw - 1), unw)];
        if (k >= from_lanes<int64_t, offsetof(SlotDesc, steps_left)>(mine)) continue; // uniform per block
        KParams p;
        p.g = from_lanes<Geometry, offsetof(SlotDesc, g)>(mine);
        p.ph = from_lanes<Physics, offsetof(SlotDesc, ph)>(mine);
        p.types = from_lanes<const uint8_t*, offsetof(SlotDesc, types)>(mine);
        p.links = from_lanes<const uint32_t*, offsetof(SlotDesc, links)>(mine);
        float* rin2 = from_lanes<float*, offsetof(SlotDesc, rin2)>(mine);
        const int parity = (int)((from_lanes<int64_t, offsetof(SlotDesc, steps_done)>(mine) + k) & 1);
        p.rin = rin2 ? rin2 + parity * p.g.ny : nullptr;
        p.rout = rin2 ? rin2 + (parity ^ 1) * p.g.ny : nullptr;
        void* lat0 = from_lanes<void*, offsetof(SlotDesc, lat)>(mine);
        void* lat1 = from_lanes<void*, offsetof(SlotDesc, lat) + sizeof(void*)>(mine);
        const T* src = (const T*)(parity ? lat1 : lat0);
        T* dst = (T*)(parity ? lat0 : lat1);
        const int x = it.x0 + (int)threadIdx.x;
        const int y = it.y0 + (int)threadIdx.y;
        if (x >= p.g.nx || y >= p.g.ny) continue;
        const int64_t n = (int64_t)y * p.g.px + x;
        const uint8_t t = as_global(p.types)[n];
        float f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int cx = dir_cx(i), cy = dir_cy(i);
            f[i] = ld(as_global(src)[lat_at<L>(i, n - cx - cy * p.g.px, p.g.P)]);
        }
        // the values are taken before the type test, so the compiler cannot
        // move the loads behind it
#pragma unroll
        for (int i = 0; i < 9; ++i) asm volatile("" : "+v"(f[i]));
        if (!(t & IRREGULAR)) {
            collide(f, p.ph.omc, p.ph.F);
            const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
            for (int i = 0; i < 9; ++i) as_global(dst)[lat_at<L>(i, n, p.g.P)] = enc<T>(f[i], rng.draw(i));
        } else if (updated(t)) {
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
