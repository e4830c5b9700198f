// lbm_stage.hpp -- LDS staging of a tile's lattice region with 16-byte
// global accesses, for the kernels whose per-node accesses are not coalesced
// on their own: the push scheme's scattered stores, and the collision (AoS)
// layout, where the 9 values of a node sit together and a wavefront's access
// of one direction touches 64 records of 9 elements.
//
// The region of a 64 x ty tile with first node (x0, y0) holds every slot of
// grid rows y0 - 1 .. y0 + ty (region rows 0 .. ty + 1) and nodes
// x0 - 1 .. x0 + 64 (region records 0 .. 65).  A layout stores one grid row as
// segments of contiguous elements: stream 9 (one per direction plane, 1
// element per node), bundle 3 (one per bundle, 3 per node), collision 1 (9 per
// node).  Each segment is staged from the 16-byte boundary at or before its
// first element, so every global access of the staging is a whole, aligned
// 16-byte piece: the row pitch px is a multiple of 16 nodes, x0 of 64, and the
// plane / bundle strides of 64 elements.
#pragma once

#include <type_traits>

#include "lbm_device.hpp"

namespace lbm {

template <int L, class T> struct Stage {
    static constexpr int CH = 16 / (int)sizeof(T);                                        // elements per piece
    static constexpr int NSEG = L == L_STREAM ? 9 : (L == L_BUNDLE ? 3 : 1);              // segments per row
    static constexpr int SPN = L == L_STREAM ? 1 : (L == L_BUNDLE ? 3 : 9);               // elements per node
    static constexpr int BACK = (SPN + CH - 1) / CH * CH;   // a staged segment starts BACK elements before node x0
    static constexpr int LEAD = BACK - SPN;                 // elements before record 0 (node x0 - 1)
    static constexpr int SEG = (LEAD + 66 * SPN + CH - 1) / CH * CH; // staged elements per segment
    static constexpr int NCH = SEG / CH;                    // pieces per segment
    static constexpr int RROW = NSEG * SEG;                 // staged elements per region row

    static __host__ __device__ constexpr int seg(int i) { return L == L_STREAM ? i : (L == L_BUNDLE ? i / 3 : 0); }
    static __host__ __device__ constexpr int lane(int i) { return L == L_STREAM ? 0 : (L == L_BUNDLE ? i % 3 : i); }
    // staged element of slot i of region record c in region row r
    static __device__ __forceinline__ int at(int r, int c, int i) { return r * RROW + seg(i) * SEG + LEAD + c * SPN + lane(i); }
    // global element index of the first staged element of segment s of grid row y
    static __device__ __forceinline__ int64_t gbase(const Geometry& g, int64_t y, int x0, int s)
    {
        const int64_t plane = L == L_STREAM ? (int64_t)s * g.P : (L == L_BUNDLE ? (int64_t)s * 3 * g.P : 0);
        return plane + SPN * (y * g.px + x0) - BACK;
    }
    // one past the last element of the allocation (the lattice and its guard)
    static __device__ __forceinline__ int64_t limit(const Geometry& g)
    {
        return (L == L_COLLISION ? 9 * g.px * g.ny : 9 * g.P) + lattice_guard(g);
    }
    // the region rows, then one 16-byte slot (element dummy(ty)) that takes
    // the pieces a staging copy drops
    static constexpr int dummy(int ty) { return (ty + 2) * RROW; }
    static constexpr size_t bytes(int ty) { return (size_t)(ty + 2) * RROW * sizeof(T) + 16; }
};

// Copy region rows [r0, r1] (grid rows y0 - 1 + r) of the lattice into LDS,
// whole 16-byte pieces, all threads of the block taking part.  Pieces past
// the end of the allocation are skipped (nothing a node reads lies there).
template <int L, class T>
__device__ __forceinline__ void stage_load(const Geometry& g, const T* __restrict__ lat, T* s, int x0, int y0, int r0,
                                           int r1, int tid, int nthr)
{
    using S = Stage<L, T>;
    const int64_t lim = S::limit(g);
    const int per_row = S::NSEG * S::NCH;
    const int ty = nthr / 64; // blocks of 64 x ty threads
    pieces_to_lds<4>(lat, s, (r1 - r0 + 1) * per_row, S::dummy(ty), tid, nthr, [&](int k, int64_t& e, int& o) {
        const int rr = k / per_row, rem = k - rr * per_row;
        const int sg = rem / S::NCH, q = rem - sg * S::NCH;
        const int r = r0 + rr;
        e = S::gbase(g, (int64_t)(y0 - 1 + r), x0, sg) + (int64_t)q * S::CH;
        o = r * S::RROW + sg * S::SEG + q * S::CH;
        return e + S::CH <= lim;
    });
}

// Write back the staged elements whose mask byte is set, for region rows
// [r0, r1]: a piece with all its elements set leaves as one 16-byte store,
// any other element by element.  Only grid rows inside the domain are ever
// marked.
template <int L, class T>
__device__ __forceinline__ void stage_store_masked(const Geometry& g, T* __restrict__ lat, const T* s,
                                                   const uint8_t* mask, int x0, int y0, int r0, int r1, int tid,
                                                   int nthr)
{
    using S = Stage<L, T>;
    const int per_row = S::NSEG * S::NCH;
    for (int k = tid; k < (r1 - r0 + 1) * per_row; k += nthr) {
        const int rr = k / per_row, rem = k - rr * per_row;
        const int sg = rem / S::NCH, q = rem - sg * S::NCH;
        const int r = r0 + rr;
        const int o = r * S::RROW + sg * S::SEG + q * S::CH;
        // the CH mask bytes of a piece as one word (o is a multiple of CH)
        using MW = typename std::conditional<S::CH == 4, uint32_t, uint64_t>::type;
        const MW mw = *reinterpret_cast<const MW*>(mask + o);
        if (mw == 0) continue;
        const bool all = mw == (MW)0x0101010101010101ull;
        T* d = lat + S::gbase(g, (int64_t)(y0 - 1 + r), x0, sg) + (int64_t)q * S::CH;
        if (all) {
            *reinterpret_cast<uint4*>(d) = *reinterpret_cast<const uint4*>(s + o);
        } else {
#pragma unroll
            for (int j = 0; j < S::CH; ++j)
                if (mask[o + j]) d[j] = s[o + j];
        }
    }
}

} // namespace lbm
