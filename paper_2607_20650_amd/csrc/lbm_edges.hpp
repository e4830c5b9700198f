// lbm_edges.hpp -- tile decomposition and the "buffer grid" of the
// one-lattice schemes (paper Section 3.3, NPOL / NSOL): every tile publishes
// the post-collision values that leave it through its four sides, and a reader
// whose pull source lies in another tile takes the value from there.  The
// buffers are double-buffered by step parity, so a tile never waits for, or
// races with, its neighbours inside one update.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

// ------------------------------------------------------------ tile mapping
// Consecutive workgroups are dealt round-robin to the 8 XCDs (each with its
// own L2).  Remap so that every XCD works on a contiguous band of tiles:
// vertically adjacent tiles then share halo rows in the same L2.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nb)
{
    constexpr uint32_t XCD = 8;
    const uint32_t per = nb / XCD;
    const uint32_t full = per * XCD;
    if (b >= full) return b; // ragged remainder keeps its place
    return (b % XCD) * per + b / XCD;
}

struct TileCoord {
    int bx, by;   // tile indices
    int x0, y0;   // first node of the tile
    int x1, y1;   // one past the last node of the tile (clipped to the domain)
};

__device__ __forceinline__ TileCoord tile_of_block(const Geometry& g)
{
    const uint32_t nb = (uint32_t)g.ntx * (uint32_t)g.nty;
    const uint32_t t = xcd_tile(blockIdx.x, nb);
    TileCoord c;
    c.by = (int)(t / (uint32_t)g.ntx);
    c.bx = (int)(t - (uint32_t)c.by * (uint32_t)g.ntx);
    c.x0 = c.bx * g.tx;
    c.y0 = c.by * g.ty;
    c.x1 = min((int64_t)(c.x0 + g.tx), g.nx);
    c.y1 = min((int64_t)(c.y0 + g.ty), g.ny);
    return c;
}

// ------------------------------------------------------- edge buffer access
// Edge buffers of one parity: X edges (left, right: values leaving with
// c_x = -1 / +1, indexed by c_y + 1) then Y edges (bottom, top: c_y = -1 / +1,
// indexed by c_x + 1).
__device__ __forceinline__ int64_t edge_x_at(const Geometry& g, int tile, int side, int r, int k)
{
    return (((int64_t)tile * 2 + side) * g.ty + r) * 3 + k;
}
__device__ __forceinline__ int64_t edge_y_at(const Geometry& g, int tile, int side, int col, int k)
{
    return edge_x_elems(g) + (((int64_t)tile * 2 + side) * g.tx + col) * 3 + k;
}

// Index of the edge-buffer entry holding f*_i of source node (sx, sy), which
// lies in another tile than the reader (reader tile column rbx).
__device__ __forceinline__ int64_t edge_src(const Geometry& g, int sx, int sy, int i, int rbx)
{
    const int tsx = sx / g.tx, tsy = sy / g.ty;
    const int tile = tsy * g.ntx + tsx;
    if (tsx != rbx) return edge_x_at(g, tile, dir_cx(i) > 0 ? 1 : 0, sy - tsy * g.ty, dir_cy(i) + 1);
    return edge_y_at(g, tile, dir_cy(i) > 0 ? 1 : 0, sx - tsx * g.tx, dir_cx(i) + 1);
}

// Write the values of an updated node that leave its tile.
template <class T>
__device__ __forceinline__ void edge_emit(const Geometry& g, const TileCoord& c, int x, int y, const float* f,
                                          T* __restrict__ eout)
{
    const int tile = c.by * g.ntx + c.bx;
    if (x == c.x0)
        for (int k = 0; k < 3; ++k) eout[edge_x_at(g, tile, 0, y - c.y0, k)] = st<T>(f[3 * k + 0]);
    if (x == c.x1 - 1)
        for (int k = 0; k < 3; ++k) eout[edge_x_at(g, tile, 1, y - c.y0, k)] = st<T>(f[3 * k + 2]);
    if (y == c.y0)
        for (int k = 0; k < 3; ++k) eout[edge_y_at(g, tile, 0, x - c.x0, k)] = st<T>(f[k]);
    if (y == c.y1 - 1)
        for (int k = 0; k < 3; ++k) eout[edge_y_at(g, tile, 1, x - c.x0, k)] = st<T>(f[6 + k]);
}

// Pull source with coordinates (same rules as pull_source).
__device__ __forceinline__ int pull_source_xy(const Geometry& g, const uint8_t* __restrict__ types, int x, int y,
                                              int i, int& sx, int& sy)
{
    sx = x - dir_cx(i);
    sy = y - dir_cy(i);
    if (sy < 0 || sy >= g.ny) {
        if (g.ya != AX_PERIODIC) return K_SOLID;
        sy = sy < 0 ? sy + (int)g.ny : sy - (int)g.ny;
    }
    if (sx < 0 || sx >= g.nx) {
        if (g.xa == AX_PERIODIC)
            sx = sx < 0 ? sx + (int)g.nx : sx - (int)g.nx;
        else if (g.xa == AX_INOUT && sx >= g.nx)
            sx = (int)g.nx - 1;
        else
            return K_SOLID;
    }
    const uint8_t t = node_type(types[(int64_t)sy * g.px + sx]);
    return t == T_SOLID ? K_SOLID : (t == T_INLET ? K_INLET : K_NODE);
}

} // namespace lbm
