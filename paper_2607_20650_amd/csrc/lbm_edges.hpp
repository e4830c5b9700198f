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
// Edge buffers of one parity, indexed by global row or column so that a
// reader needs no tile arithmetic beyond its neighbour's tile index:
//   X edges [tile column][side][c_y + 1][row]: values leaving a tile column
//           through its left (side 0, c_x = -1) or right (side 1, c_x = +1) side;
//   Y edges [tile row][side][c_x + 1][column]: values leaving a tile row
//           through its bottom (side 0, c_y = -1) or top (side 1, c_y = +1) side.
// A corner node publishes to both; readers take corners from the Y edges.
__device__ __forceinline__ int64_t edge_x_at(const Geometry& g, int bx, int side, int k, int y)
{
    return ((int64_t)(bx * 2 + side) * 3 + k) * edge_rows(g) + y;
}
__device__ __forceinline__ int64_t edge_y_at(const Geometry& g, int by, int side, int k, int x)
{
    return edge_x_elems(g) + ((int64_t)(by * 2 + side) * 3 + k) * edge_cols(g) + x;
}

// Entry holding f*_i of the source (sx, sy) (already wrapped or clamped into
// the domain) of a reader in tile c, the source lying outside tile c.
__device__ __forceinline__ int64_t edge_src(const Geometry& g, const TileCoord& c, int sx, int sy, int i)
{
    if (sy < c.y0 || sy >= c.y1) return edge_y_at(g, sy / g.ty, dir_cy(i) > 0 ? 1 : 0, dir_cx(i) + 1, sx);
    return edge_x_at(g, sx / g.tx, dir_cx(i) > 0 ? 1 : 0, dir_cy(i) + 1, sy);
}

// Whether the plain neighbour (x, y) - c_I of a node of tile c lies beyond
// the tile's bottom/top side (row) or its left/right side (column).
template <int I> __device__ __forceinline__ bool crosses_row(const TileCoord& c, int y)
{
    constexpr int Y = dir_cy(I);
    return Y > 0 ? y == c.y0 : (Y < 0 ? y == c.y1 - 1 : false);
}
template <int I> __device__ __forceinline__ bool crosses_col(const TileCoord& c, int x)
{
    constexpr int X = dir_cx(I);
    return X > 0 ? x == c.x0 : (X < 0 ? x == c.x1 - 1 : false);
}

// Entry of f*_I at the plain neighbour (x, y) - c_I of node (x, y) of tile
// c, for a neighbour inside the domain but outside the tile.
template <int I>
__device__ __forceinline__ int64_t edge_neighbour(const Geometry& g, const TileCoord& c, int x, int y)
{
    constexpr int X = dir_cx(I), Y = dir_cy(I);
    if (crosses_row<I>(c, y)) return edge_y_at(g, c.by - Y, Y > 0 ? 1 : 0, X + 1, x - X);
    return edge_x_at(g, c.bx - X, X > 0 ? 1 : 0, Y + 1, y - Y);
}

// The same entry with the direction's components as (inlined, constant
// folded) arguments: for a regular node, whose neighbour tile is the
// adjacent one, no division by the tile extents is needed.
__device__ __forceinline__ int64_t edge_neighbour_xy(const Geometry& g, const TileCoord& c, int x, int y, int X, int Y)
{
    const bool row = Y > 0 ? y == c.y0 : (Y < 0 ? y == c.y1 - 1 : false);
    if (row) return edge_y_at(g, c.by - Y, Y > 0 ? 1 : 0, X + 1, x - X);
    return edge_x_at(g, c.bx - X, X > 0 ? 1 : 0, Y + 1, y - Y);
}

// The same entry with tile indices and the row / column clamped into the
// buffers: a valid address for any node on a tile side, so the load can be
// issued before the node is known to be regular (for a regular node the
// clamps change nothing).
__device__ __forceinline__ int64_t edge_neighbour_clamped(const Geometry& g, const TileCoord& c, int x, int y, int X,
                                                          int Y)
{
    const bool row = Y > 0 ? y == c.y0 : (Y < 0 ? y == c.y1 - 1 : false);
    if (row)
        return edge_y_at(g, min(max(c.by - Y, 0), g.nty - 1), Y > 0 ? 1 : 0, X + 1,
                         min(max(x - X, 0), (int)edge_cols(g) - 1));
    return edge_x_at(g, min(max(c.bx - X, 0), g.ntx - 1), X > 0 ? 1 : 0, Y + 1,
                     min(max(y - Y, 0), (int)edge_rows(g) - 1));
}

// Write the values of an updated node that leave its tile.
template <class T>
__device__ __forceinline__ void edge_emit(const Geometry& g, const TileCoord& c, int x, int y, const float* f,
                                          T* __restrict__ eout)
{
    if (x == c.x0)
        for (int k = 0; k < 3; ++k) eout[edge_x_at(g, c.bx, 0, k, y)] = st<T>(f[3 * k + 0]);
    if (x == c.x1 - 1)
        for (int k = 0; k < 3; ++k) eout[edge_x_at(g, c.bx, 1, k, y)] = st<T>(f[3 * k + 2]);
    if (y == c.y0)
        for (int k = 0; k < 3; ++k) eout[edge_y_at(g, c.by, 0, k, x)] = st<T>(f[k]);
    if (y == c.y1 - 1)
        for (int k = 0; k < 3; ++k) eout[edge_y_at(g, c.by, 1, k, x)] = st<T>(f[6 + k]);
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
