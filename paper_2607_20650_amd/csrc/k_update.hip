// k_update.hip -- one lattice update per launch, for every scheme of the
// paper's Section 3.3 in each layout of Section 3.2 and each storage precision.
//
//   LPTL  linear pull, two lattices: a 1-D launch over all nodes, block size
//         left to the runtime's occupancy query.
//   NPTL  pull, two lattices, explicit 2-D decomposition into tiles of
//         tile_x * tile_y nodes (one tile per block); the grid is padded to
//         whole tiles and out-of-domain threads idle.
//   PUSH  one-step push, two lattices: each node collides its own incoming
//         values and scatters them to its neighbours.
//   NPOL  pull, ONE lattice: each thread keeps its node's incoming values in
//         registers, a block barrier separates all reads from all in-place
//         writes, and values crossing a tile edge travel through the "buffer
//         grid" of edge buffers (double-buffered by step parity, so tiles
//         never wait for each other).
//   NSOL  swap scheme, ONE lattice: every node keeps its post-collision value
//         of direction i in slot opposite(i); streaming is the exchange with
//         the neighbour's opposite slot in each direction, done in LDS inside a
//         tile and through the same edge buffers across tiles.  A solid
//         neighbour does not exchange, which is exactly halfway bounce-back.
//
// All schemes call the same collide(), so they agree bit for bit.
#include "lbm_device.hpp"
#include "lbm_edges.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// ------------------------------------------------- NPTL, vectorised
// Each thread updates VX consecutive nodes of one row (VX * sizeof(T) = 16
// bytes), so every plane / bundle / node run moves with 16-byte accesses.
// Runs of VX regular nodes (no IRREGULAR mark: interior fluid, all pull
// sources plain fluid nodes in range) pull with fixed offsets and no flag
// lookups; any other run falls back to the per-node boundary rules.
template <int VX>
__device__ __forceinline__ bool all_regular(const uint8_t* __restrict__ t)
{
    if constexpr (VX == 8) {
        const uint2 v = *reinterpret_cast<const uint2*>(t);
        return ((v.x | v.y) & 0x80808080u) == 0;
    } else if constexpr (VX == 4) {
        return (*reinterpret_cast<const uint32_t*>(t) & 0x80808080u) == 0;
    } else {
        bool r = true;
#pragma unroll
        for (int k = 0; k < VX; ++k) r = r && !(t[k] & IRREGULAR);
        return r;
    }
}

// Incoming populations of VX regular nodes starting at (x0, y), node n0.
template <int L, class T, int VX>
__device__ __forceinline__ void pull_regular(const KParams& p, const T* __restrict__ src, int64_t y, int64_t n0,
                                             float (*f)[9])
{
    const int64_t P = p.g.P, px = p.g.px;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int64_t r = n0 + (1 - b) * px; // node index of (x0, y - c_y) with c_y = b - 1
        if constexpr (L == L_STREAM) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int i = 3 * b + k;
                float v[VX];
                if (k == 1)
                    vload<T, VX, true>(src + (int64_t)i * P + r, v);
                else
                    vload<T, VX, false>(src + (int64_t)i * P + r - (k - 1), v);
#pragma unroll
                for (int c = 0; c < VX; ++c) f[c][i] = v[c];
            }
        } else if constexpr (L == L_BUNDLE) {
            const T* base = src + (int64_t)b * 3 * P + 3 * r;
            float span[3 * VX];
            vload_run<T, 3 * VX>(base, span);
            const float left = ld(base[-1]);      // node x0-1, k = 2
            const float right = ld(base[3 * VX]); // node x0+VX, k = 0
#pragma unroll
            for (int c = 0; c < VX; ++c) {
                f[c][3 * b + 0] = c + 1 < VX ? span[3 * (c + 1)] : right;
                f[c][3 * b + 1] = span[3 * c + 1];
                f[c][3 * b + 2] = c > 0 ? span[3 * (c - 1) + 2] : left;
            }
        } else {
#pragma unroll
            for (int c = 0; c < VX; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) f[c][3 * b + k] = ld(src[9 * (r + c - (k - 1)) + 3 * b + k]);
        }
    }
}

template <int L, class T, int VX>
__device__ __forceinline__ void store_run(const KParams& p, T* __restrict__ dst, int64_t x0, int64_t y, int64_t n0,
                                          float (*f)[9])
{
    NodeRng<T> rng[VX];
#pragma unroll
    for (int c = 0; c < VX; ++c) rng[c] = NodeRng<T>(p.g, x0 + c, y, f[c]);
    if constexpr (L == L_STREAM) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            T v[VX];
#pragma unroll
            for (int c = 0; c < VX; ++c) v[c] = enc<T>(f[c][i], rng[c].draw(i));
            vstore_t<T, VX>(dst + (int64_t)i * p.g.P + n0, v);
        }
    } else if constexpr (L == L_BUNDLE) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            T v[3 * VX];
#pragma unroll
            for (int c = 0; c < VX; ++c)
#pragma unroll
                for (int k = 0; k < 3; ++k) v[3 * c + k] = enc<T>(f[c][3 * b + k], rng[c].draw(3 * b + k));
            vstore_run_t<T, 3 * VX>(dst + (int64_t)b * 3 * p.g.P + 3 * n0, v);
        }
    } else {
        T v[9 * VX];
#pragma unroll
        for (int c = 0; c < VX; ++c)
#pragma unroll
            for (int i = 0; i < 9; ++i) v[9 * c + i] = enc<T>(f[c][i], rng[c].draw(i));
        vstore_run_t<T, 9 * VX>(dst + 9 * n0, v);
    }
}

// Update of the VX nodes starting at (x0, y), node n0 (x0 < nx, y < ny).
template <int L, class T, int VX>
__device__ __forceinline__ void pull_update_run(const KParams& p, const T* __restrict__ src, T* __restrict__ dst,
                                                int64_t x0, int64_t y, int64_t n0)
{
    if (all_regular<VX>(p.types + n0)) {
        float f[VX][9];
        pull_regular<L, T, VX>(p, src, y, n0, f);
#pragma unroll
        for (int k = 0; k < VX; ++k) collide(f[k], p.ph.omc, p.ph.F);
        store_run<L, T, VX>(p, dst, x0, y, n0, f);
    } else {
#pragma unroll 1
        for (int k = 0; k < VX; ++k) {
            const int64_t x = x0 + k;
            const int64_t n = n0 + k;
            if (x >= p.g.nx || !updated(p.types[n])) continue;
            float f[9];
            gather_pull<L, ST_PULL>(p, src, x, y, n, f);
            collide(f, p.ph.omc, p.ph.F);
            const NodeRng<T> rng(p.g, x, y, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
            for (int i = 0; i < 9; ++i) dst[lat_at<L>(i, n, p.g.P)] = enc<T>(f[i], rng.draw(i));
        }
    }
}

// LPTL: a linear 1-D launch over all nx * ny nodes, block size from the
// runtime's occupancy query; one node per thread.
template <int L, class T>
__global__ void __launch_bounds__(1024) k_lptl(KParams p, const T* __restrict__ src, T* __restrict__ dst)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = p.g.nx * p.g.ny;
    if (m >= total) return;
    int64_t y, x;
    if (total <= 0xffffffffll) {
        const uint32_t q = (uint32_t)m / (uint32_t)p.g.nx;
        y = q;
        x = (uint32_t)m - q * (uint32_t)p.g.nx;
    } else {
        y = m / p.g.nx;
        x = m - y * p.g.nx;
    }
    pull_update_run<L, T, 1>(p, src, dst, x, y, y * p.g.px + x);
}

// NPTL: one tile per block; a thread updates VX consecutive nodes of a row.
template <int L, class T, int VX>
__global__ void __launch_bounds__(256) k_nptl(KParams p, const T* __restrict__ src, T* __restrict__ dst)
{
    const TileCoord c = tile_of_block(p.g);
    const int x0 = c.x0 + (int)threadIdx.x * VX;
    const int y = c.y0 + (int)threadIdx.y;
    if (x0 >= c.x1 || y >= c.y1) return;
    pull_update_run<L, T, VX>(p, src, dst, x0, y, (int64_t)y * p.g.px + x0);
}

// ------------------------------------------------------------------ PUSH
// State: slot i of a node holds its incoming (streamed) value f_in_i, except
// that slots fed by an inlet are never read (the inlet equilibrium is used).
template <int L, class T>
__device__ __forceinline__ void push_general(const KParams& p, const T* __restrict__ src, T* __restrict__ dst,
                                             int x, int y, int64_t n)
{
    int kind[9];
    float f[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int64_t sn;
        kind[i] = pull_source(p.g, p.types, x, y, i, sn);
        const float v = ld(src[lat_at<L>(i, n, p.g.P)]); // unconditional: see gather_pull
        f[i] = kind[i] == K_INLET ? p.ph.ein[i] : v;
    }
    collide(f, p.ph.omc, p.ph.F);
    const NodeRng<T> rng(p.g, x, y, f); // stochastic-rounding bits (FP16S-SR only)
    const bool outlet_col = p.g.xa == AX_INOUT && x == p.g.nx - 1;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        // own slot i when its pull source cannot push: solid -> bounce-back
        if (kind[i] == K_SOLID) dst[lat_at<L>(i, n, p.g.P)] = enc<T>(f[dir_opp(i)], rng.draw(dir_opp(i)));
        // scatter f*_i to (x, y) + c_i
        int64_t tx = x + dir_cx(i), ty = y + dir_cy(i);
        bool ok = true;
        if (ty < 0 || ty >= p.g.ny) {
            if (p.g.ya == AX_PERIODIC) ty = ty < 0 ? ty + p.g.ny : ty - p.g.ny;
            else ok = false;
        }
        if (tx < 0 || tx >= p.g.nx) {
            if (p.g.xa == AX_PERIODIC) tx = tx < 0 ? tx + p.g.nx : tx - p.g.nx;
            else ok = false;
        }
        if (ok) {
            const int64_t tn = ty * p.g.px + tx;
            if (updated(p.types[tn])) dst[lat_at<L>(i, tn, p.g.P)] = enc<T>(f[i], rng.draw(i));
        }
        // zero-gradient outlet: the last column also feeds its own column
        if (dir_cx(i) == -1 && outlet_col) {
            int64_t ty2 = y + dir_cy(i);
            bool ok2 = true;
            if (ty2 < 0 || ty2 >= p.g.ny) {
                if (p.g.ya == AX_PERIODIC) ty2 = ty2 < 0 ? ty2 + p.g.ny : ty2 - p.g.ny;
                else ok2 = false;
            }
            if (ok2) {
                const int64_t tn = ty2 * p.g.px + (p.g.nx - 1);
                if (updated(p.types[tn])) dst[lat_at<L>(i, tn, p.g.P)] = enc<T>(f[i], rng.draw(i));
            }
        }
    }
}

template <int L, class T>
__global__ void __launch_bounds__(256) k_push(KParams p, const T* __restrict__ src, T* __restrict__ dst)
{
    const TileCoord c = tile_of_block(p.g);
    const int x = c.x0 + (int)threadIdx.x;
    const int y = c.y0 + (int)threadIdx.y;
    if (x >= c.x1 || y >= c.y1) return;
    const int64_t n = (int64_t)y * p.g.px + x;
    const uint8_t t = p.types[n];
    if (!(t & IRREGULAR)) {
        // regular node: every neighbour is a plain fluid node in range
        float f[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = ld(src[lat_at<L>(i, n, p.g.P)]);
        collide(f, p.ph.omc, p.ph.F);
        const NodeRng<T> rng(p.g, x, y, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
        for (int i = 0; i < 9; ++i)
            dst[lat_at<L>(i, n + dir_cx(i) + dir_cy(i) * p.g.px, p.g.P)] = enc<T>(f[i], rng.draw(i));
    } else if (updated(t)) {
        push_general<L, T>(p, src, dst, x, y, n);
    }
}

// ------------------------------------------------------------------ NPOL
// Tiles are tile_x (a multiple of 64, so a wavefront is one tile row) by
// tile_y nodes, one node per thread.  For a regular node only a source across
// the tile's edge needs the buffer grid: whether a row crosses is uniform per
// wavefront, whether a column crosses concerns the first and last lane.
__device__ __forceinline__ int64_t edge_adjacent(const Geometry& g, const TileCoord& c, int sx, int sy, int i)
{
    const int dtx = sx < c.x0 ? -1 : (sx >= c.x1 ? 1 : 0);
    const int dty = sy < c.y0 ? -1 : (sy >= c.y1 ? 1 : 0);
    const int tsx = c.bx + dtx, tsy = c.by + dty;
    const int tile = tsy * g.ntx + tsx;
    if (dtx != 0) return edge_x_at(g, tile, dir_cx(i) > 0 ? 1 : 0, sy - tsy * g.ty, dir_cy(i) + 1);
    return edge_y_at(g, tile, dir_cy(i) > 0 ? 1 : 0, sx - tsx * g.tx, dir_cx(i) + 1);
}

template <int I>
__device__ __forceinline__ bool crosses_tile(const TileCoord& c, int x, int y)
{
    constexpr int X = dir_cx(I), Y = dir_cy(I);
    // the source (x, y) - c_I lies outside the tile
    const bool ox = X > 0 ? x == c.x0 : (X < 0 ? x == c.x1 - 1 : false);
    const bool oy = Y > 0 ? y == c.y0 : (Y < 0 ? y == c.y1 - 1 : false);
    return ox || oy;
}

template <int L, class T, int I>
__device__ __forceinline__ float npol_regular_one(const KParams& p, const TileCoord& c, const T* lat,
                                                  const T* __restrict__ edge_in, int x, int y, int64_t n)
{
    constexpr int X = dir_cx(I), Y = dir_cy(I);
    if (crosses_tile<I>(c, x, y)) return ld(edge_in[edge_adjacent(p.g, c, x - X, y - Y, I)]);
    return ld(lat[lat_at<L>(I, n - X - Y * p.g.px, p.g.P)]);
}

template <int L, class T>
__global__ void __launch_bounds__(1024) k_npol(KParams p, T* lat, const T* __restrict__ edge_in, T* __restrict__ edge_out)
{
    const TileCoord c = tile_of_block(p.g);
    const int x = c.x0 + (int)threadIdx.x;
    const int y = c.y0 + (int)threadIdx.y;
    const bool inside = x < c.x1 && y < c.y1;
    const int64_t n = (int64_t)y * p.g.px + x;
    const uint8_t t = inside ? p.types[n] : (uint8_t)T_SOLID;
    const bool active = inside && updated(t);
    float f[9];
    if (active) {
        if (!(t & IRREGULAR)) {
            f[0] = npol_regular_one<L, T, 0>(p, c, lat, edge_in, x, y, n);
            f[1] = npol_regular_one<L, T, 1>(p, c, lat, edge_in, x, y, n);
            f[2] = npol_regular_one<L, T, 2>(p, c, lat, edge_in, x, y, n);
            f[3] = npol_regular_one<L, T, 3>(p, c, lat, edge_in, x, y, n);
            f[4] = ld(lat[lat_at<L>(4, n, p.g.P)]);
            f[5] = npol_regular_one<L, T, 5>(p, c, lat, edge_in, x, y, n);
            f[6] = npol_regular_one<L, T, 6>(p, c, lat, edge_in, x, y, n);
            f[7] = npol_regular_one<L, T, 7>(p, c, lat, edge_in, x, y, n);
            f[8] = npol_regular_one<L, T, 8>(p, c, lat, edge_in, x, y, n);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                int sx = x, sy = y;
                const int k = pull_source_xy(p.g, p.types, x, y, i, sx, sy);
                const bool in_tile = sx >= c.x0 && sx < c.x1 && sy >= c.y0 && sy < c.y1;
                // one load from a valid global address, value chosen afterwards (see gather_pull)
                const T* at = k == K_NODE ? (in_tile ? lat + lat_at<L>(i, (int64_t)sy * p.g.px + sx, p.g.P)
                                                     : edge_in + edge_src(p.g, sx, sy, i, c.bx))
                                          : lat + lat_at<L>(dir_opp(i), n, p.g.P);
                const float v = ld(*at);
                f[i] = k == K_INLET ? p.ph.ein[i] : v;
            }
        }
    }
    // every read of this tile's nodes precedes every in-place write
    __syncthreads();
    if (!active) return;
    collide(f, p.ph.omc, p.ph.F);
    const NodeRng<T> rng(p.g, x, y, f); // stochastic-rounding bits (FP16S-SR only)
    float r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T e = enc<T>(f[i], rng.draw(i));
        lat[lat_at<L>(i, n, p.g.P)] = e;
        r[i] = ld(e); // edges carry the stored (rounded) values, exactly what the lattice holds
    }
    edge_emit(p.g, c, x, y, r, edge_out);
}

// ------------------------------------------------------------------ NSOL
// Tile nodes publish their stored slots in LDS (the in-flight exchange
// buffer); each node then takes its incoming value of direction i from the
// opposite slot of the neighbour it exchanges with.
template <int L, class T>
__global__ void __launch_bounds__(1024) k_nsol(KParams p, T* lat, const T* __restrict__ edge_in, T* __restrict__ edge_out)
{
    extern __shared__ float s[]; // [9][tile_y][tile_x]
    const TileCoord c = tile_of_block(p.g);
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int x = c.x0 + lx;
    const int y = c.y0 + ly;
    const bool inside = x < c.x1 && y < c.y1;
    const int64_t n = (int64_t)y * p.g.px + x;
    const uint8_t t = inside ? p.types[n] : (uint8_t)T_SOLID;
    const bool active = inside && updated(t);
    const int plane = p.g.tx * p.g.ty;
    const int me = ly * p.g.tx + lx;
    float own[9];
    if (active) {
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            own[j] = ld(lat[lat_at<L>(j, n, p.g.P)]); // slot j = f*_{opp(j)}
            s[j * plane + me] = own[j];
        }
    }
    __syncthreads();
    if (!active) return;
    float f[9];
    if (!(t & IRREGULAR)) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int X = dir_cx(i), Y = dir_cy(i);
            const bool ox = X > 0 ? x == c.x0 : (X < 0 ? x == c.x1 - 1 : false);
            const bool oy = Y > 0 ? y == c.y0 : (Y < 0 ? y == c.y1 - 1 : false);
            if (i == 4)
                f[i] = own[4];
            else if (ox || oy)
                f[i] = ld(edge_in[edge_adjacent(p.g, c, x - X, y - Y, i)]);
            else
                f[i] = s[dir_opp(i) * plane + me - X - Y * p.g.tx];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int sx = x, sy = y;
            const int k = pull_source_xy(p.g, p.types, x, y, i, sx, sy);
            const bool in_tile = sx >= c.x0 && sx < c.x1 && sy >= c.y0 && sy < c.y1;
            const bool cross = k == K_NODE && !in_tile;
            // LDS and edge reads at always-valid addresses; the value is
            // chosen afterwards (no pointer select across address spaces)
            const float vl = s[dir_opp(i) * plane + (in_tile ? (sy - c.y0) * p.g.tx + (sx - c.x0) : me)];
            const float ve = ld(edge_in[cross ? edge_src(p.g, sx, sy, i, c.bx) : 0]);
            // K_SOLID: no exchange, slot i still holds f*_{opp(i)}
            f[i] = k == K_SOLID ? own[i] : (k == K_INLET ? p.ph.ein[i] : (cross ? ve : vl));
        }
    }
    collide(f, p.ph.omc, p.ph.F);
    const NodeRng<T> rng(p.g, x, y, f); // stochastic-rounding bits (FP16S-SR only)
    float r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T e = enc<T>(f[i], rng.draw(i));
        lat[lat_at<L>(dir_opp(i), n, p.g.P)] = e; // swap state: f*_i in slot opposite(i)
        r[i] = ld(e);
    }
    edge_emit(p.g, c, x, y, r, edge_out);
}

// ------------------------------------------------------ NSOL, per wavefront
// Wavefront-level swap: one wavefront owns a strip of 64 columns x tile_y
// rows and marches up its rows.  Every node keeps f*_i in slot opposite(i).
// The exchange partners of a node are its own lane in the rows below and
// above (registers), the neighbouring lanes (cross-lane shuffles), and, for
// partners outside the strip, the buffer grid written by the neighbouring
// strips in the previous update.  Nothing else is shared, so no LDS and no
// barrier: each wavefront reads a row's slots before it overwrites them.
__device__ __forceinline__ float lane_up(float v, int lane) { return __shfl(v, lane + 1 < 64 ? lane + 1 : lane, 64); }
__device__ __forceinline__ float lane_down(float v, int lane) { return __shfl(v, lane > 0 ? lane - 1 : lane, 64); }

// Edge-buffer entry of f*_i at the unwrapped source (sxu, syu), which lies
// outside the reader's strip c.
__device__ __forceinline__ int64_t edge_of_source(const Geometry& g, const TileCoord& c, int sxu, int syu, int i)
{
    int sx = sxu, sy = syu;
    if (sx < 0) sx += (int)g.nx;
    else if (sx >= g.nx) sx -= (int)g.nx;
    if (sy < 0) sy += (int)g.ny;
    else if (sy >= g.ny) sy -= (int)g.ny;
    const int tsx = sx / g.tx, tsy = sy / g.ty;
    const int tile = tsy * g.ntx + tsx;
    if (sxu < c.x0 || sxu >= c.x1) return edge_x_at(g, tile, dir_cx(i) > 0 ? 1 : 0, sy - tsy * g.ty, dir_cy(i) + 1);
    return edge_y_at(g, tile, dir_cy(i) > 0 ? 1 : 0, sx - tsx * g.tx, dir_cx(i) + 1);
}

template <int L, class T>
__device__ __forceinline__ void load_slots(const T* lat, int64_t n, int64_t P, float* v)
{
#pragma unroll
    for (int j = 0; j < 9; ++j) v[j] = ld(lat[lat_at<L>(j, n, P)]);
}

template <int L, class T>
__global__ void __launch_bounds__(256) k_nsol_w(KParams p, T* lat, const T* __restrict__ edge_in,
                                                T* __restrict__ edge_out)
{
    const Geometry& g = p.g;
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= g.ntx * g.nty) return; // whole wavefront
    TileCoord c;
    c.by = tile / g.ntx;
    c.bx = tile - c.by * g.ntx;
    c.x0 = c.bx * g.tx;
    c.y0 = c.by * g.ty;
    c.x1 = (int)min((int64_t)(c.x0 + g.tx), g.nx);
    c.y1 = (int)min((int64_t)(c.y0 + g.ty), g.ny);
    const int x = c.x0 + lane;
    const bool lane_in = x < c.x1;
    const int xs = lane_in ? x : c.x1 - 1; // inactive lanes read a valid node, results unused
    const bool left = x == c.x0, right = x == c.x1 - 1;
    const bool clamp_col = g.xa == AX_INOUT && x == g.nx - 1;

    float cur[9], nxt[9], nn[9], prv[3] = {0.f, 0.f, 0.f};
    load_slots<L>(lat, (int64_t)c.y0 * g.px + xs, g.P, cur);
    if (c.y0 + 1 < c.y1) load_slots<L>(lat, (int64_t)(c.y0 + 1) * g.px + xs, g.P, nxt);
#pragma unroll 1
    for (int y = c.y0; y < c.y1; ++y) {
        const bool first = y == c.y0, last = y == c.y1 - 1;
        if (y + 2 < c.y1) load_slots<L>(lat, (int64_t)(y + 2) * g.px + xs, g.P, nn);
        const int64_t n = (int64_t)y * g.px + xs;
        // partners in neighbouring lanes
        const float l_prv0 = lane_down(prv[0], lane), r_prv2 = lane_up(prv[2], lane);
        const float l_cur3 = lane_down(cur[3], lane), r_cur5 = lane_up(cur[5], lane);
        const float l_nxt6 = lane_down(nxt[6], lane), r_nxt8 = lane_up(nxt[8], lane);
        const uint8_t t = p.types[n];
        float f[9];
        // default partners (unwrapped source inside the strip)
        f[0] = r_nxt8;
        f[1] = nxt[7];
        f[2] = l_nxt6;
        f[3] = r_cur5;
        f[4] = cur[4];
        f[5] = l_cur3;
        f[6] = r_prv2;
        f[7] = prv[1];
        f[8] = l_prv0;
        if (!(t & IRREGULAR)) {
            // regular node: only the strip's edges need the buffer grid
            if (left | right | first | last) {
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int X = dir_cx(i), Y = dir_cy(i);
                    const bool out = (X > 0 && left) || (X < 0 && right) || (Y > 0 && first) || (Y < 0 && last);
                    if (out) f[i] = ld(edge_in[edge_of_source(g, c, x - X, y - Y, i)]);
                }
            }
        } else if (lane_in && updated(t)) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                int sx = x, sy = y;
                const int k = pull_source_xy(g, p.types, x, y, i, sx, sy);
                const int X = dir_cx(i), Y = dir_cy(i);
                const bool clamp = clamp_col && X < 0;
                const int sxu = clamp ? x : x - X, syu = y - Y;
                const bool out = sxu < c.x0 || sxu >= c.x1 || syu < c.y0 || syu >= c.y1;
                // in-strip partner: default register, or own lane for the outlet clamp
                float reg = f[i];
                if (clamp) reg = Y < 0 ? nxt[8] : (Y > 0 ? prv[2] : cur[5]);
                const float ve = ld(edge_in[(k == K_NODE && out) ? edge_of_source(g, c, sxu, syu, i) : 0]);
                f[i] = k == K_SOLID ? cur[i] : (k == K_INLET ? p.ph.ein[i] : (out ? ve : reg));
            }
        }
        if (lane_in && updated(t)) {
            collide(f, p.ph.omc, p.ph.F);
            const NodeRng<T> rng(p.g, x, y, f); // stochastic-rounding bits (FP16S-SR only)
            float r[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const T e = enc<T>(f[i], rng.draw(i));
                lat[lat_at<L>(dir_opp(i), n, g.P)] = e; // f*_i in slot opposite(i)
                r[i] = ld(e);
            }
            edge_emit(g, c, x, y, r, edge_out);
        }
        prv[0] = cur[0];
        prv[1] = cur[1];
        prv[2] = cur[2];
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            cur[j] = nxt[j];
            nxt[j] = nn[j];
        }
    }
}

// ------------------------------------------------------------------ dispatch
template <int L, class T>
static hipError_t launch_update_t(int scheme, const KParams& p, int block, const void* src, void* dst,
                                  const void* ein, void* eout, hipStream_t s)
{
    const int64_t tiles = (int64_t)p.g.ntx * p.g.nty;
    const dim3 tb(p.g.tx, p.g.ty);
    switch (scheme) {
    case S_LPTL: {
        const int64_t total = p.g.nx * p.g.ny;
        const int64_t blocks = (total + block - 1) / block;
        hipLaunchKernelGGL((k_lptl<L, T>), dim3((uint32_t)blocks), dim3(block), 0, s, p, (const T*)src, (T*)dst);
        break;
    }
    case S_NPTL: {
        const dim3 blk(p.g.tx / p.g.vx, p.g.ty);
        if (p.g.vx == 2)
            hipLaunchKernelGGL((k_nptl<L, T, 2>), dim3((uint32_t)tiles), blk, 0, s, p, (const T*)src, (T*)dst);
        else
            hipLaunchKernelGGL((k_nptl<L, T, 1>), dim3((uint32_t)tiles), blk, 0, s, p, (const T*)src, (T*)dst);
        break;
    }
    case S_PUSH:
        hipLaunchKernelGGL((k_push<L, T>), dim3((uint32_t)tiles), tb, 0, s, p, (const T*)src, (T*)dst);
        break;
    case S_NPOL:
        hipLaunchKernelGGL((k_npol<L, T>), dim3((uint32_t)tiles), tb, 0, s, p, (T*)dst, (const T*)ein, (T*)eout);
        break;
    case S_NSOL:
        if (p.g.tx == 64) // one wavefront per strip, four strips per block
            hipLaunchKernelGGL((k_nsol_w<L, T>), dim3((uint32_t)((tiles + 3) / 4)), dim3(256), 0, s, p, (T*)dst,
                               (const T*)ein, (T*)eout);
        else
            hipLaunchKernelGGL((k_nsol<L, T>), dim3((uint32_t)tiles), tb, (size_t)9 * p.g.tx * p.g.ty * sizeof(float),
                               s, p, (T*)dst, (const T*)ein, (T*)eout);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_update(int scheme, int layout, int prec, const KParams& p, int block, const void* src, void* dst,
                         const void* ein, void* eout, hipStream_t s)
{
    if (prec == P_FP32) {
        switch (layout) {
        case L_STREAM: return launch_update_t<L_STREAM, float>(scheme, p, block, src, dst, ein, eout, s);
        case L_BUNDLE: return launch_update_t<L_BUNDLE, float>(scheme, p, block, src, dst, ein, eout, s);
        case L_COLLISION: return launch_update_t<L_COLLISION, float>(scheme, p, block, src, dst, ein, eout, s);
        }
    } else if (prec == P_FP16S) {
        switch (layout) {
        case L_STREAM: return launch_update_t<L_STREAM, _Float16>(scheme, p, block, src, dst, ein, eout, s);
        case L_BUNDLE: return launch_update_t<L_BUNDLE, _Float16>(scheme, p, block, src, dst, ein, eout, s);
        case L_COLLISION: return launch_update_t<L_COLLISION, _Float16>(scheme, p, block, src, dst, ein, eout, s);
        }
    } else if (prec == P_FP16SR) {
        switch (layout) {
        case L_STREAM: return launch_update_t<L_STREAM, uint16_t>(scheme, p, block, src, dst, ein, eout, s);
        case L_BUNDLE: return launch_update_t<L_BUNDLE, uint16_t>(scheme, p, block, src, dst, ein, eout, s);
        case L_COLLISION: return launch_update_t<L_COLLISION, uint16_t>(scheme, p, block, src, dst, ein, eout, s);
        }
    }
    return hipErrorInvalidValue;
}

int lptl_block_size(int layout, int prec)
{
    int grid = 0, block = 0;
    hipError_t e = hipErrorInvalidValue;
    if (prec == P_FP32) {
        if (layout == L_STREAM) e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_STREAM, float>, 0, 1024);
        if (layout == L_BUNDLE) e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_BUNDLE, float>, 0, 1024);
        if (layout == L_COLLISION)
            e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_COLLISION, float>, 0, 1024);
    } else if (prec == P_FP16SR) {
        if (layout == L_STREAM) e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_STREAM, uint16_t>, 0, 1024);
        if (layout == L_BUNDLE) e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_BUNDLE, uint16_t>, 0, 1024);
        if (layout == L_COLLISION)
            e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_COLLISION, uint16_t>, 0, 1024);
    } else {
        if (layout == L_STREAM)
            e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_STREAM, _Float16>, 0, 1024);
        if (layout == L_BUNDLE)
            e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_BUNDLE, _Float16>, 0, 1024);
        if (layout == L_COLLISION)
            e = hipOccupancyMaxPotentialBlockSize(&grid, &block, k_lptl<L_COLLISION, _Float16>, 0, 1024);
    }
    if (e != hipSuccess || block <= 0) return 256;
    return block;
}

} // namespace lbm
