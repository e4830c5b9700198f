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
//   AA    in-place AA streaming, ONE lattice and no buffer grid: even updates
//         are local, odd updates exchange pairwise with the neighbours (the
//         state-of-the-art scheme Section 3.3 cites).
//
// All schemes call the same collide(), so they agree bit for bit.
#include "lbm_device.hpp"
#include "lbm_edges.hpp"
#include "lbm_kernels.hpp"
#include "lbm_stage.hpp"

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
    for (int c = 0; c < VX; ++c) rng[c] = NodeRng<T>((uint32_t)(n0 + c), f[c]);
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
// MODE 1: the Neumann inlet is on (p.rin and p.rout set).  MODE 2: full-way
// bounce-back -- solid nodes are updated too, reversing what streamed into
// them instead of colliding, and fluid nodes pull from them like from any
// node.  MODE 0: neither; the kernels are instantiated per mode because the
// extra code of the other two measurably slows even the regular path.
template <int L, class T, int VX, int MODE>
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
            const uint8_t t = p.types[n];
            const bool reflect = MODE == 2 && node_type(t) == T_SOLID;
            if (x >= p.g.nx || !(updated(t) || reflect)) continue;
            float g9[9];
            const uint32_t lk = p.links[n];
            if (lk & LINK_GENERAL)
                gather_pull<L, ST_PULL, T, MODE == 1, MODE == 2 ? 1 : 0>(p, src, x, y, n, g9);
            else
                gather_linked<L, ST_PULL, T, MODE == 1>(p, src, x, y, n, lk, g9);
            if constexpr (MODE == 1) record_inlet_density(p, x, y, g9);
            if (reflect) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = g9[i];
                    g9[i] = g9[dir_opp(i)];
                    g9[dir_opp(i)] = v;
                }
            } else {
                collide(g9, p.ph.omc, p.ph.F);
            }
            const NodeRng<T> rng((uint32_t)n, g9); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
            for (int i = 0; i < 9; ++i) dst[lat_at<L>(i, n, p.g.P)] = enc<T>(g9[i], rng.draw(i));
        }
    }
}

// LPTL: a linear 1-D launch over all nx * ny nodes, block size from the
// runtime's occupancy query; one node per thread.
template <int L, class T, int MODE>
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
    pull_update_run<L, T, 1, MODE>(p, src, dst, x, y, y * p.g.px + x);
}

// NPTL: one tile per block; a thread updates VX consecutive nodes of a row.
template <int L, class T, int VX, int MODE>
__global__ void __launch_bounds__(256) k_nptl(KParams p, const T* __restrict__ src, T* __restrict__ dst)
{
    const TileCoord c = tile_of_block(p.g);
    const int x0 = c.x0 + (int)threadIdx.x * VX;
    const int y = c.y0 + (int)threadIdx.y;
    if (x0 >= c.x1 || y >= c.y1) return;
    pull_update_run<L, T, VX, MODE>(p, src, dst, x0, y, (int64_t)y * p.g.px + x0);
}

// ------------------------------------------- NPTL, collision layout, staged
// The collision (AoS) layout keeps the 9 values of a node together, so the
// per-direction loads of k_nptl touch, for 64 neighbouring nodes, 18 (FP32)
// cache lines for 256 useful bytes each, nine times over.  Here a block
// covering a 64 x ty tile moves whole records instead: it copies the records
// of the source rows y0 - 1 .. y1, nodes x0 - 1 .. x0 + 64, into LDS with
// 16-byte loads; every regular node takes its 9 incoming values from there;
// the encoded results go back through LDS and leave as whole records of the
// tile's rows, 16 bytes per store.  Nodes that are not updated get 0, which
// is what every lattice holds there (creation, initial state and state loads
// never write them).  Irregular nodes gather from global memory as in k_nptl.
template <class T> struct AosRows {
    static constexpr int CH = 16 / (int)sizeof(T);       // elements per 16-byte piece
    static constexpr int BACK = (9 + CH - 1) / CH * CH;  // a region row starts BACK elements before node x0
    static constexpr int LEAD = BACK - 9;                // elements before the record of node x0 - 1
    static constexpr int ROW = (LEAD + 66 * 9 + CH - 1) / CH * CH; // elements per staged source row
    static constexpr int OUT = 64 * 9;                   // elements per staged result row
    static constexpr int NCH = ROW / CH;
    static constexpr int OCH = OUT / CH;
};

// the source rows, then one 16-byte slot (element (ty + 2) ROW) that takes
// the pieces a staging copy drops
template <class T> __host__ __device__ constexpr size_t aos_stage_bytes(int ty)
{
    return (size_t)(ty + 2) * AosRows<T>::ROW * sizeof(T) + 16;
}

template <class T, int MODE>
__global__ void __launch_bounds__(512) k_nptl_aos(KParams p, const T* __restrict__ src, T* __restrict__ dst)
{
    using R = AosRows<T>;
    extern __shared__ __align__(16) unsigned char smem_aos[];
    T* s = reinterpret_cast<T*>(smem_aos);
    const TileCoord c = tile_of_block(p.g);
    const int lx = threadIdx.x, ly = threadIdx.y;
    const int tid = ly * 64 + lx, nthr = 64 * (int)blockDim.y;
    const int64_t px = p.g.px;
    // region row r holds grid row y0 - 1 + r; only rows inside the grid and
    // at most one past the tile are ever read
    const int r_lo = c.y0 == 0 ? 1 : 0;
    const int r_hi = min(c.y1 - c.y0 + 1, (int)p.g.ny - c.y0); // inclusive
    const int64_t lim = 9 * px * p.g.ny + lattice_guard(p.g);  // end of the allocation (guard included)
    pieces_to_lds<4>(src, s, (r_hi - r_lo + 1) * R::NCH, ((int)blockDim.y + 2) * R::ROW, tid, nthr,
                     [&](int k, int64_t& e, int& o) {
        const int r = r_lo + k / R::NCH, q = k - (k / R::NCH) * R::NCH;
        e = 9 * ((int64_t)(c.y0 - 1 + r) * px + c.x0) - R::BACK + (int64_t)q * R::CH;
        o = r * R::ROW + q * R::CH;
        return e + R::CH <= lim;
    });
    __syncthreads();
    const int x = c.x0 + lx, y = c.y0 + ly;
    const bool inside = x < c.x1 && y < c.y1;
    const int64_t n = (int64_t)y * px + x;
    const uint8_t t = inside ? p.types[n] : (uint8_t)T_SOLID;
    T e9[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) e9[i] = T{};
    if (inside && updated(t)) {
        float f[9];
        if (!(t & IRREGULAR)) {
            // source (x - c_x, y - c_y): region row ly + 1 - c_y, record lx + 1 - c_x
            const T* b = s + (ly + 1) * R::ROW + R::LEAD + 9 * (lx + 1);
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = ld(b[-dir_cy(i) * R::ROW - 9 * dir_cx(i) + i]);
        } else {
            const uint32_t lk = p.links[n];
            if (lk & LINK_GENERAL)
                gather_pull<L_COLLISION, ST_PULL, T, MODE == 1, 0>(p, src, x, y, n, f);
            else
                gather_linked<L_COLLISION, ST_PULL, T, MODE == 1>(p, src, x, y, n, lk, f);
            if constexpr (MODE == 1) record_inlet_density(p, x, y, f);
        }
        collide(f, p.ph.omc, p.ph.F);
        const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
        for (int i = 0; i < 9; ++i) e9[i] = enc<T>(f[i], rng.draw(i));
    }
    __syncthreads(); // every read of the staged source rows is done
    T* o = s + ly * R::OUT + 9 * lx;
#pragma unroll
    for (int i = 0; i < 9; ++i) o[i] = e9[i];
    __syncthreads();
    // whole records of nodes x0 .. min(x0 + 64, px) - 1 of every tile row
    const int wch = 9 * (min(c.x0 + 64, (int)px) - c.x0) / R::CH;
    pieces_from_lds<4>(dst, s, (c.y1 - c.y0) * R::OCH, tid, nthr, [&](int k, int64_t& e, int& o) {
        const int r = k / R::OCH, q = k - (k / R::OCH) * R::OCH;
        e = 9 * ((int64_t)(c.y0 + r) * px + c.x0) + (int64_t)q * R::CH;
        o = r * R::OUT + q * R::CH;
        return q < wch;
    });
}

// ------------------------------------------------------------------ PUSH
// State: slot i of a node holds its incoming (streamed) value f_in_i, except
// that slots fed by an inlet are never read (the inlet equilibrium is used).
//
// Stores of the post-collision values f*_i of node (x, y) in that state: to
// every slot that pulls them in the next update under the rules of the pull
// definition -- slot i of (x, y) + c_i (wrapped on periodic axes, dropped past
// a closed side or the outlet, never into an inlet or solid node), the node's
// own slot i for a direction whose pull source is solid (bounce-back), and,
// in the outlet column, slot i of the outlet node in row y + c_y for c_x = -1
// (the push form of the zero-gradient outlet).
template <int L, class T>
__device__ __forceinline__ void push_store(const KParams& p, T* __restrict__ dst, int x, int y, int64_t n,
                                           const float* f, const int* kind, const NodeRng<T>& rng)
{
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
__device__ __forceinline__ void push_general(const KParams& p, const T* __restrict__ src, T* __restrict__ dst,
                                             int x, int y, int64_t n)
{
    int kind[9];
    float f[9];
    const uint32_t lk = p.links[n];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int64_t sn;
        int sx, sy;
        kind[i] = (lk & LINK_GENERAL) ? pull_source(p.g, p.types, x, y, i, sn) : linked_source(lk, i, x, y, sx, sy);
        const float v = ld(src[lat_at<L>(i, n, p.g.P)]); // unconditional: see gather_pull
        f[i] = kind[i] == K_INLET ? inlet_value(p, i) : v;
    }
    boundary_fix(p, x, y, f);
    record_inlet_density(p, x, y, f);
    collide(f, p.ph.omc, p.ph.F);
    const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
    push_store<L, T>(p, dst, x, y, n, f, kind, rng);
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
        const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
        for (int i = 0; i < 9; ++i)
            dst[lat_at<L>(i, n + dir_cx(i) + dir_cy(i) * p.g.px, p.g.P)] = enc<T>(f[i], rng.draw(i));
    } else if (updated(t)) {
        push_general<L, T>(p, src, dst, x, y, n);
    }
}

// PUSH with staged stores (64-wide tiles): the block's regular nodes put
// their post-collision values into the LDS image of the tile's region at
// their push targets (slot i of node + c_i) and mark them; the marked
// elements leave in whole 16-byte pieces wherever a piece is complete (all of
// a target row between the tile's side columns), element by element at the
// sides.  In the bundle and collision layouts the nodes' own incoming values
// are staged as whole records first; the stream layout reads them directly
// (one contiguous run per direction already).  Irregular nodes keep the
// direct rules (push_general); their targets are never marked, and each
// target element has one writer, so the direct and the staged stores never
// meet.
template <int L, class T>
__global__ void __launch_bounds__(512) k_push_staged(KParams p, const T* __restrict__ src, T* __restrict__ dst)
{
    using S = Stage<L, T>;
    extern __shared__ __align__(16) unsigned char smem_push[];
    T* s = reinterpret_cast<T*>(smem_push);
    const int ty = (int)blockDim.y;
    uint8_t* mask = smem_push + S::bytes(ty);
    const TileCoord c = tile_of_block(p.g);
    const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * 64 + lx, nthr = 64 * ty;
    const int rows = c.y1 - c.y0;
    for (int k = tid; k < (ty + 2) * S::RROW / 4; k += nthr) reinterpret_cast<uint32_t*>(mask)[k] = 0u;
    if constexpr (L != L_STREAM) stage_load<L, T>(p.g, src, s, c.x0, c.y0, 1, rows, tid, nthr);
    __syncthreads();
    const int x = c.x0 + lx, y = c.y0 + ly;
    const bool inside = x < c.x1 && y < c.y1;
    const int64_t n = (int64_t)y * p.g.px + x;
    const uint8_t t = inside ? p.types[n] : (uint8_t)T_SOLID;
    float f[9];
    const bool regular = inside && !(t & IRREGULAR); // implies a plain fluid node
    if (regular) {
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            if constexpr (L == L_STREAM)
                f[i] = ld(src[(int64_t)i * p.g.P + n]);
            else
                f[i] = ld(s[S::at(ly + 1, lx + 1, i)]);
        }
        collide(f, p.ph.omc, p.ph.F);
    } else if (inside && updated(t)) {
        push_general<L, T>(p, src, dst, x, y, n);
    }
    __syncthreads(); // the staged own values are read: the image takes the results
    if (regular) {
        const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int o = S::at(ly + 1 + dir_cy(i), lx + 1 + dir_cx(i), i);
            s[o] = enc<T>(f[i], rng.draw(i));
            mask[o] = 1;
        }
    }
    __syncthreads();
    stage_store_masked<L, T>(p.g, dst, s, mask, c.x0, c.y0, 0, rows + 1, tid, nthr);
}

// ------------------------------------------------------------------ AA
// In-place AA streaming (Bailey et al.; the state-of-the-art one-lattice
// scheme Section 3.3 cites, and the first further direction of Section 6).
// One lattice, two kinds of update that alternate:
//  * even update: a node reads its incoming values from its own slots (the
//    push state: slot i holds f_in_i, inlet-fed slots take the inlet
//    equilibrium), collides and writes f*_i into its own slot opposite(i)
//    (the swap state).  Purely local.
//  * odd update: a node reads f*_i of its pull source from the source's slot
//    opposite(i) (its own slot i for bounce-back), collides, and stores the
//    results in the push state with the push rules.  The slots a node reads
//    are exactly the slots it writes: slot opposite(i) of (x, y) - c_i is
//    where its f*_opposite(i) goes.  No two nodes touch one location, so no
//    barrier and no buffer grid.
// The exception is the zero-gradient outlet: an outlet node's clamped source
// lies in another node's exchange set.  Even updates therefore also copy the
// outlet column's c_x = -1 values (directions 0, 3, 6) into a side buffer of
// 3 values per row, which odd updates read instead.
template <int L, class T>
__global__ void __launch_bounds__(256) k_aa_even(KParams p, T* lat, T* __restrict__ obuf)
{
    const TileCoord c = tile_of_block(p.g);
    const int x = c.x0 + (int)threadIdx.x;
    const int y = c.y0 + (int)threadIdx.y;
    if (x >= c.x1 || y >= c.y1) return;
    const int64_t n = (int64_t)y * p.g.px + x;
    const uint8_t t = p.types[n];
    if (!updated(t)) return;
    float f[9];
    if (!(t & IRREGULAR)) {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = ld(lat[lat_at<L>(i, n, p.g.P)]);
    } else {
        const uint32_t lk = p.links[n];
        if (lk & LINK_GENERAL)
            gather_push<L>(p, lat, x, y, n, f);
        else
            gather_push_linked<L>(p, lat, x, y, n, lk, f);
        record_inlet_density(p, x, y, f);
    }
    collide(f, p.ph.omc, p.ph.F);
    const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
    const bool outlet_col = p.g.xa == AX_INOUT && x == p.g.nx - 1;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T e = enc<T>(f[i], rng.draw(i));
        lat[lat_at<L>(dir_opp(i), n, p.g.P)] = e;
        if (dir_cx(i) == -1 && outlet_col) obuf[3 * (int64_t)y + i / 3] = e;
    }
}

template <int L, class T>
__global__ void __launch_bounds__(256) k_aa_odd(KParams p, T* lat, const T* __restrict__ obuf)
{
    const TileCoord c = tile_of_block(p.g);
    const int x = c.x0 + (int)threadIdx.x;
    const int y = c.y0 + (int)threadIdx.y;
    if (x >= c.x1 || y >= c.y1) return;
    const int64_t n = (int64_t)y * p.g.px + x;
    const uint8_t t = p.types[n];
    if (!updated(t)) return;
    float f[9];
    if (!(t & IRREGULAR)) {
        // regular node: plain neighbours in range
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = ld(lat[lat_at<L>(dir_opp(i), n - dir_cx(i) - dir_cy(i) * p.g.px, p.g.P)]);
        collide(f, p.ph.omc, p.ph.F);
        const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
        for (int i = 0; i < 9; ++i)
            lat[lat_at<L>(i, n + dir_cx(i) + dir_cy(i) * p.g.px, p.g.P)] = enc<T>(f[i], rng.draw(i));
    } else {
        int kind[9];
        const bool outlet_col = p.g.xa == AX_INOUT && x == p.g.nx - 1;
        const uint32_t lk = p.links[n];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int sx = x, sy = y;
            kind[i] = (lk & LINK_GENERAL) ? pull_source_xy(p.g, p.types, x, y, i, sx, sy)
                                          : linked_source(lk, i, x, y, sx, sy);
            // a clamped outlet source comes from the side buffer; one load
            // from a valid address, the value chosen afterwards
            const bool clamped = kind[i] == K_NODE && outlet_col && dir_cx(i) == -1;
            const T* at = clamped ? obuf + (3 * (int64_t)sy + i / 3)
                                  : lat + (kind[i] == K_NODE ? lat_at<L>(dir_opp(i), (int64_t)sy * p.g.px + sx, p.g.P)
                                                             : lat_at<L>(i, n, p.g.P));
            const float v = ld(*at);
            f[i] = kind[i] == K_INLET ? inlet_value(p, i) : v;
        }
        boundary_fix(p, x, y, f);
        record_inlet_density(p, x, y, f);
        collide(f, p.ph.omc, p.ph.F);
        const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
        push_store<L, T>(p, lat, x, y, n, f, kind, rng);
    }
}

// AA in the collision layout with whole records staged through LDS (64-wide
// tiles).  Even update: the tile rows' records are staged, every node reads
// its own values there and puts its results back into its own record; the
// records leave as whole 16-byte pieces (nodes that are not updated rewrite
// the values they were staged with).  Odd update: the region of the tile plus
// its one-node ring is staged; regular nodes read their sources' opposite
// slots there and put their results at their push targets, marked; only the
// marked elements are written back, since the rest of the ring belongs to the
// exchange sets of other tiles.  Irregular nodes of an odd update read and
// store directly with the boundary rules (their exchange sets are theirs
// alone).
template <class T>
__global__ void __launch_bounds__(512) k_aa_even_aos(KParams p, T* lat, T* __restrict__ obuf)
{
    using S = Stage<L_COLLISION, T>;
    extern __shared__ __align__(16) unsigned char smem_aae[];
    T* s = reinterpret_cast<T*>(smem_aae);
    const int ty = (int)blockDim.y;
    uint8_t* mask = smem_aae + S::bytes(ty);
    const TileCoord c = tile_of_block(p.g);
    const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * 64 + lx, nthr = 64 * ty;
    const int rows = c.y1 - c.y0;
    for (int k = tid; k < (ty + 2) * S::RROW / 4; k += nthr) reinterpret_cast<uint32_t*>(mask)[k] = 0u;
    stage_load<L_COLLISION, T>(p.g, lat, s, c.x0, c.y0, 1, rows, tid, nthr);
    __syncthreads();
    const int x = c.x0 + lx, y = c.y0 + ly;
    const bool inside = x < c.x1 && y < c.y1;
    const int64_t n = (int64_t)y * p.g.px + x;
    const uint8_t t = inside ? p.types[n] : (uint8_t)T_SOLID;
    const bool active = inside && updated(t);
    float f[9];
    if (active) {
        if (!(t & IRREGULAR)) {
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = ld(s[S::at(ly + 1, lx + 1, i)]);
        } else {
            const uint32_t lk = p.links[n];
            if (lk & LINK_GENERAL)
                gather_push<L_COLLISION>(p, lat, x, y, n, f);
            else
                gather_push_linked<L_COLLISION>(p, lat, x, y, n, lk, f);
            record_inlet_density(p, x, y, f);
        }
        collide(f, p.ph.omc, p.ph.F);
    }
    __syncthreads(); // every staged value is read
    if (active) {
        const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
        const bool outlet_col = p.g.xa == AX_INOUT && x == p.g.nx - 1;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const T e = enc<T>(f[i], rng.draw(i));
            s[S::at(ly + 1, lx + 1, dir_opp(i))] = e;
            if (dir_cx(i) == -1 && outlet_col) obuf[3 * (int64_t)y + i / 3] = e;
        }
    }
    // every record of the tile's rows up to the row pitch leaves whole
    if (ly < rows && x < p.g.px) {
#pragma unroll
        for (int i = 0; i < 9; ++i) mask[S::at(ly + 1, lx + 1, i)] = 1;
    }
    __syncthreads();
    stage_store_masked<L_COLLISION, T>(p.g, lat, s, mask, c.x0, c.y0, 1, rows, tid, nthr);
}

template <class T>
__global__ void __launch_bounds__(512) k_aa_odd_aos(KParams p, T* lat, const T* __restrict__ obuf)
{
    using S = Stage<L_COLLISION, T>;
    extern __shared__ __align__(16) unsigned char smem_aao[];
    T* s = reinterpret_cast<T*>(smem_aao);
    const int ty = (int)blockDim.y;
    uint8_t* mask = smem_aao + S::bytes(ty);
    const TileCoord c = tile_of_block(p.g);
    const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * 64 + lx, nthr = 64 * ty;
    const int rows = c.y1 - c.y0;
    for (int k = tid; k < (ty + 2) * S::RROW / 4; k += nthr) reinterpret_cast<uint32_t*>(mask)[k] = 0u;
    const int r_lo = c.y0 == 0 ? 1 : 0;
    const int r_hi = min(rows + 1, (int)p.g.ny - c.y0);
    stage_load<L_COLLISION, T>(p.g, lat, s, c.x0, c.y0, r_lo, r_hi, tid, nthr);
    __syncthreads();
    const int x = c.x0 + lx, y = c.y0 + ly;
    const bool inside = x < c.x1 && y < c.y1;
    const int64_t n = (int64_t)y * p.g.px + x;
    const uint8_t t = inside ? p.types[n] : (uint8_t)T_SOLID;
    const bool regular = inside && !(t & IRREGULAR);
    float f[9];
    if (regular) {
        // f*_i of the source (x, y) - c_i sits in its slot opposite(i)
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = ld(s[S::at(ly + 1 - dir_cy(i), lx + 1 - dir_cx(i), dir_opp(i))]);
        collide(f, p.ph.omc, p.ph.F);
    } else if (inside && updated(t)) {
        int kind[9];
        const bool outlet_col = p.g.xa == AX_INOUT && x == p.g.nx - 1;
        const uint32_t lk = p.links[n];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int sx = x, sy = y;
            kind[i] = (lk & LINK_GENERAL) ? pull_source_xy(p.g, p.types, x, y, i, sx, sy)
                                          : linked_source(lk, i, x, y, sx, sy);
            const bool clamped = kind[i] == K_NODE && outlet_col && dir_cx(i) == -1;
            const T* at = clamped ? obuf + (3 * (int64_t)sy + i / 3)
                                  : lat + (kind[i] == K_NODE
                                               ? lat_at<L_COLLISION>(dir_opp(i), (int64_t)sy * p.g.px + sx, p.g.P)
                                               : lat_at<L_COLLISION>(i, n, p.g.P));
            const float v = ld(*at);
            f[i] = kind[i] == K_INLET ? inlet_value(p, i) : v;
        }
        boundary_fix(p, x, y, f);
        record_inlet_density(p, x, y, f);
        collide(f, p.ph.omc, p.ph.F);
        const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
        push_store<L_COLLISION, T>(p, lat, x, y, n, f, kind, rng);
    }
    __syncthreads(); // every staged value is read
    if (regular) {
        const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int o = S::at(ly + 1 + dir_cy(i), lx + 1 + dir_cx(i), i);
            s[o] = enc<T>(f[i], rng.draw(i));
            mask[o] = 1;
        }
    }
    __syncthreads();
    stage_store_masked<L_COLLISION, T>(p.g, lat, s, mask, c.x0, c.y0, 0, rows + 1, tid, nthr);
}

// ------------------------------------------------------------------ NPOL
// Tiles of tile_x by tile_y nodes, one node per thread, any shape up to 1024
// threads (one-wavefront-wide tiles on lattices below 2 GiB take the lean
// kernel further down).  A regular node reads its plain neighbour, or the
// buffer grid when that neighbour lies across a side of the tile.
template <int L, class T, int I>
__device__ __forceinline__ float npol_regular_one(const KParams& p, const TileCoord& c, const T* lat,
                                                  const T* __restrict__ edge_in, int x, int y, int64_t n)
{
    constexpr int X = dir_cx(I), Y = dir_cy(I);
    const T* a = lat + lat_at<L>(I, n - X - Y * p.g.px, p.g.P);
    if (crosses_row<I>(c, y) || crosses_col<I>(c, x)) a = edge_in + edge_neighbour<I>(p.g, c, x, y);
    return ld(*a);
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
            const uint32_t lk = p.links[n];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                int sx = x, sy = y;
                const int k = (lk & LINK_GENERAL) ? pull_source_xy(p.g, p.types, x, y, i, sx, sy)
                                                  : linked_source(lk, i, x, y, sx, sy);
                const bool in_tile = sx >= c.x0 && sx < c.x1 && sy >= c.y0 && sy < c.y1;
                // one load from a valid global address, value chosen afterwards (see gather_pull)
                const T* at = k == K_NODE ? (in_tile ? lat + lat_at<L>(i, (int64_t)sy * p.g.px + sx, p.g.P)
                                                     : edge_in + edge_src(p.g, c, sx, sy, i))
                                          : lat + lat_at<L>(dir_opp(i), n, p.g.P);
                const float v = ld(*at);
                f[i] = k == K_INLET ? p.ph.ein[i] : v;
            }
            boundary_fix(p, x, y, f);
            record_inlet_density(p, x, y, f);
        }
    }
    // every read of this tile's nodes precedes every in-place write
    __syncthreads();
    if (!active) return;
    collide(f, p.ph.omc, p.ph.F);
    const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
    float r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T e = enc<T>(f[i], rng.draw(i));
        lat[lat_at<L>(i, n, p.g.P)] = e;
        r[i] = ld(e); // edges carry the stored (rounded) values, exactly what the lattice holds
    }
    edge_emit(p.g, c, x, y, r, edge_out);
}

// NPOL for tiles one wavefront wide (tile_x = 64) on lattices whose byte
// offsets fit 31 bits.  The tile row of a wavefront is uniform, so the bottom
// and top sides are scalar branches; the left and right sides are lanes 0 and
// 63, served by one two-lane block.  Every access is a kernel-argument base
// plus a 32-bit byte offset: a per-direction uniform part and the node's one
// per-lane part.
template <int L, class T>
__device__ __forceinline__ uint32_t pull_off(int i, const Geometry& g, uint32_t vo)
{
    const int X = dir_cx(i), Y = dir_cy(i), S = lat_stride<L>();
    const int64_t e = lat_plane<L>(i, g.P) - (int64_t)S * Y * g.px + (lat_lane<L>(i) - S * X);
    return (uint32_t)e * (uint32_t)sizeof(T) + vo;
}

// Byte offset of the node's own slot of direction i (same base as pull_off).
template <int L, class T>
__device__ __forceinline__ uint32_t own_off(int i, const Geometry& g, uint32_t vo)
{
    return (uint32_t)(lat_plane<L>(i, g.P) + lat_lane<L>(i)) * (uint32_t)sizeof(T) + vo;
}

// What a thread of the lean NPOL kernel keeps for one of its nodes between
// the read phase and the in-place write phase.  Scalars only: populations
// travel in plain arrays of their own, which stay in registers (an array
// inside a struct indexed in a loop is moved to LDS or scratch).
struct Npol64Node {
    uint32_t n;
    int y;
    uint8_t t;
    bool inside, active, bottom, top;
};

// Issue step of one node (x = c.x0 + lane, row y; the row is uniform per
// wavefront): every load is issued together with the node-type load, before
// the node is known to be regular -- plain neighbours (in bounds thanks to the
// lattice guards) and the edge entries a regular node on a side would use
// (tile indices clamped into the grid, so those addresses are valid too).
// The raw stored values are kept undecoded: nothing consumes a load here, so
// the loads of all of a thread's nodes are in flight together.
template <int L, class T>
__device__ __forceinline__ void npol64_issue(const KParams& p, const TileCoord& c, const T* lat,
                                             const T* __restrict__ edge_in, int lane, int y, Npol64Node& q,
                                             T (&fr)[9], T (&er)[9])
{
    const Geometry& g = p.g;
    constexpr uint32_t E = sizeof(T);
    const int x = c.x0 + lane;
    q.y = y;
    q.bottom = y == c.y0; // uniform per wavefront
    q.top = y == c.y1 - 1;
    q.inside = x < c.x1 && y < c.y1;
    q.n = (uint32_t)y * (uint32_t)g.px + (uint32_t)x;
    q.t = T_SOLID;
    // offsets count from the start of the lower guard, so every one is
    // non-negative; the guards keep each plain neighbour of an in-domain
    // node inside the allocation
    const int64_t G = lattice_guard(g);
    const T* latg = lat - G;
    const uint32_t vo = ((uint32_t)G + q.n * (uint32_t)lat_stride<L>()) * E; // node byte offset
    const uint32_t xo = (uint32_t)x * E;                                     // column byte offset (Y edges)
    const uint32_t R = (uint32_t)g.nty * (uint32_t)g.ty;  // X edges: rows per [side][k] run
    const uint32_t C = (uint32_t)g.ntx * 64u;             // Y edges: columns per [side][k] run
    const uint32_t YE = (uint32_t)g.ntx * 6u * R;        // start of the Y edges
#pragma unroll
    for (int k = 0; k < 9; ++k) er[k] = T{};
    if (!q.inside) return;
    q.t = p.types[q.n];
    // rows across the bottom/top side come from the Y edges only.  Plane
    // layouts point those loads at the node's own slot of that direction
    // instead (a line the tile reads anyway, coalesced), which keeps the issue
    // step free of branches; in the collision layout every slot is a request
    // of its own, so there they are skipped
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const bool across = (i < 3 && q.top) || (i >= 6 && q.bottom);
        if constexpr (L == L_COLLISION) {
            if (!across) fr[i] = at_byte(latg, pull_off<L, T>(i, g, vo));
        } else {
            fr[i] = at_byte(latg, across ? own_off<L, T>(i, g, vo) : pull_off<L, T>(i, g, vo));
        }
    }
    if (q.top) { // c_y = -1: row y + 1 is the bottom row of the tile row above
        const uint32_t o = (YE + (uint32_t)min(c.by + 1, g.nty - 1) * 6u * C) * E + xo;
        er[0] = at_byte(edge_in, o + E);
        er[1] = at_byte(edge_in, o + C * E);
        er[2] = at_byte(edge_in, o + 2 * C * E - E);
    }
    if (q.bottom) { // c_y = +1: row y - 1 is the top row of the tile row below
        const uint32_t o = (YE + ((uint32_t)max(c.by - 1, 0) * 6u + 3u) * C) * E + xo;
        er[3] = at_byte(edge_in, o + E);
        er[4] = at_byte(edge_in, o + C * E);
        er[5] = at_byte(edge_in, o + 2 * C * E - E);
    }
    if (lane == 0 || lane == 63) { // right side of column bx - 1 / left side of column bx + 1
        const bool left = lane == 0;
        const int col = left ? max(c.bx - 1, 0) : min(c.bx + 1, g.ntx - 1);
        const uint32_t o = (((uint32_t)col * 6u + (left ? 3u : 0u)) * R + (uint32_t)y) * E;
        er[6] = at_byte(edge_in, o + E);             // k = 0: row y + 1
        er[7] = at_byte(edge_in, o + R * E);         // k = 1: row y
        er[8] = at_byte(edge_in, o + 2 * R * E - E); // k = 2: row y - 1
    }
}

// Resolve step: a regular node takes its sources across the tile sides from
// the edge entries (bottom/top rows the Y edges, corners included; lanes 0
// and 63 the X edges -- a regular node on the right side implies an unclipped
// tile, so it is lane 63); an irregular node gathers through its link word
// and applies its boundary rules.
template <int L, class T>
__device__ __forceinline__ void npol64_resolve(const KParams& p, const TileCoord& c, const T* lat,
                                               const T* __restrict__ edge_in, int lane, Npol64Node& q,
                                               const T (&fr)[9], const T (&er)[9], float (&f)[9])
{
    const Geometry& g = p.g;
    q.active = q.inside && updated(q.t);
    if (!q.active) return;
    const int x = c.x0 + lane, y = q.y;
    if (!(q.t & IRREGULAR)) {
        const bool top = q.top, bottom = q.bottom, left = lane == 0, right = lane == 63;
        f[0] = ld(top ? er[0] : right ? er[6] : fr[0]);
        f[1] = ld(top ? er[1] : fr[1]);
        f[2] = ld(top ? er[2] : left ? er[6] : fr[2]);
        f[3] = ld(right ? er[7] : fr[3]);
        f[4] = ld(fr[4]);
        f[5] = ld(left ? er[7] : fr[5]);
        f[6] = ld(bottom ? er[3] : right ? er[8] : fr[6]);
        f[7] = ld(bottom ? er[4] : fr[7]);
        f[8] = ld(bottom ? er[5] : left ? er[8] : fr[8]);
    } else {
        const uint32_t n = q.n;
        const uint32_t lk = p.links[n];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int sx = x, sy = y;
            const int k = (lk & LINK_GENERAL) ? pull_source_xy(g, p.types, x, y, i, sx, sy)
                                              : linked_source(lk, i, x, y, sx, sy);
            const bool in_tile = sx >= c.x0 && sx < c.x1 && sy >= c.y0 && sy < c.y1;
            const T* at = k == K_NODE ? (in_tile ? lat + lat_at<L>(i, (int64_t)sy * g.px + sx, g.P)
                                                 : edge_in + edge_src(g, c, sx, sy, i))
                                      : lat + lat_at<L>(dir_opp(i), n, g.P);
            const float v = ld(*at);
            f[i] = k == K_INLET ? p.ph.ein[i] : v;
        }
        boundary_fix(p, x, y, f);
        record_inlet_density(p, x, y, f);
    }
}

// Write phase of one node: collide, store in place, publish the values that
// leave the tile (the entries edge_emit writes).
template <int L, class T>
__device__ __forceinline__ void npol64_write(const KParams& p, const TileCoord& c, T* lat, T* __restrict__ edge_out,
                                             int lane, const Npol64Node& q, float (&f)[9])
{
    if (!q.active) return;
    const Geometry& g = p.g;
    constexpr uint32_t E = sizeof(T);
    const int x = c.x0 + lane, y = q.y;
    const uint32_t n = q.n;
    const uint32_t R = (uint32_t)g.nty * (uint32_t)g.ty;
    const uint32_t C = (uint32_t)g.ntx * 64u;
    const uint32_t YE = (uint32_t)g.ntx * 6u * R;
    collide(f, p.ph.omc, p.ph.F);
    const NodeRng<T> rng(n, f); // stochastic-rounding bits (FP16S-SR only)
    float r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        // 64-bit element index: the stores of one bundle or node stay
        // provably adjacent and merge into wide stores
        const T e = enc<T>(f[i], rng.draw(i));
        lat[lat_at<L>(i, (int64_t)n, g.P)] = e;
        r[i] = ld(e);
    }
    if (x == c.x0) {
        const uint32_t o = ((uint32_t)c.bx * 6u * R + (uint32_t)y) * E;
#pragma unroll
        for (int k = 0; k < 3; ++k) at_byte(edge_out, o + k * R * E) = st<T>(r[3 * k]);
    }
    if (x == c.x1 - 1) {
        const uint32_t o = (((uint32_t)c.bx * 6u + 3u) * R + (uint32_t)y) * E;
#pragma unroll
        for (int k = 0; k < 3; ++k) at_byte(edge_out, o + k * R * E) = st<T>(r[3 * k + 2]);
    }
    if (q.bottom) {
        const uint32_t o = (YE + (uint32_t)c.by * 6u * C + (uint32_t)x) * E;
#pragma unroll
        for (int k = 0; k < 3; ++k) at_byte(edge_out, o + k * C * E) = st<T>(r[k]);
    }
    if (q.top) {
        const uint32_t o = (YE + ((uint32_t)c.by * 6u + 3u) * C + (uint32_t)x) * E;
#pragma unroll
        for (int k = 0; k < 3; ++k) at_byte(edge_out, o + k * C * E) = st<T>(r[6 + k]);
    }
}

template <int L, class T>
__global__ void __launch_bounds__(1024) k_npol64(KParams p, T* lat, const T* __restrict__ edge_in,
                                                 T* __restrict__ edge_out)
{
    const Geometry& g = p.g;
    TileCoord c;
    {
        const uint32_t t = xcd_tile(blockIdx.x, (uint32_t)g.ntx * (uint32_t)g.nty);
        const uint32_t by = __umulhi(t, g.ntx_rcp); // t / ntx, exact for this grid
        c.by = (int)by;
        c.bx = (int)(t - by * (uint32_t)g.ntx);
        c.x0 = c.bx * 64;
        c.y0 = c.by * g.ty;
        c.x1 = min(c.x0 + 64, (int)g.nx);
        c.y1 = min(c.y0 + g.ty, (int)g.ny);
    }
    const int lane = (int)threadIdx.x;
    const int y = c.y0 + (int)__builtin_amdgcn_readfirstlane(threadIdx.y);
    Npol64Node q;
    T fr[9], er[9];
    float f[9];
    npol64_issue<L, T>(p, c, lat, edge_in, lane, y, q, fr, er);
    npol64_resolve<L, T>(p, c, lat, edge_in, lane, q, fr, er, f);
    // every read of this tile's nodes precedes every in-place write
    __syncthreads();
    npol64_write<L, T>(p, c, lat, edge_out, lane, q, f);
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
    const int plane = p.g.tx * p.g.ty;
    const int me = ly * p.g.tx + lx;
    // Every load is issued before any is consumed and before the node is
    // known to be regular: the node's own slots and, on a tile side, the
    // three values a regular node there takes from the adjacent tile (tile
    // indices, rows and columns clamped into the buffers, so the addresses
    // are valid for any node).  Stored values stay undecoded until all are
    // in flight.
    const bool bottom = y == c.y0, top = y == c.y1 - 1, left = x == c.x0, right = x == c.x1 - 1;
    const int rows = (int)edge_rows(p.g), cols = (int)edge_cols(p.g);
    uint8_t t = T_SOLID;
    T raw[9];
    T eb[3] = {}, et[3] = {}, el[3] = {}, er[3] = {};
    if (inside) {
        t = p.types[n];
#pragma unroll
        for (int j = 0; j < 9; ++j) raw[j] = lat[lat_at<L>(j, n, p.g.P)]; // slot j = f*_{opp(j)}
        // directions 6 + k (c_y = +1) cross the bottom side, k (c_y = -1)
        // the top side, 2 + 3k (c_x = +1) the left side, 3k (c_x = -1) the
        // right side; k = c_x + 1 or c_y + 1 along the side
        if (bottom)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                eb[k] = edge_in[edge_y_at(p.g, max(c.by - 1, 0), 1, k, min(max(x - (k - 1), 0), cols - 1))];
        if (top)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                et[k] = edge_in[edge_y_at(p.g, min(c.by + 1, p.g.nty - 1), 0, k, min(max(x - (k - 1), 0), cols - 1))];
        if (left)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                el[k] = edge_in[edge_x_at(p.g, max(c.bx - 1, 0), 1, k, min(max(y - (k - 1), 0), rows - 1))];
        if (right)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                er[k] = edge_in[edge_x_at(p.g, min(c.bx + 1, p.g.ntx - 1), 0, k, min(max(y - (k - 1), 0), rows - 1))];
    }
    float own[9];
    if (inside) {
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            own[j] = ld(raw[j]);
            s[j * plane + me] = own[j];
        }
    }
    __syncthreads();
    const bool active = inside && updated(t);
    if (!active) return;
    float f[9];
    if (!(t & IRREGULAR)) {
        // the adjacent tile's published value where the source lies across a
        // side (corners from the bottom/top sides), else the tile's own LDS
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const int X = dir_cx(i), Y = dir_cy(i);
            const float v = s[dir_opp(i) * plane + me - X - Y * p.g.tx];
            if (i == 4)
                f[i] = own[4];
            else if (Y > 0 && bottom)
                f[i] = ld(eb[X + 1]);
            else if (Y < 0 && top)
                f[i] = ld(et[X + 1]);
            else if (X > 0 && left)
                f[i] = ld(el[Y + 1]);
            else if (X < 0 && right)
                f[i] = ld(er[Y + 1]);
            else
                f[i] = v;
        }
    } else {
        const uint32_t lk = p.links[n];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            int sx = x, sy = y;
            const int k = (lk & LINK_GENERAL) ? pull_source_xy(p.g, p.types, x, y, i, sx, sy)
                                              : linked_source(lk, i, x, y, sx, sy);
            const bool in_tile = sx >= c.x0 && sx < c.x1 && sy >= c.y0 && sy < c.y1;
            const bool cross = k == K_NODE && !in_tile;
            // LDS and edge reads at always-valid addresses; the value is
            // chosen afterwards (no pointer select across address spaces)
            const float vl = s[dir_opp(i) * plane + (in_tile ? (sy - c.y0) * p.g.tx + (sx - c.x0) : me)];
            const float ve = ld(edge_in[cross ? edge_src(p.g, c, sx, sy, i) : 0]);
            // K_SOLID: no exchange, slot i still holds f*_{opp(i)}
            f[i] = k == K_SOLID ? own[i] : (k == K_INLET ? p.ph.ein[i] : (cross ? ve : vl));
        }
        boundary_fix(p, x, y, f);
        record_inlet_density(p, x, y, f);
    }
    collide(f, p.ph.omc, p.ph.F);
    const NodeRng<T> rng((uint32_t)n, f); // stochastic-rounding bits (FP16S-SR only)
    float r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const T e = enc<T>(f[i], rng.draw(i));
        lat[lat_at<L>(dir_opp(i), n, p.g.P)] = e; // swap state: f*_i in slot opposite(i)
        r[i] = ld(e);
    }
    edge_emit(p.g, c, x, y, r, edge_out);
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
        if (p.rin)
            hipLaunchKernelGGL((k_lptl<L, T, 1>), dim3((uint32_t)blocks), dim3(block), 0, s, p, (const T*)src,
                               (T*)dst);
        else if (p.g.fw)
            hipLaunchKernelGGL((k_lptl<L, T, 2>), dim3((uint32_t)blocks), dim3(block), 0, s, p, (const T*)src,
                               (T*)dst);
        else
            hipLaunchKernelGGL((k_lptl<L, T, 0>), dim3((uint32_t)blocks), dim3(block), 0, s, p, (const T*)src,
                               (T*)dst);
        break;
    }
    case S_NPTL: {
        const dim3 blk(p.g.tx / p.g.vx, p.g.ty);
        const int mode = p.rin ? 1 : (p.g.fw ? 2 : 0);
        if (nptl_staged(p.g, L) && mode != 2) {
            const size_t sh = aos_stage_bytes<T>(p.g.ty);
            if (mode == 1)
                hipLaunchKernelGGL((k_nptl_aos<T, 1>), dim3((uint32_t)tiles), blk, sh, s, p, (const T*)src, (T*)dst);
            else
                hipLaunchKernelGGL((k_nptl_aos<T, 0>), dim3((uint32_t)tiles), blk, sh, s, p, (const T*)src, (T*)dst);
            break;
        }
#define LBM_NPTL_LAUNCH(VXV, MV)                                                                                     \
    hipLaunchKernelGGL((k_nptl<L, T, VXV, MV>), dim3((uint32_t)tiles), blk, 0, s, p, (const T*)src, (T*)dst)
        if (p.g.vx == 2) {
            if (mode == 1) LBM_NPTL_LAUNCH(2, 1);
            else if (mode == 2) LBM_NPTL_LAUNCH(2, 2);
            else LBM_NPTL_LAUNCH(2, 0);
        } else {
            if (mode == 1) LBM_NPTL_LAUNCH(1, 1);
            else if (mode == 2) LBM_NPTL_LAUNCH(1, 2);
            else LBM_NPTL_LAUNCH(1, 0);
        }
#undef LBM_NPTL_LAUNCH
        break;
    }
    case S_PUSH:
        // staged stores only for FP32 records of the collision layout: in the
        // stream and bundle layouts the direct stores are one contiguous run
        // per direction already, and binary16 staging is bound by its 2-byte
        // LDS accesses
        if constexpr (L == L_COLLISION) {
            if (sizeof(T) == 4 && tile_staged(p.g)) {
                using S = Stage<L, T>;
                const size_t sh = S::bytes(p.g.ty) + (size_t)(p.g.ty + 2) * S::RROW;
                hipLaunchKernelGGL((k_push_staged<L, T>), dim3((uint32_t)tiles), tb, sh, s, p, (const T*)src,
                                   (T*)dst);
                break;
            }
        }
        hipLaunchKernelGGL((k_push<L, T>), dim3((uint32_t)tiles), tb, 0, s, p, (const T*)src, (T*)dst);
        break;
    case S_NPOL:
        if (npol_lean(p.g, sizeof(T)))
            hipLaunchKernelGGL((k_npol64<L, T>), dim3((uint32_t)tiles), tb, 0, s, p, (T*)dst, (const T*)ein,
                               (T*)eout);
        else
            hipLaunchKernelGGL((k_npol<L, T>), dim3((uint32_t)tiles), tb, 0, s, p, (T*)dst, (const T*)ein, (T*)eout);
        break;
    case S_NSOL:
        hipLaunchKernelGGL((k_nsol<L, T>), dim3((uint32_t)tiles), tb, (size_t)9 * p.g.tx * p.g.ty * sizeof(float), s,
                           p, (T*)dst, (const T*)ein, (T*)eout);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L, class T>
static hipError_t launch_aa_t(const KParams& p, int parity, void* lat, void* obuf, hipStream_t s)
{
    const dim3 tb(p.g.tx, p.g.ty);
    const dim3 grid((uint32_t)((int64_t)p.g.ntx * p.g.nty));
    if constexpr (L == L_COLLISION) {
        if (tile_staged(p.g)) {
            using S = Stage<L, T>;
            const size_t sh = S::bytes(p.g.ty) + (size_t)(p.g.ty + 2) * S::RROW;
            if (parity == 0)
                hipLaunchKernelGGL((k_aa_even_aos<T>), grid, tb, sh, s, p, (T*)lat, (T*)obuf);
            else
                hipLaunchKernelGGL((k_aa_odd_aos<T>), grid, tb, sh, s, p, (T*)lat, (const T*)obuf);
            return hipGetLastError();
        }
    }
    if (parity == 0)
        hipLaunchKernelGGL((k_aa_even<L, T>), grid, tb, 0, s, p, (T*)lat, (T*)obuf);
    else
        hipLaunchKernelGGL((k_aa_odd<L, T>), grid, tb, 0, s, p, (T*)lat, (const T*)obuf);
    return hipGetLastError();
}

hipError_t launch_aa(int layout, int prec, const KParams& p, int parity, void* lat, void* obuf, hipStream_t s)
{
    return with_layout_storage(layout, prec, [&](auto L, auto TT) {
        return launch_aa_t<decltype(L)::value, typename decltype(TT)::type>(p, parity, lat, obuf, s);
    });
}

hipError_t launch_update(int scheme, int layout, int prec, const KParams& p, int block, const void* src, void* dst,
                         const void* ein, void* eout, hipStream_t s)
{
    return with_layout_storage(layout, prec, [&](auto L, auto TT) {
        return launch_update_t<decltype(L)::value, typename decltype(TT)::type>(scheme, p, block, src, dst, ein, eout,
                                                                               s);
    });
}

int lptl_block_size(int layout, int prec)
{
    int grid = 0, block = 0;
    const hipError_t e = with_layout_storage(layout, prec, [&](auto L, auto TT) {
        return hipOccupancyMaxPotentialBlockSize(&grid, &block,
                                                 k_lptl<decltype(L)::value, typename decltype(TT)::type, 0>, 0,
                                                 1024);
    });
    if (e != hipSuccess || block <= 0) return 256;
    return block;
}

} // namespace lbm
