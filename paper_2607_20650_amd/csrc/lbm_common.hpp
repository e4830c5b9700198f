// lbm_common.hpp -- types shared by the host runtime and the gfx950 kernels.
//
// D2Q9 in the direction order of the paper's Fig. 2 (b): i = 3*(c_y+1) + (c_x+1)
// (SW, S, SE, W, rest, E, NW, N, NE), opposite(i) = 8 - i.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum NodeType : uint8_t { T_FLUID = 0, T_SOLID = 1, T_INLET = 2, T_OUTLET = 3 };
enum AxisKind : int32_t { AX_PERIODIC = 0, AX_CLOSED = 1, AX_INOUT = 2 };
enum LayoutKind : int32_t { L_STREAM = 0, L_BUNDLE = 1, L_COLLISION = 2, L_BLOCKED = 3 /* D3Q19 only */ };
enum PrecKind : int32_t { P_FP32 = 0, P_FP16S = 1, P_FP16SR = 2, P_FP16C = 3, P_FP16CSR = 4 };
enum SchemeKind : int32_t { S_LPTL = 0, S_NPTL = 1, S_PUSH = 2, S_NPOL = 3, S_NSOL = 4, S_AA = 5 };

// What the stored slot (i, node) holds between updates.
enum StateKind : int32_t {
    ST_PULL = 0, // post-collision f*_i(node), not yet streamed (LPTL, NPTL, NPOL)
    ST_PUSH = 1, // streamed, pre-collision f_in_i(node) (two-lattice push)
    ST_SWAP = 2  // post-collision f*_i(node) kept in slot opposite(i) (swap scheme)
};

__host__ __device__ constexpr int dir_cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int dir_cy(int i) { return i / 3 - 1; }
__host__ __device__ constexpr int dir_opp(int i) { return 8 - i; }

// Everything a kernel needs about one simulation, passed by value.
struct Geometry {
    int64_t nx, ny;  // nodes per axis
    int64_t px;      // row pitch (nx rounded up to a multiple of 16)
    int64_t P;       // node stride between planes (stream) / bundles (bundle)
    int32_t xa, ya;  // AxisKind per axis
    int32_t tx, ty;  // tile extents (tiled schemes)
    int32_t ntx, nty;// tile counts
    int32_t vx;      // nodes per thread of the tiled pull
    uint32_t ntx_rcp;// ceil(2^32 / ntx) when t / ntx == umulhi(t, ntx_rcp) for every tile t, else 0
    int32_t zh;      // 1: the outlet column is a pressure (Zou-He) outlet, 0: zero gradient
    int32_t fw;      // 1: full-way bounce-back at solid nodes (two-lattice pull only), 0: halfway
};

struct Physics {
    float omc;        // 1 - 1/tau
    float F[9];       // force term 3 w_i (c_i . g)
    float ein[9];     // shifted inlet equilibrium feq(1, u_in) - w
    float e0[9];      // shifted initial equilibrium feq(1, u0) - w
    float hg[2];      // g / 2 added to the reported velocity
    float u_in[2];
};

struct KParams {
    Geometry g;
    Physics ph;
    const uint8_t* types; // node types [ny][px]; padding columns are solid
    // Neumann inlet only (null for the Dirichlet inlet): rho - 1 of the node
    // (1, y) of every row y after the previous update, read by this update
    // (rin) and recorded by it for the next one (rout; null in readouts).
    const float* rin;
    float* rout;
    // Source kinds of every node's pull, 2 bits per direction i at bits 2i
    // (LINK_* below), bit 31 set where a source lies across a periodic side;
    // null in readouts.
    const uint32_t* links;
};

// Kinds of a pull source in the per-node link words.
enum LinkKind : uint32_t {
    LINK_PLAIN = 0, // the neighbour (x, y) - c_i
    LINK_SOLID = 1, // bounce-back: the node's own value of the opposite direction
    LINK_INLET = 2, // an inlet node: the inlet equilibrium
    LINK_CLAMP = 3  // past the outlet: the outlet node (x, y - c_y) (zero gradient)
};
constexpr uint32_t LINK_GENERAL = 0x80000000u; // a source across a periodic side

// Edge-buffer ("buffer grid") extents of the one-lattice schemes, per parity:
// X edges hold, per tile column, 2 sides x 3 values (c_y+1) x every row of
// the tile grid; Y edges, per tile row, 2 sides x 3 values (c_x+1) x every
// column of the tile grid.
__host__ __device__ inline int64_t edge_rows(const Geometry& g) { return (int64_t)g.nty * g.ty; }
__host__ __device__ inline int64_t edge_cols(const Geometry& g) { return (int64_t)g.ntx * g.tx; }
__host__ __device__ inline int64_t edge_x_elems(const Geometry& g) { return (int64_t)g.ntx * 2 * 3 * edge_rows(g); }
__host__ __device__ inline int64_t edge_y_elems(const Geometry& g) { return (int64_t)g.nty * 2 * 3 * edge_cols(g); }

// Elements kept before and after every lattice of a simulation context, so
// that the plain-neighbour loads of any in-domain node stay inside the
// allocation and can be issued before the node type is known: a plain
// neighbour is at most px + 1 nodes away (one more for the second node of a
// two-node run), 9 elements a node.
__host__ __device__ inline int64_t lattice_guard(const Geometry& g) { return (9 * (g.px + 3) + 63) / 64 * 64; }

// Whether the lean NPOL kernel serves a grid: tiles one wavefront wide, every
// lattice byte offset (guards included) below 2^31, so the edge offsets are
// too, and tile indices that ntx_rcp divides exactly.
__host__ __device__ inline bool npol_lean(const Geometry& g, int elem_bytes)
{
    return g.tx == 64 && g.ntx_rcp != 0 && (9 * g.P + 2 * lattice_guard(g)) * elem_bytes < ((int64_t)1 << 31);
}

// Whether the two-lattice tiled pull of a collision-layout grid runs the
// LDS-staged kernel: tiles of 64 x ty nodes, one node per thread, up to 512
// threads.
__host__ __device__ inline bool nptl_staged(const Geometry& g, int layout)
{
    return layout == L_COLLISION && g.tx == 64 && g.vx == 1 && g.ty >= 1 && g.ty <= 8;
}

// Whether a 64-wide tiled kernel with one node per thread and at most 512
// threads can stage its tile region through LDS (PUSH with FP32 and AA, in
// the collision layout).
__host__ __device__ inline bool tile_staged(const Geometry& g)
{
    return g.tx == 64 && g.ty >= 1 && g.ty <= 8;
}

} // namespace lbm
