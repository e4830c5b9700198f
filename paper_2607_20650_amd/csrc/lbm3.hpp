// lbm3.hpp -- the D3Q19 extension (the 3-D direction Section 6 names):
// types shared by the host runtime and the gfx950 kernels.
//
// Velocities ordered by (c_z, c_y, c_x) lexicographically among the vectors
// with components in {-1, 0, 1} and |c|^2 <= 2: five with c_z = -1, the nine
// of the D2Q9 plane, five with c_z = +1.  Rest is i = 9, opposite(i) = 18 - i.
// Node n = (z ny + y) px + x with the row pitch px of the 2-D case.
#pragma once

#include "lbm_common.hpp"

namespace lbm {

constexpr int Q3 = 19;

// In-plane position j of the five vectors with c_z = -1 or +1:
// (0,-1), (-1,0), (0,0), (1,0), (0,1) as (c_x, c_y).
__host__ __device__ constexpr int q3_cz(int i) { return i < 5 ? -1 : (i < 14 ? 0 : 1); }
__host__ __device__ constexpr int q3_cx(int i)
{
    return (i >= 5 && i < 14) ? (i - 5) % 3 - 1 : ((i < 5 ? i : i - 14) == 1 ? -1 : ((i < 5 ? i : i - 14) == 3 ? 1 : 0));
}
__host__ __device__ constexpr int q3_cy(int i)
{
    return (i >= 5 && i < 14) ? (i - 5) / 3 - 1 : ((i < 5 ? i : i - 14) == 0 ? -1 : ((i < 5 ? i : i - 14) == 4 ? 1 : 0));
}
__host__ __device__ constexpr int q3_opp(int i) { return 18 - i; }
__host__ __device__ constexpr int q3_c2(int i) { return q3_cx(i) * q3_cx(i) + q3_cy(i) * q3_cy(i) + q3_cz(i) * q3_cz(i); }

struct Geometry3 {
    int64_t nx, ny, nz;
    int64_t px;     // row pitch (nx rounded up to a multiple of 16)
    int64_t plane;  // px * ny
    int64_t P;      // node stride between direction planes (stream layout)
    int32_t xa, ya, za; // AxisKind per axis (x may be AX_INOUT)
    int32_t tx, ty; // block tile in (x, y); one z plane per block
    int32_t ntx, nty;
    // Blocked layout: one row and one plane, and ny rows and nz planes, as
    // steps of the slot index (whole blocks of 19 * 64 slots).
    int64_t rstep, pstep, yspan, zspan;
};

struct Physics3 {
    float omc;       // 1 - 1/tau
    float F[Q3];     // force term 3 w_i (c_i . g)
    float ein[Q3];   // shifted inlet equilibrium feq(1, u_in) - w
    float e0[Q3];    // shifted initial equilibrium feq(1, u0) - w
    float hg[3];     // g / 2 added to the reported velocity
    float u_in[3];
};

struct KParams3 {
    Geometry3 g;
    Physics3 ph;
    const uint8_t* types; // [nz][ny][px]; padding columns are solid
};

// Whether the collision layout runs the LDS-staged kernels: 64 x ty tiles
// (ty <= 8) and planes small enough that every element offset within one
// plane (plus a row) fits 32 bits (the staging copies' per-piece arithmetic).
__host__ __device__ inline bool aos3_staged(int64_t px, int64_t ny, int32_t tx, int32_t ty)
{
    return tx == 64 && ty >= 1 && ty <= 8 && (int64_t)Q3 * (px * ny + px) + 64 < ((int64_t)1 << 31);
}

} // namespace lbm
