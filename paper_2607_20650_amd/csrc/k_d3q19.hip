// k_d3q19.hip -- the D3Q19 extension of the lattice update (the 3-D direction
// Section 6 names): the same BGK stream-and-collide with the incompressible
// equilibrium (Eq. 1-2), halfway bounce-back, inlet equilibrium and
// zero-gradient outlet, on a 19-velocity lattice.
//
// Two schemes, each for the stream (SoA), collision (AoS) and blocked (AoSoA)
// layouts and all five storage precisions:
//   PULL  two lattices, one-step pull (Section 3.3's two-lattice scheme);
//   AA    one lattice updated in place, alternating a local even update and a
//         pairwise-exchange odd update.
// One thread per node, a block covers a tile_x x tile_y patch of one z plane
// (rows of 64 nodes keep every direction's loads contiguous).  All kernels
// share one collide3(), so all variants of one precision agree bit for bit.
#include <algorithm>
#include <type_traits>

#include "lbm3.hpp"
#include "lbm3_kernels.hpp"
#include "lbm_device.hpp"
#include "lbm_edges.hpp"

namespace lbm {

// ------------------------------------------------------------------ layouts
// stream (SoA): i * P + n      collision (AoS): 19 n + i
// blocked (AoSoA): rows are cut into blocks of 64 nodes (the row pitch is a
// multiple of 64) and a block stores its 19 directions one after the other,
// 64 nodes each: ((n / 64) 19 + i) 64 + n mod 64.  A wavefront's load of one
// direction stays one contiguous run as in SoA, but all 19 directions of a
// block share a few DRAM pages, so an update touches 9 source rows and 1
// destination region instead of 19 + 19 separate planes.
template <int L> __device__ __forceinline__ int64_t lat3(int i, int64_t n, int64_t P)
{
    if constexpr (L == L_STREAM)
        return (int64_t)i * P + n;
    else if constexpr (L == L_BLOCKED)
        return (((n >> 6) * Q3 + i) << 6) + (n & 63);
    else
        return (int64_t)Q3 * n + i;
}

// Node offset of the neighbour at +c_i.
__device__ __forceinline__ int64_t q3_off(const Geometry3& g, int i)
{
    return q3_cx(i) + q3_cy(i) * g.px + q3_cz(i) * g.plane;
}

// Periodic wrap of the fixed neighbour offsets for a node on the border of a
// periodic axis (regular nodes lie on no other border): lo[a] is added when
// the neighbour at -1 along axis a lies across the low border, hi[a] when the
// one at +1 lies across the high border.
struct Wrap3 {
    int64_t lo[3], hi[3];
};
__device__ __forceinline__ Wrap3 wrap_of(const Geometry3& g, int64_t x, int64_t y, int64_t z)
{
    Wrap3 w;
    const int64_t span[3] = {g.nx, g.ny * g.px, g.nz * g.plane};
    const int64_t c[3] = {x, y, z}, n[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        w.lo[a] = c[a] == 0 ? span[a] : 0;
        w.hi[a] = c[a] == n[a] - 1 ? -span[a] : 0;
    }
    return w;
}
// Offset of the neighbour at +c_i (S = +1) or -c_i (S = -1) with the wrap.
template <int S> __device__ __forceinline__ int64_t wrapped_off(const Geometry3& g, const Wrap3& w, int i)
{
    int64_t o = S * q3_off(g, i);
    const int c[3] = {S * q3_cx(i), S * q3_cy(i), S * q3_cz(i)};
#pragma unroll
    for (int a = 0; a < 3; ++a) o += c[a] < 0 ? w.lo[a] : (c[a] > 0 ? w.hi[a] : 0);
    return o;
}
// Whether a thread's node lies on the border of an axis (periodic for a
// regular node).
__device__ __forceinline__ bool on_border(const Geometry3& g, int64_t x, int64_t y, int64_t z)
{
    return x == 0 || y == 0 || z == 0 || x == g.nx - 1 || y == g.ny - 1 || z == g.nz - 1;
}

// Blocked layout: indices of the slots of the 27 nodes (x + a, y + b, z + c),
// a, b, c in {-1, 0, 1}, around a regular node; at(a, b, c, s) is the index of
// slot s.  A row or plane step moves whole blocks (the row pitch is a multiple
// of 64), so only the three x neighbours need the block arithmetic and every
// slot index is one of them plus a wavefront-uniform offset (row and plane
// steps computed on the host).  With WRAP the parts take the periodic wrap of
// a node on a border (regular nodes lie on no other border, so a border of
// theirs is periodic).
template <bool WRAP> struct Blocked3 {
    int64_t xp[3], yo[3], zo[3];
    __device__ __forceinline__ Blocked3(const Geometry3& g, int64_t x, int64_t y, int64_t z, int64_t n)
    {
        int64_t dxm = -1, dxp = 1;
        yo[0] = -g.rstep, yo[1] = 0, yo[2] = g.rstep;
        zo[0] = -g.pstep, zo[1] = 0, zo[2] = g.pstep;
        if (WRAP) {
            if (x == 0) dxm += g.nx;
            if (x == g.nx - 1) dxp -= g.nx;
            if (y == 0) yo[0] += g.yspan;
            if (y == g.ny - 1) yo[2] -= g.yspan;
            if (z == 0) zo[0] += g.zspan;
            if (z == g.nz - 1) zo[2] -= g.zspan;
        }
        xp[0] = lat3<L_BLOCKED>(0, n + dxm, 0);
        xp[1] = lat3<L_BLOCKED>(0, n, 0);
        xp[2] = lat3<L_BLOCKED>(0, n + dxp, 0);
    }
    __device__ __forceinline__ int64_t at(int a, int b, int c, int s) const
    {
        return xp[a + 1] + yo[b + 1] + zo[c + 1] + 64 * s;
    }
};

// ------------------------------------------------------------------ collision
// Weights 1/3, 1/18, 1/36; first-moment constants t_i = 3 w_i with t_edge
// the float nearest 1/12 and t_axis = (1 - 8 t_edge) / 2 (both exact), so
// that 2 t_axis + 8 t_edge == 1 exactly along every axis; 9/2 w_i is exact.
constexpr float W3_REST = 1.0f / 3.0f;
constexpr float W3_AXIS = 1.0f / 18.0f;
constexpr float W3_EDGE = 1.0f / 36.0f;
constexpr float T3_EDGE = 1.0f / 12.0f;
constexpr float T3_AXIS = (1.0f - 8.0f * T3_EDGE) / 2.0f;
constexpr float H3_AXIS = 0.25f;
constexpr float H3_EDGE = 0.125f;

template <int I> __device__ __forceinline__ float c_dot3(float jx, float jy, float jz)
{
    constexpr int X = q3_cx(I), Y = q3_cy(I), Z = q3_cz(I);
    float s = 0.0f;
    bool first = true;
    if constexpr (X != 0) {
        s = X > 0 ? jx : -jx;
        first = false;
    }
    if constexpr (Y != 0) {
        s = first ? (Y > 0 ? jy : -jy) : (Y > 0 ? s + jy : s - jy);
        first = false;
    }
    if constexpr (Z != 0) s = first ? (Z > 0 ? jz : -jz) : (Z > 0 ? s + jz : s - jz);
    return s;
}

template <int I> __device__ __forceinline__ float feq3_shifted(float base, float jx, float jy, float jz)
{
    constexpr int C2 = q3_c2(I);
    if constexpr (C2 == 0) {
        return W3_REST * base;
    } else {
        const float cu = c_dot3<I>(jx, jy, jz);
        if constexpr (C2 == 1)
            return __builtin_fmaf(W3_AXIS, base, cu * __builtin_fmaf(H3_AXIS, cu, T3_AXIS));
        else
            return __builtin_fmaf(W3_EDGE, base, cu * __builtin_fmaf(H3_EDGE, cu, T3_EDGE));
    }
}

template <int I>
__device__ __forceinline__ void relax3(float* f, float base, float jx, float jy, float jz, float omc, const float* F)
{
    const float e = feq3_shifted<I>(base, jx, jy, jz);
    f[I] = e + __builtin_fmaf(omc, f[I] - e, F[I]);
}

template <int... Is>
__device__ __forceinline__ void relax3_all(float* f, float base, float jx, float jy, float jz, float omc,
                                           const float* F, std::integer_sequence<int, Is...>)
{
    (relax3<Is>(f, base, jx, jy, jz, omc, F), ...);
}

// Moments of shifted populations in a fixed order (collide3 and readouts).
__device__ __forceinline__ void moments3(const float* f, float& rho, float& jx, float& jy, float& jz)
{
    rho = ((((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) +
           (((f[8] + f[9]) + (f[10] + f[11])) + ((f[12] + f[13]) + (f[14] + f[15])))) +
          ((f[16] + f[17]) + f[18]);
    jx = (((f[3] + f[7]) + (f[10] + f[13])) + f[17]) - (((f[1] + f[5]) + (f[8] + f[11])) + f[15]);
    jy = (((f[4] + f[11]) + (f[12] + f[13])) + f[18]) - (((f[0] + f[5]) + (f[6] + f[7])) + f[14]);
    jz = (((f[14] + f[15]) + (f[16] + f[17])) + f[18]) - (((f[0] + f[1]) + (f[2] + f[3])) + f[4]);
}

// In: shifted incoming populations.  Out: shifted post-collision values.
__device__ __forceinline__ void collide3(float* f, float omc, const float* F)
{
    float rho, jx, jy, jz;
    moments3(f, rho, jx, jy, jz);
    const float jj = __builtin_fmaf(jx, jx, __builtin_fmaf(jy, jy, jz * jz));
    const float base = __builtin_fmaf(-1.5f, jj, rho);
    relax3_all(f, base, jx, jy, jz, omc, F, std::make_integer_sequence<int, Q3>{});
}

// ------------------------------------------------------------------ sources
// Pull source of direction i for node (x, y, z): (x, y, z) - c_i after the
// axis rules (periodic wraps, outside a closed side is solid, past the
// outlet the last plane is used).  Returns K_NODE with its index in sn,
// K_SOLID or K_INLET.
__device__ __forceinline__ int pull_source3(const Geometry3& g, const uint8_t* __restrict__ types, int64_t x,
                                            int64_t y, int64_t z, int i, int64_t& sn, int64_t& row)
{
    int64_t sx = x - q3_cx(i), sy = y - q3_cy(i), sz = z - q3_cz(i);
    if (sy < 0 || sy >= g.ny) {
        if (g.ya != AX_PERIODIC) return K_SOLID;
        sy = sy < 0 ? sy + g.ny : sy - g.ny;
    }
    if (sz < 0 || sz >= g.nz) {
        if (g.za != AX_PERIODIC) return K_SOLID;
        sz = sz < 0 ? sz + g.nz : sz - g.nz;
    }
    if (sx < 0 || sx >= g.nx) {
        if (g.xa == AX_PERIODIC)
            sx = sx < 0 ? sx + g.nx : sx - g.nx;
        else if (g.xa == AX_INOUT && sx >= g.nx)
            sx = g.nx - 1;
        else
            return K_SOLID;
    }
    row = sz * g.ny + sy;
    sn = row * g.px + sx;
    const uint8_t t = node_type(types[sn]);
    return t == T_SOLID ? K_SOLID : (t == T_INLET ? K_INLET : K_NODE);
}
__device__ __forceinline__ int pull_source3(const Geometry3& g, const uint8_t* __restrict__ types, int64_t x,
                                            int64_t y, int64_t z, int i, int64_t& sn)
{
    int64_t row;
    return pull_source3(g, types, x, y, z, i, sn, row);
}

// The five directions with c_x = -1 (1, 5, 8, 11, 15) numbered 0..4: their
// post-collision values at the outlet plane go to the AA side buffer, 5 per
// (y, z) row.
__host__ __device__ constexpr int q3_west(int i) { return i == 1 ? 0 : (i == 5 ? 1 : (i == 8 ? 2 : (i == 11 ? 3 : 4))); }

template <int S> __device__ __forceinline__ int post_slot3(int i) { return S == ST_SWAP ? q3_opp(i) : i; }

__device__ __forceinline__ float inlet3(const KParams3& p, int i)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, p.ph.ein[i])));
}

// Incoming populations of an updated node from a pull-like state (pull or
// swap form): one load per direction from a valid address, the inlet value
// chosen afterwards by value.
template <int L, int S, class T>
__device__ __forceinline__ void gather_pull3(const KParams3& p, const T* __restrict__ lat, int64_t x, int64_t y,
                                             int64_t z, int64_t n, float* f)
{
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
        int64_t sn = n;
        const int k = pull_source3(p.g, p.types, x, y, z, i, sn);
        const int64_t at = k == K_NODE ? lat3<L>(post_slot3<S>(i), sn, p.g.P) : lat3<L>(post_slot3<S>(q3_opp(i)), n, p.g.P);
        const float v = ld(lat[at]);
        f[i] = k == K_INLET ? inlet3(p, i) : v;
    }
}

// Incoming populations held in the push form: own slots, inlet-fed slots
// take the inlet equilibrium.
template <int L, class T>
__device__ __forceinline__ void gather_push3(const KParams3& p, const T* __restrict__ lat, int64_t x, int64_t y,
                                             int64_t z, int64_t n, float* f)
{
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
        int64_t sn = n;
        const int k = pull_source3(p.g, p.types, x, y, z, i, sn);
        const float v = ld(lat[lat3<L>(i, n, p.g.P)]);
        f[i] = k == K_INLET ? inlet3(p, i) : v;
    }
}

template <int L, int S, class T>
__device__ __forceinline__ void gather_state3(const KParams3& p, const T* __restrict__ lat, int64_t x, int64_t y,
                                              int64_t z, int64_t n, float* f)
{
    if constexpr (S == ST_PUSH)
        gather_push3<L>(p, lat, x, y, z, n, f);
    else
        gather_pull3<L, S>(p, lat, x, y, z, n, f);
}

// Node of the calling thread: block = one tile_x x tile_y patch of a z plane.
struct Node3 {
    int64_t x, y, z, n;
    uint32_t key; // unpadded node index (z ny + y) nx + x: the rounding key, the same in every layout
    bool in;
};
__device__ __forceinline__ Node3 node_of_thread(const Geometry3& g)
{
    const uint32_t per_plane = (uint32_t)g.ntx * (uint32_t)g.nty;
    const uint32_t b = blockIdx.x;
    const uint32_t z = b / per_plane, r = b - z * per_plane;
    const uint32_t by = r / (uint32_t)g.ntx, bx = r - by * (uint32_t)g.ntx;
    Node3 o;
    o.x = (int64_t)bx * g.tx + threadIdx.x;
    o.y = (int64_t)by * g.ty + threadIdx.y;
    o.z = z;
    o.in = o.x < g.nx && o.y < g.ny;
    o.n = (o.z * g.ny + o.y) * g.px + o.x;
    o.key = (uint32_t)((o.z * g.ny + o.y) * g.nx + o.x);
    return o;
}

// Store of a pull result.  FP32 results in the stream and blocked layouts go
// out as non-temporal stores (the destination lattice is not read again in
// this update): +7% (stream) and +8.6% (blocked) on the 256^3 sphere array in
// same-box A/Bs; in the collision layout they cost 47%.  16-bit non-temporal
// stores ran 38% slower (2-D measurement), and in 2-D the effect on the FP32
// pull was mixed (+5% on a 302 MB two-lattice case, -4.7% on a 78 GB one), so
// the 2-D kernels keep plain stores.
template <int L, class T> __device__ __forceinline__ void put_pulled3(T* p, T v)
{
    if constexpr ((L == L_STREAM || L == L_BLOCKED) && sizeof(T) == 4)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// ------------------------------------------------------------------ PULL
template <int L, class T>
__global__ void __launch_bounds__(256) k3_pull(KParams3 p, const T* __restrict__ src, T* __restrict__ dst)
{
    const Node3 q = node_of_thread(p.g);
    if (!q.in) return;
    const uint8_t t = p.types[q.n];
    float f[Q3];
    if (!(t & IRREGULAR)) {
        if (!__any(on_border(p.g, q.x, q.y, q.z))) {
            if constexpr (L == L_BLOCKED) {
                const Blocked3<false> nb(p.g, q.x, q.y, q.z, q.n);
#pragma unroll
                for (int i = 0; i < Q3; ++i) f[i] = ld(src[nb.at(-q3_cx(i), -q3_cy(i), -q3_cz(i), i)]);
            } else {
#pragma unroll
                for (int i = 0; i < Q3; ++i) f[i] = ld(src[lat3<L>(i, q.n - q3_off(p.g, i), p.g.P)]);
            }
        } else { // a wavefront with nodes on a periodic border
            if constexpr (L == L_BLOCKED) {
                const Blocked3<true> nb(p.g, q.x, q.y, q.z, q.n);
#pragma unroll
                for (int i = 0; i < Q3; ++i) f[i] = ld(src[nb.at(-q3_cx(i), -q3_cy(i), -q3_cz(i), i)]);
            } else {
                const Wrap3 w = wrap_of(p.g, q.x, q.y, q.z);
#pragma unroll
                for (int i = 0; i < Q3; ++i) f[i] = ld(src[lat3<L>(i, q.n + wrapped_off<-1>(p.g, w, i), p.g.P)]);
            }
        }
    } else if (updated(t)) {
        gather_pull3<L, ST_PULL>(p, src, q.x, q.y, q.z, q.n, f);
    } else {
        return;
    }
    collide3(f, p.ph.omc, p.ph.F);
    const NodeRng<T, Q3> rng(q.key, f); // stochastic-rounding bits (SR formats only)
#pragma unroll
    for (int i = 0; i < Q3; ++i) put_pulled3<L, T>(&dst[lat3<L>(i, q.n, p.g.P)], enc<T>(f[i], rng.draw(i)));
}

// ------------------------------------------------------------------ AA
// Even update: incoming values in the node's own slots (push form), results
// into its own slot opposite(i) (swap form).  Odd update: f*_i of the pull
// source read from the source's slot opposite(i) (own slot i on bounce-back),
// results stored with the push rules -- each location is read and written by
// one node only.  The exception is the zero-gradient outlet: a clamped source
// lies in another node's exchange set, so even updates also copy the outlet
// plane's c_x = -1 values into a side buffer (5 per (y, z) row) that odd
// updates read instead.
template <int L, class T>
__global__ void __launch_bounds__(256) k3_aa_even(KParams3 p, T* lat, T* __restrict__ obuf)
{
    const Node3 q = node_of_thread(p.g);
    if (!q.in) return;
    const uint8_t t = p.types[q.n];
    if (!updated(t)) return;
    float f[Q3];
    if (!(t & IRREGULAR)) {
#pragma unroll
        for (int i = 0; i < Q3; ++i) f[i] = ld(lat[lat3<L>(i, q.n, p.g.P)]);
    } else {
        gather_push3<L>(p, lat, q.x, q.y, q.z, q.n, f);
    }
    collide3(f, p.ph.omc, p.ph.F);
    const NodeRng<T, Q3> rng(q.key, f);
    const bool outlet = p.g.xa == AX_INOUT && q.x == p.g.nx - 1;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
        const T e = enc<T>(f[i], rng.draw(i));
        lat[lat3<L>(q3_opp(i), q.n, p.g.P)] = e;
        if (q3_cx(i) == -1 && outlet) obuf[(q.z * p.g.ny + q.y) * 5 + q3_west(i)] = e;
    }
}

// Odd AA update of a regular node: f*_i of (x, y, z) - c_i from its slot
// opposite(i), results into slot i of (x, y, z) + c_i.
template <int L, class T, bool WRAP>
__device__ __forceinline__ void aa_odd_regular(const KParams3& p, T* lat, const Node3& q)
{
    float f[Q3];
    if constexpr (L == L_BLOCKED) {
        const Blocked3<WRAP> nb(p.g, q.x, q.y, q.z, q.n);
#pragma unroll
        for (int i = 0; i < Q3; ++i) f[i] = ld(lat[nb.at(-q3_cx(i), -q3_cy(i), -q3_cz(i), q3_opp(i))]);
        collide3(f, p.ph.omc, p.ph.F);
        const NodeRng<T, Q3> rng(q.key, f);
#pragma unroll
        for (int i = 0; i < Q3; ++i) lat[nb.at(q3_cx(i), q3_cy(i), q3_cz(i), i)] = enc<T>(f[i], rng.draw(i));
    } else if constexpr (!WRAP) {
#pragma unroll
        for (int i = 0; i < Q3; ++i) f[i] = ld(lat[lat3<L>(q3_opp(i), q.n - q3_off(p.g, i), p.g.P)]);
        collide3(f, p.ph.omc, p.ph.F);
        const NodeRng<T, Q3> rng(q.key, f);
#pragma unroll
        for (int i = 0; i < Q3; ++i) lat[lat3<L>(i, q.n + q3_off(p.g, i), p.g.P)] = enc<T>(f[i], rng.draw(i));
    } else {
        const Wrap3 w = wrap_of(p.g, q.x, q.y, q.z);
#pragma unroll
        for (int i = 0; i < Q3; ++i) f[i] = ld(lat[lat3<L>(q3_opp(i), q.n + wrapped_off<-1>(p.g, w, i), p.g.P)]);
        collide3(f, p.ph.omc, p.ph.F);
        const NodeRng<T, Q3> rng(q.key, f);
#pragma unroll
        for (int i = 0; i < Q3; ++i) lat[lat3<L>(i, q.n + wrapped_off<1>(p.g, w, i), p.g.P)] = enc<T>(f[i], rng.draw(i));
    }
}

// Odd AA update of an irregular node: the boundary rules, loads and stores
// direct.
template <int L, class T>
__device__ __forceinline__ void aa_odd_boundary3(const KParams3& p, T* lat, const T* __restrict__ obuf, const Node3& q)
{
    float f[Q3];
    int kind[Q3];
    const bool outlet = p.g.xa == AX_INOUT && q.x == p.g.nx - 1;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
        int64_t sn = q.n, row = 0;
        kind[i] = pull_source3(p.g, p.types, q.x, q.y, q.z, i, sn, row);
        // a clamped outlet source comes from the side buffer; one load from a
        // valid address, the value chosen afterwards
        const bool clamped = kind[i] == K_NODE && outlet && q3_cx(i) == -1;
        const T* at = clamped ? obuf + (row * 5 + q3_west(i))
                              : lat + (kind[i] == K_NODE ? lat3<L>(q3_opp(i), sn, p.g.P) : lat3<L>(i, q.n, p.g.P));
        const float v = ld(*at);
        f[i] = kind[i] == K_INLET ? inlet3(p, i) : v;
    }
    collide3(f, p.ph.omc, p.ph.F);
    const NodeRng<T, Q3> rng(q.key, f);
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
        // own slot i when the pull source of i is solid: bounce-back
        if (kind[i] == K_SOLID) lat[lat3<L>(i, q.n, p.g.P)] = enc<T>(f[q3_opp(i)], rng.draw(q3_opp(i)));
        // zero-gradient outlet: the outlet plane also feeds itself along c_x = -1
        if (q3_cx(i) == -1 && outlet) {
            int64_t ty = q.y + q3_cy(i), tz = q.z + q3_cz(i);
            bool ok = true;
            if (ty < 0 || ty >= p.g.ny) {
                if (p.g.ya == AX_PERIODIC) ty = ty < 0 ? ty + p.g.ny : ty - p.g.ny;
                else ok = false;
            }
            if (tz < 0 || tz >= p.g.nz) {
                if (p.g.za == AX_PERIODIC) tz = tz < 0 ? tz + p.g.nz : tz - p.g.nz;
                else ok = false;
            }
            if (ok) {
                const int64_t tn = (tz * p.g.ny + ty) * p.g.px + (p.g.nx - 1);
                if (updated(p.types[tn])) lat[lat3<L>(i, tn, p.g.P)] = enc<T>(f[i], rng.draw(i));
            }
        }
        // f*_i to slot i of (x, y, z) + c_i when that node is updated
        int64_t tx = q.x + q3_cx(i), ty = q.y + q3_cy(i), tz = q.z + q3_cz(i);
        bool ok = true;
        if (tx < 0 || tx >= p.g.nx) {
            if (p.g.xa == AX_PERIODIC) tx = tx < 0 ? tx + p.g.nx : tx - p.g.nx;
            else ok = false;
        }
        if (ty < 0 || ty >= p.g.ny) {
            if (p.g.ya == AX_PERIODIC) ty = ty < 0 ? ty + p.g.ny : ty - p.g.ny;
            else ok = false;
        }
        if (tz < 0 || tz >= p.g.nz) {
            if (p.g.za == AX_PERIODIC) tz = tz < 0 ? tz + p.g.nz : tz - p.g.nz;
            else ok = false;
        }
        if (ok) {
            const int64_t tn = (tz * p.g.ny + ty) * p.g.px + tx;
            if (updated(p.types[tn])) lat[lat3<L>(i, tn, p.g.P)] = enc<T>(f[i], rng.draw(i));
        }
    }
}

template <int L, class T>
__global__ void __launch_bounds__(256) k3_aa_odd(KParams3 p, T* lat, const T* __restrict__ obuf)
{
    const Node3 q = node_of_thread(p.g);
    if (!q.in) return;
    const uint8_t t = p.types[q.n];
    if (!updated(t)) return;
    if (!(t & IRREGULAR)) {
        if (!__any(on_border(p.g, q.x, q.y, q.z)))
            aa_odd_regular<L, T, false>(p, lat, q);
        else // a wavefront with nodes on a periodic border
            aa_odd_regular<L, T, true>(p, lat, q);
        return;
    }
    aa_odd_boundary3<L, T>(p, lat, obuf, q);
}

// ------------------------------------------- collision layout, staged
// In the collision (AoS) layout a node's 19 values sit together (76 bytes in
// FP32), so a wavefront's load of one direction for 64 nodes touches 38
// cache lines for 256 useful bytes, 19 times over.  These kernels move whole
// records: a block covers a 64 x ty patch of one z plane (ty <= 8) and, for
// each of the three source planes in turn, copies the records of rows
// y0 - 1 .. y0 + ty,
// nodes x0 - 1 .. x0 + 64, into LDS with aligned 16-byte loads; every node
// whose sources all lie in that region takes the values of the directions
// with that c_z from there.  Rows and planes across a periodic side are
// staged wrapped, so nodes on those sides are served too; nodes on a
// periodic x side (their source lies at the far end of the row) and
// irregular nodes keep the direct accesses.  Results leave as whole records
// of the patch's rows (pull, even AA update) or, for the odd AA update,
// through three masked write-backs, one per target plane, of the elements
// the block's nodes own.
template <class T> struct Aos3 {
    static constexpr int CH = 16 / (int)sizeof(T);                  // elements per 16-byte piece
    static constexpr int BACK = (Q3 + CH - 1) / CH * CH;            // a staged row starts BACK elements before x0
    static constexpr int LEAD = BACK - Q3;                          // elements before the record of x0 - 1
    static constexpr int SEG = (LEAD + 66 * Q3 + CH - 1) / CH * CH; // staged elements per row
    static constexpr int NCH = SEG / CH;
    static constexpr int OUT = 64 * Q3; // elements of one result row
    static constexpr int OCH = OUT / CH;
    // the region rows, then one 16-byte slot (element dummy(ty)) that takes
    // the pieces a staging copy drops
    static constexpr int dummy(int ty) { return (ty + 2) * SEG; }
    static constexpr size_t bytes(int ty) { return (size_t)(ty + 2) * SEG * sizeof(T) + 16; }
    // staged element of slot i of record c (node x0 - 1 + c) in region row r (row y0 - 1 + r)
    static __device__ __forceinline__ int at(int r, int c, int i) { return r * SEG + LEAD + Q3 * c + i; }
};

// Plane z wrapped once across a periodic side, or -1 outside a closed one.
__device__ __forceinline__ int64_t wrap_plane3(const Geometry3& g, int64_t z)
{
    if (z >= 0 && z < g.nz) return z;
    if (g.za != AX_PERIODIC) return -1;
    z = z < 0 ? z + g.nz : z - g.nz;
    return z >= 0 && z < g.nz ? z : -1;
}

// Row y wrapped once across a periodic side, or -1 outside a closed one (or
// still outside after one wrap: a staged row below the last one any node of
// the patch reads).  32-bit: a plane has fewer than 2^31 / 19 nodes (the
// staged kernels are launched only then).
__device__ __forceinline__ int wrap_row3(const Geometry3& g, int y)
{
    const int ny = (int)g.ny;
    if (y >= 0 && y < ny) return y;
    if (g.ya != AX_PERIODIC) return -1;
    y = y < 0 ? y + ny : y - ny;
    return y >= 0 && y < ny ? y : -1;
}

// Stage region rows 0 .. ty + 1 (rows y0 - 1 .. y0 + ty of plane z, wrapped)
// or, with own_rows, only the patch's rows 1 .. ty.  The copy is cut into
// units of 64 consecutive pieces of one row (1 KB for FP32), dealt to the
// wavefronts: a unit's row, wrap and bounds are wavefront-uniform (scalar
// arithmetic), so a lane only adds its own piece index.  Each wavefront
// issues the loads of up to CHUNK units before it writes any of them; an
// empty asm takes the loaded values first (else the optimiser fuses each
// load with its write and waits a round trip per piece), and a piece that is
// not copied loads from the lattice's first element and goes to the dummy
// LDS slot.  The per-plane offsets are 32-bit (the staged kernels run only
// for planes that fit, aos3_staged).
template <int CHUNK, class T>
__device__ __forceinline__ void stage3(const Geometry3& g, const T* __restrict__ lat, T* s, int x0, int y0, int64_t z,
                                       bool own_rows, int ty, int tid, int nthr)
{
    using A = Aos3<T>;
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    constexpr int M = (A::NCH + 63) / 64; // units per row
    const int64_t lim = (int64_t)Q3 * g.plane * g.nz;
    const int r0 = own_rows ? 1 : 0, nr = own_rows ? ty : ty + 2;
    const int64_t zw = wrap_plane3(g, z);
    const int64_t base = (int64_t)Q3 * (zw < 0 ? 0 : zw) * g.plane; // element of node (0, 0, zw)
    const int64_t lo = -base, hi = lim - A::CH - base;               // valid offsets from base
    const int rel_lo = (int)max(lo, (int64_t)INT32_MIN), rel_hi = (int)min(hi, (int64_t)INT32_MAX);
    const int px = (int)g.px;
    const int wave = (int)__builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, nwv = nthr >> 6;
    const int units = nr * M;
    for (int ub = 0; ub < units; ub += CHUNK * nwv) {
        u32x4 v[CHUNK];
        int so[CHUNK];
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            if (ub + j * nwv >= units) break; // block-uniform
            const int u = ub + j * nwv + wave;  // wavefront-uniform
            const int r = r0 + u / M, q = (u % M) * 64 + lane;
            const int yw = wrap_row3(g, y0 - 1 + r);
            const int rel = Q3 * (yw * px + x0) - A::BACK + q * A::CH;
            const bool ok = u < units && zw >= 0 && yw >= 0 && q < A::NCH && rel >= rel_lo && rel <= rel_hi;
            so[j] = ok ? r * A::SEG + q * A::CH : A::dummy(ty);
            v[j] = *reinterpret_cast<const u32x4*>(lat + (ok ? base + rel : 0));
        }
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            if (ub + j * nwv >= units) break;
            asm volatile("" : "+v"(v[j]));
        }
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            if (ub + j * nwv >= units) break;
            *reinterpret_cast<u32x4*>(s + so[j]) = v[j];
        }
    }
}

// Whole result records of the patch's rows, staged at s[r * OUT + 19 lx + i]
// for patch row r, to the lattice (nodes x0 .. min(x0 + 64, px) - 1): units
// of 64 consecutive pieces of one row per wavefront, as in stage3.
template <class T>
__device__ __forceinline__ void store_rows3(const Geometry3& g, T* __restrict__ lat, const T* s, int x0, int y0,
                                            int64_t z, int ty, int tid, int nthr)
{
    using A = Aos3<T>;
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    constexpr int M = (A::OCH + 63) / 64; // units per row
    const int rows = (int)min((int64_t)ty, g.ny - y0);
    const int wch = Q3 * (int)(min((int64_t)x0 + 64, g.px) - x0) / A::CH;
    T* const base = lat + (int64_t)Q3 * (z * g.plane + (int64_t)y0 * g.px + x0); // first element of the patch
    const int rowlen = Q3 * (int)g.px;
    const int wave = (int)__builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, nwv = nthr >> 6;
    for (int u = wave; u < rows * M; u += nwv) {
        const int r = u / M, q = (u % M) * 64 + lane;
        if (q < wch)
            *reinterpret_cast<u32x4*>(base + (r * rowlen + q * A::CH)) =
                *reinterpret_cast<const u32x4*>(s + r * A::OUT + q * A::CH);
    }
}

// Values of the directions with c_z = CZ for a node served from the staged
// plane: slot SLOT(i) of the record at (x, y) - (c_x, c_y) -- slot i for the
// pull, slot opposite(i) for the odd AA update.
template <int CZ, bool OPP, class T>
__device__ __forceinline__ void take3(const T* s, int lx, int ly, float* f)
{
    using A = Aos3<T>;
#pragma unroll
    for (int i = 0; i < Q3; ++i)
        if (q3_cz(i) == CZ) f[i] = ld(s[A::at(ly + 1 - q3_cy(i), lx + 1 - q3_cx(i), OPP ? q3_opp(i) : i)]);
}

template <class T>
__global__ void __launch_bounds__(512) k3_pull_aos(KParams3 p, const T* __restrict__ src, T* __restrict__ dst)
{
    using A = Aos3<T>;
    extern __shared__ __align__(16) unsigned char smem3[];
    T* s = reinterpret_cast<T*>(smem3);
    const Node3 q = node_of_thread(p.g);
    const int lx = threadIdx.x, ly = threadIdx.y, ty = (int)blockDim.y, tid = ly * 64 + lx, nthr = 64 * ty;
    const int x0 = (int)q.x - lx, y0 = (int)q.y - ly;
    const uint8_t t = q.in ? p.types[q.n] : (uint8_t)T_SOLID;
    const bool upd = q.in && updated(t);
    const bool staged = upd && !(t & IRREGULAR) && q.x > 0 && q.x < p.g.nx - 1;
    float f[Q3];
    // directions with c_z come from plane z - c_z (one loop body for the
    // three planes).  Four staging units in flight per wavefront: eight held
    // more registers (119 VGPRs, 4 waves per SIMD) and ran 6% slower
    // (256^3 sphere array A/B)
#pragma unroll 1
    for (int cz = -1; cz <= 1; ++cz) {
        stage3<4, T>(p.g, src, s, x0, y0, q.z - cz, false, ty, tid, nthr);
        __syncthreads();
        if (staged) {
            if (cz < 0)
                take3<-1, false>(s, lx, ly, f);
            else if (cz == 0)
                take3<0, false>(s, lx, ly, f);
            else
                take3<1, false>(s, lx, ly, f);
        }
        __syncthreads();
    }
    if (upd && !staged) {
        if (!(t & IRREGULAR)) { // regular node on a periodic x side: fixed offsets with the wrap
            const Wrap3 w = wrap_of(p.g, q.x, q.y, q.z);
#pragma unroll
            for (int i = 0; i < Q3; ++i) f[i] = ld(src[lat3<L_COLLISION>(i, q.n + wrapped_off<-1>(p.g, w, i), p.g.P)]);
        } else {
            gather_pull3<L_COLLISION, ST_PULL>(p, src, q.x, q.y, q.z, q.n, f);
        }
    }
    T e[Q3];
#pragma unroll
    for (int i = 0; i < Q3; ++i) e[i] = T{};
    if (upd) {
        collide3(f, p.ph.omc, p.ph.F);
        const NodeRng<T, Q3> rng(q.key, f); // stochastic-rounding bits (SR formats only)
#pragma unroll
        for (int i = 0; i < Q3; ++i) e[i] = enc<T>(f[i], rng.draw(i));
    }
    // not updated: 0, what every lattice holds there
#pragma unroll
    for (int i = 0; i < Q3; ++i) s[ly * A::OUT + Q3 * lx + i] = e[i];
    __syncthreads();
    store_rows3<T>(p.g, dst, s, x0, y0, q.z, ty, tid, nthr);
}

// The same pull marching in z: a block covers one 64 x ty patch of zb
// consecutive planes z0 .. z0 + zb - 1 and stages the planes z0 - 1 ..
// z0 + zb one at a time, each once.  From staged plane k every node takes
// the directions with c_z = +1 of its node in plane k + 1, those with
// c_z = 0 of plane k and those with c_z = -1 of plane k - 1, whose inflow is
// then complete: it collides and leaves through LDS as whole records.  The
// partial inflows of planes k and k + 1 stay in registers.  Against
// k3_pull_aos (three staged planes per result plane) this stages
// (zb + 2) / zb planes per result plane.  It runs for FP32 records: 24k
// against 20.6k MLUPS (256^3 sphere array, 64 x 8 patches, 16 planes per
// block).  With 16-bit records the three-plane kernel stays ahead (32.4k
// against 28.4k): the carried inflows hold the kernel at 4 wavefronts per
// SIMD, and halving the bytes of each copy left less to save.
template <class T>
__global__ void __launch_bounds__(512) k3_pull_aos_z(KParams3 p, const T* __restrict__ src, T* __restrict__ dst,
                                                     int zb)
{
    using A = Aos3<T>;
    extern __shared__ __align__(16) unsigned char smem3z[];
    T* s = reinterpret_cast<T*>(smem3z);
    const uint32_t per_plane = (uint32_t)p.g.ntx * (uint32_t)p.g.nty;
    const uint32_t nzc = (uint32_t)((p.g.nz + zb - 1) / zb);
    // each XCD takes a contiguous band of the blocks: the patches of one
    // z range next to each other, sharing their halo rows in one L2
    const uint32_t b = xcd_tile(blockIdx.x, per_plane * nzc);
    const uint32_t zc = b / per_plane, r = b - zc * per_plane;
    const uint32_t by = r / (uint32_t)p.g.ntx, bx = r - by * (uint32_t)p.g.ntx;
    const int lx = threadIdx.x, ly = threadIdx.y, ty = (int)blockDim.y, tid = ly * 64 + lx, nthr = 64 * ty;
    const int x0 = (int)bx * 64, y0 = (int)by * ty;
    const int64_t x = x0 + lx, y = y0 + ly;
    const bool in = x < p.g.nx && y < p.g.ny;
    const int64_t za = (int64_t)zc * zb, zend = min(za + zb, p.g.nz);
    // fp: inflow of plane k - 1 (all but c_z = -1 taken), fc: of plane k
    // (c_z = +1 taken), fn: of plane k + 1
    float fp[Q3], fc[Q3], fn[Q3];
#pragma unroll
    for (int i = 0; i < Q3; ++i) fp[i] = fc[i] = fn[i] = 0.0f;
#pragma unroll 1
    for (int64_t k = za - 1; k <= zend; ++k) {
        stage3<4, T>(p.g, src, s, x0, y0, k, false, ty, tid, nthr);
        __syncthreads();
        take3<1, false>(s, lx, ly, fn);
        take3<0, false>(s, lx, ly, fc);
        take3<-1, false>(s, lx, ly, fp);
        __syncthreads();
        if (k > za) { // block-uniform: plane k - 1 is complete
            const int64_t z = k - 1;
            const int64_t n = (z * p.g.ny + y) * p.g.px + x;
            const uint8_t t = in ? p.types[n] : (uint8_t)T_SOLID;
            const bool upd = in && updated(t);
            const bool staged = upd && !(t & IRREGULAR) && x > 0 && x < p.g.nx - 1;
            if (upd && !staged) {
                if (!(t & IRREGULAR)) { // regular node on a periodic x side: fixed offsets with the wrap
                    const Wrap3 w = wrap_of(p.g, x, y, z);
#pragma unroll
                    for (int i = 0; i < Q3; ++i)
                        fp[i] = ld(src[lat3<L_COLLISION>(i, n + wrapped_off<-1>(p.g, w, i), p.g.P)]);
                } else {
                    gather_pull3<L_COLLISION, ST_PULL>(p, src, x, y, z, n, fp);
                }
            }
            T e[Q3];
#pragma unroll
            for (int i = 0; i < Q3; ++i) e[i] = T{};
            if (upd) {
                collide3(fp, p.ph.omc, p.ph.F);
                const NodeRng<T, Q3> rng((uint32_t)((z * p.g.ny + y) * p.g.nx + x), fp);
#pragma unroll
                for (int i = 0; i < Q3; ++i) e[i] = enc<T>(fp[i], rng.draw(i));
            }
            // not updated: 0, what every lattice holds there
#pragma unroll
            for (int i = 0; i < Q3; ++i) s[ly * A::OUT + Q3 * lx + i] = e[i];
            __syncthreads();
            store_rows3<T>(p.g, dst, s, x0, y0, z, ty, tid, nthr);
            __syncthreads(); // the next staging overwrites s
        }
#pragma unroll
        for (int i = 0; i < Q3; ++i) {
            if (q3_cz(i) >= 0) fp[i] = fc[i];
            if (q3_cz(i) == 1) fc[i] = fn[i];
        }
    }
}

// Planes per block of k3_pull_aos_z: 4 to 16, as many as keep 2048 or more
// blocks (the chip holds 512 of them at once).  Small lattices get 4: a
// partial last range then has as few as one plane.
static inline int aos3_zb(const Geometry3& g)
{
    const int64_t per_plane = (int64_t)g.ntx * g.nty;
    return (int)std::max<int64_t>(4, std::min<int64_t>(16, g.nz * per_plane / 2048));
}

template <class T>
__global__ void __launch_bounds__(512) k3_aa_even_aos(KParams3 p, T* lat, T* __restrict__ obuf)
{
    using A = Aos3<T>;
    extern __shared__ __align__(16) unsigned char smem3e[];
    T* s = reinterpret_cast<T*>(smem3e);
    const Node3 q = node_of_thread(p.g);
    const int lx = threadIdx.x, ly = threadIdx.y, ty = (int)blockDim.y, tid = ly * 64 + lx, nthr = 64 * ty;
    const int x0 = (int)q.x - lx, y0 = (int)q.y - ly;
    stage3<4, T>(p.g, lat, s, x0, y0, q.z, true, ty, tid, nthr);
    __syncthreads();
    const uint8_t t = q.in ? p.types[q.n] : (uint8_t)T_SOLID;
    const bool upd = q.in && updated(t);
    float f[Q3];
    // the node's own record: the incoming values (push form)
    T e[Q3];
#pragma unroll
    for (int i = 0; i < Q3; ++i) e[i] = s[A::at(ly + 1, lx + 1, i)];
    if (upd) {
        if (!(t & IRREGULAR)) {
#pragma unroll
            for (int i = 0; i < Q3; ++i) f[i] = ld(e[i]);
        } else {
            gather_push3<L_COLLISION>(p, lat, q.x, q.y, q.z, q.n, f);
        }
        collide3(f, p.ph.omc, p.ph.F);
        const NodeRng<T, Q3> rng(q.key, f);
        const bool outlet = p.g.xa == AX_INOUT && q.x == p.g.nx - 1;
#pragma unroll
        for (int i = 0; i < Q3; ++i) {
            const T v = enc<T>(f[i], rng.draw(i));
            e[q3_opp(i)] = v; // swap form
            if (q3_cx(i) == -1 && outlet) obuf[(q.z * p.g.ny + q.y) * 5 + q3_west(i)] = v;
        }
    }
    __syncthreads(); // every staged record is read
    // nodes that are not updated put back what they were staged with
#pragma unroll
    for (int i = 0; i < Q3; ++i) s[ly * A::OUT + Q3 * lx + i] = e[i];
    __syncthreads();
    store_rows3<T>(p.g, lat, s, x0, y0, q.z, ty, tid, nthr);
}

// Masked write-back of the slots with c_z = CZ of the staged region of plane
// z: in a record they are one run (slots 0-4, 5-13 or 14-18), and
// consecutive lanes take consecutive elements of the runs of consecutive
// records, so one store instruction covers a few whole runs.
template <int CZ, class T>
__device__ __forceinline__ void store_group3(const Geometry3& g, T* __restrict__ lat, const T* s,
                                             const uint8_t* mask, int x0, int y0, int64_t z, int ty, int tid,
                                             int nthr)
{
    using A = Aos3<T>;
    constexpr int S0 = CZ < 0 ? 0 : (CZ == 0 ? 5 : 14); // first slot of the run
    constexpr int G = CZ == 0 ? 9 : 5;                  // slots in the run
    constexpr int PER_ROW = 66 * G;                     // records x0 - 1 .. x0 + 64
    static_assert(q3_cz(S0) == CZ && q3_cz(S0 + G - 1) == CZ && (S0 == 0 || q3_cz(S0 - 1) != CZ) &&
                      (S0 + G == Q3 || q3_cz(S0 + G) != CZ),
                  "the slots of one c_z form one run");
    // marked rows and planes exist (wrapped at most once): 64-bit plane base,
    // 32-bit offsets within the plane
    const int64_t base = (int64_t)Q3 * wrap_plane3(g, z) * g.plane;
    const int px = (int)g.px;
    for (int k = tid; k < (ty + 2) * PER_ROW; k += nthr) {
        const int r = k / PER_ROW, e = k - r * PER_ROW;
        const int c = e / G, j = S0 + (e - c * G); // slot j of record c (node x0 - 1 + c)
        const int o = A::at(r, c, j);
        if (mask[o]) lat[base + (Q3 * (wrap_row3(g, y0 - 1 + r) * px + x0 - 1 + c) + j)] = s[o];
    }
}

// Targets of the directions with c_z = CZ: slot i of (x, y) + (c_x, c_y).
template <int CZ, class T>
__device__ __forceinline__ void put3(T* s, uint8_t* mask, int lx, int ly, const T* e)
{
    using A = Aos3<T>;
#pragma unroll
    for (int i = 0; i < Q3; ++i)
        if (q3_cz(i) == CZ) {
            const int o = A::at(ly + 1 + q3_cy(i), lx + 1 + q3_cx(i), i);
            s[o] = e[i];
            mask[o] = 1;
        }
}

template <class T>
__global__ void __launch_bounds__(512) k3_aa_odd_aos(KParams3 p, T* lat, const T* __restrict__ obuf)
{
    using A = Aos3<T>;
    extern __shared__ __align__(16) unsigned char smem3o[];
    T* s = reinterpret_cast<T*>(smem3o);
    uint8_t* mask = smem3o + A::bytes(blockDim.y);
    const Node3 q = node_of_thread(p.g);
    const int lx = threadIdx.x, ly = threadIdx.y, ty = (int)blockDim.y, tid = ly * 64 + lx, nthr = 64 * ty;
    const int x0 = (int)q.x - lx, y0 = (int)q.y - ly;
    const uint8_t t = q.in ? p.types[q.n] : (uint8_t)T_SOLID;
    const bool upd = q.in && updated(t);
    const bool staged = upd && !(t & IRREGULAR) && q.x > 0 && q.x < p.g.nx - 1;
    float f[Q3];
    // f*_i of the source (x, y, z) - c_i sits in its slot opposite(i)
    stage3<4, T>(p.g, lat, s, x0, y0, q.z + 1, false, ty, tid, nthr);
    __syncthreads();
    if (staged) take3<-1, true>(s, lx, ly, f);
    __syncthreads();
    stage3<4, T>(p.g, lat, s, x0, y0, q.z, false, ty, tid, nthr);
    __syncthreads();
    if (staged) take3<0, true>(s, lx, ly, f);
    __syncthreads();
    stage3<4, T>(p.g, lat, s, x0, y0, q.z - 1, false, ty, tid, nthr);
    __syncthreads();
    if (staged) take3<1, true>(s, lx, ly, f);
    __syncthreads();
    if (upd && !staged) {
        if (!(t & IRREGULAR))
            aa_odd_regular<L_COLLISION, T, true>(p, lat, q);
        else
            aa_odd_boundary3<L_COLLISION, T>(p, lat, obuf, q);
    }
    T e[Q3];
    if (staged) {
        collide3(f, p.ph.omc, p.ph.F);
        const NodeRng<T, Q3> rng(q.key, f);
#pragma unroll
        for (int i = 0; i < Q3; ++i) e[i] = enc<T>(f[i], rng.draw(i));
    }
    // one masked write-back per target plane z + c_z; each writes only the
    // slots with that c_z, so the results of all three are put and marked
    // in one pass
    const int nmask = (ty + 2) * A::SEG / 4;
    for (int k = tid; k < nmask; k += nthr) reinterpret_cast<uint32_t*>(mask)[k] = 0u;
    __syncthreads();
    if (staged) {
        put3<-1>(s, mask, lx, ly, e);
        put3<0>(s, mask, lx, ly, e);
        put3<1>(s, mask, lx, ly, e);
    }
    __syncthreads();
    store_group3<-1, T>(p.g, lat, s, mask, x0, y0, q.z - 1, ty, tid, nthr);
    store_group3<0, T>(p.g, lat, s, mask, x0, y0, q.z, ty, tid, nthr);
    store_group3<1, T>(p.g, lat, s, mask, x0, y0, q.z + 1, ty, tid, nthr);
}

// ------------------------------------------------------------------ setup
__device__ __forceinline__ uint8_t derive_type3(const Geometry3& g, const uint8_t* __restrict__ flags, int64_t x,
                                                int64_t y, int64_t z)
{
    if (x < 0 || y < 0 || z < 0 || x >= g.nx || y >= g.ny || z >= g.nz) return T_SOLID;
    if (flags[(z * g.ny + y) * g.nx + x]) return T_SOLID;
    if (g.xa == AX_INOUT && x == 0) return T_INLET;
    if (g.xa == AX_INOUT && x == g.nx - 1) return T_OUTLET;
    return T_FLUID;
}

// Type of the node at (x, y, z) with periodic axes wrapped; outside a
// non-periodic side counts as solid.
__device__ __forceinline__ uint8_t neighbour_type3(const Geometry3& g, const uint8_t* __restrict__ flags, int64_t x,
                                                   int64_t y, int64_t z)
{
    if (g.xa == AX_PERIODIC) x = x < 0 ? x + g.nx : (x >= g.nx ? x - g.nx : x);
    if (g.ya == AX_PERIODIC) y = y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
    if (g.za == AX_PERIODIC) z = z < 0 ? z + g.nz : (z >= g.nz ? z - g.nz : z);
    return derive_type3(g, flags, x, y, z);
}

// types [nz][ny][px]: NodeType plus the IRREGULAR mark when the node or one
// of its 18 neighbours (across periodic sides: the wrapped one) is not a
// plain fluid node.  Regular nodes stream with fixed offsets, wrapped on the
// borders of periodic axes; every other node takes the boundary rules.
__global__ void k3_types(Geometry3 g, const uint8_t* __restrict__ flags, uint8_t* __restrict__ types)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.plane * g.nz) return;
    const int64_t z = m / g.plane, r = m - z * g.plane, y = r / g.px, x = r - y * g.px;
    const uint8_t t = derive_type3(g, flags, x, y, z);
    bool irr = t != T_FLUID;
    for (int i = 0; i < Q3 && !irr; ++i)
        if (neighbour_type3(g, flags, x + q3_cx(i), y + q3_cy(i), z + q3_cz(i)) != T_FLUID) irr = true;
    types[m] = (uint8_t)(t | (irr ? IRREGULAR : 0));
}

static inline uint32_t blocks3(int64_t n, int b) { return (uint32_t)((n + b - 1) / b); }

template <int S, int L, class T> __global__ void k3_init(KParams3 p, T* __restrict__ lat)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.g.plane * p.g.nz) return;
    const int64_t z = n / p.g.plane, r = n - z * p.g.plane, y = r / p.g.px, x = r - y * p.g.px;
    const bool upd = updated(p.types[n]);
#pragma unroll
    for (int j = 0; j < Q3; ++j) {
        float v = 0.0f;
        if (upd) {
            if constexpr (S == ST_PULL) {
                v = p.ph.e0[j];
            } else if constexpr (S == ST_SWAP) {
                v = p.ph.e0[q3_opp(j)];
            } else {
                int64_t sn;
                const int k = pull_source3(p.g, p.types, x, y, z, j, sn);
                v = k == K_NODE ? p.ph.e0[j] : (k == K_SOLID ? p.ph.e0[q3_opp(j)] : p.ph.ein[j]);
            }
        }
        lat[lat3<L>(j, n, p.g.P)] = st<T>(v);
    }
}

// Post-collision values f [19][nz][ny][nx] -> the slots of a pull or swap lattice.
template <int S, int L, class T> __global__ void k3_set_post(KParams3 p, const float* __restrict__ f, T* __restrict__ lat)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = p.g.nx * p.g.ny * p.g.nz;
    if (m >= N) return;
    const int64_t x = m % p.g.nx, yz = m / p.g.nx;
    const int64_t n = yz * p.g.px + x;
    if (!updated(p.types[n])) return;
#pragma unroll
    for (int i = 0; i < Q3; ++i) lat[lat3<L>(post_slot3<S>(i), n, p.g.P)] = st<T>(f[i * N + m]);
}

template <int L, class T> __global__ void k3_pull_to_push(KParams3 p, const T* __restrict__ pull, T* __restrict__ push)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.g.plane * p.g.nz) return;
    const int64_t z = n / p.g.plane, r = n - z * p.g.plane, y = r / p.g.px, x = r - y * p.g.px;
    if (!updated(p.types[n])) return;
    float f[Q3];
    gather_pull3<L, ST_PULL>(p, pull, x, y, z, n, f);
#pragma unroll
    for (int i = 0; i < Q3; ++i) push[lat3<L>(i, n, p.g.P)] = st<T>(f[i]);
}

// AA side buffer from a swap-form lattice (a state load at odd parity):
// obuf[row 5 + k] = f*_i of the outlet node of the row, for the five c_x = -1
// directions, which the swap form keeps in slot opposite(i).
template <int L, class T> __global__ void k3_aa_outlet_fill(KParams3 p, const T* __restrict__ lat, T* __restrict__ obuf)
{
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= p.g.ny * p.g.nz) return;
    const int64_t n = row * p.g.px + (p.g.nx - 1);
    if (!updated(p.types[n])) return;
#pragma unroll
    for (int i = 0; i < Q3; ++i)
        if (q3_cx(i) == -1) obuf[row * 5 + q3_west(i)] = lat[lat3<L>(q3_opp(i), n, p.g.P)];
}

// ------------------------------------------------------------------ readouts
template <int S, int L, class T> __global__ void k3_get_pop(KParams3 p, const T* __restrict__ lat, float* __restrict__ out)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = p.g.nx * p.g.ny * p.g.nz;
    if (m >= N) return;
    const int64_t x = m % p.g.nx, yz = m / p.g.nx, y = yz % p.g.ny, z = yz / p.g.ny;
    const int64_t n = yz * p.g.px + x;
    const uint8_t t = p.types[n];
    const bool upd = updated(t), inlet = node_type(t) == T_INLET;
    float f[Q3];
    gather_state3<L, S>(p, lat, x, y, z, upd ? n : 0, f); // in-bounds for every node
#pragma unroll
    for (int i = 0; i < Q3; ++i) out[i * N + m] = upd ? f[i] : (inlet ? inlet3(p, i) : 0.0f);
}

template <int S, int L, class T>
__global__ void k3_macros(KParams3 p, const T* __restrict__ lat, float* __restrict__ rho, float* __restrict__ u)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = p.g.nx * p.g.ny * p.g.nz;
    if (m >= N) return;
    const int64_t x = m % p.g.nx, yz = m / p.g.nx, y = yz % p.g.ny, z = yz / p.g.ny;
    const int64_t n = yz * p.g.px + x;
    const uint8_t t = p.types[n];
    float r = 0.0f, j[3] = {0.0f, 0.0f, 0.0f};
    if (updated(t)) {
        float f[Q3];
        gather_state3<L, S>(p, lat, x, y, z, n, f);
        float rt;
        moments3(f, rt, j[0], j[1], j[2]);
        r = 1.0f + rt;
        for (int a = 0; a < 3; ++a) j[a] += p.ph.hg[a];
    } else if (node_type(t) == T_INLET) {
        r = 1.0f;
        for (int a = 0; a < 3; ++a) j[a] = p.ph.u_in[a];
    }
    if (rho) rho[m] = r;
    if (u)
        for (int a = 0; a < 3; ++a) u[a * N + m] = j[a];
}

// ------------------------------------------------------------------ diagnostics
// FP64 mass, momentum (3) and the residual terms of the velocity change,
// summed per block in a fixed order, then over blocks (deterministic).
constexpr int DIAG3_BLOCKS = 1024;
constexpr int DIAG3_THREADS = 256;
constexpr int DIAG3_VALUES = 6;

__device__ __forceinline__ double block_sum3(double v, double* sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int w = DIAG3_THREADS / 2; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// part[block][k]: k = 0 mass, 1..3 momentum, 4 sum |u - u_prev|^2, 5 sum |u|^2;
// u_prev (3 doubles per padded node) is read when have_prev and overwritten.
template <int S, int L, class T>
__global__ void __launch_bounds__(DIAG3_THREADS)
    k3_diag(KParams3 p, const T* __restrict__ lat, double* __restrict__ u_prev, int have_prev, double* __restrict__ part)
{
    __shared__ double sh[DIAG3_THREADS];
    const int64_t N = p.g.nx * p.g.ny * p.g.nz;
    double acc[DIAG3_VALUES] = {0, 0, 0, 0, 0, 0};
    for (int64_t m = (int64_t)blockIdx.x * DIAG3_THREADS + threadIdx.x; m < N;
         m += (int64_t)DIAG3_BLOCKS * DIAG3_THREADS) {
        const int64_t x = m % p.g.nx, yz = m / p.g.nx, y = yz % p.g.ny, z = yz / p.g.ny;
        const int64_t n = yz * p.g.px + x;
        if (!updated(p.types[n])) continue;
        float f[Q3];
        gather_state3<L, S>(p, lat, x, y, z, n, f);
        double r = 1.0, j[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < Q3; ++i) {
            const double v = (double)f[i];
            r += v;
            j[0] += q3_cx(i) * v;
            j[1] += q3_cy(i) * v;
            j[2] += q3_cz(i) * v;
        }
        acc[0] += r;
        double du = 0.0, uu = 0.0;
        for (int a = 0; a < 3; ++a) {
            acc[1 + a] += j[a];
            const double u = j[a] + (double)p.ph.hg[a];
            if (have_prev) du += (u - u_prev[3 * n + a]) * (u - u_prev[3 * n + a]);
            uu += u * u;
            u_prev[3 * n + a] = u;
        }
        acc[4] += du;
        acc[5] += uu;
    }
    for (int k = 0; k < DIAG3_VALUES; ++k) {
        const double t = block_sum3(acc[k], sh);
        if (threadIdx.x == 0) part[blockIdx.x * DIAG3_VALUES + k] = t;
    }
}

__global__ void __launch_bounds__(DIAG3_THREADS) k3_diag_final(const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double sh[DIAG3_THREADS];
    for (int k = 0; k < DIAG3_VALUES; ++k) {
        double a = 0.0;
        for (int b = threadIdx.x; b < DIAG3_BLOCKS; b += DIAG3_THREADS) a += part[b * DIAG3_VALUES + k];
        const double t = block_sum3(a, sh);
        if (threadIdx.x == 0) out[k] = t;
    }
}

int diag3_partials() { return DIAG3_BLOCKS * DIAG3_VALUES; }

// ------------------------------------------------------------------ launchers
// Calls fn(IC<state>, IC<layout>, Tag<storage>) for the runtime triple
// (layouts stream, collision and blocked).
template <class Fn> static hipError_t dispatch3(int state, int layout, int prec, Fn&& fn)
{
    auto by_state = [&](auto L) -> hipError_t {
        return with_storage(prec, [&](auto TT) -> hipError_t {
            if (state == ST_PULL) return fn(IC<ST_PULL>{}, L, TT);
            if (state == ST_PUSH) return fn(IC<ST_PUSH>{}, L, TT);
            if (state == ST_SWAP) return fn(IC<ST_SWAP>{}, L, TT);
            return hipErrorInvalidValue;
        });
    };
    if (layout == L_STREAM) return by_state(IC<L_STREAM>{});
    if (layout == L_COLLISION) return by_state(IC<L_COLLISION>{});
    if (layout == L_BLOCKED) return by_state(IC<L_BLOCKED>{});
    return hipErrorInvalidValue;
}

static dim3 grid3(const Geometry3& g) { return dim3((uint32_t)((int64_t)g.ntx * g.nty * g.nz)); }

hipError_t launch3_types(const Geometry3& g, const uint8_t* flags, uint8_t* types, hipStream_t s)
{
    hipLaunchKernelGGL(k3_types, dim3(blocks3(g.plane * g.nz, 256)), dim3(256), 0, s, g, flags, types);
    return hipGetLastError();
}

hipError_t launch3_init(int state, int layout, int prec, const KParams3& p, void* lat, hipStream_t s)
{
    return dispatch3(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k3_init<decltype(S)::value, decltype(L)::value, T>),
                           dim3(blocks3(p.g.plane * p.g.nz, 256)), dim3(256), 0, s, p, (T*)lat);
        return hipGetLastError();
    });
}

hipError_t launch3_set_state(int state, int layout, int prec, const KParams3& p, const float* f, void* lat, void* tmp,
                             hipStream_t s)
{
    return dispatch3(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        constexpr int SV = decltype(S)::value, LV = decltype(L)::value;
        const uint32_t nb = blocks3(p.g.nx * p.g.ny * p.g.nz, 256);
        if constexpr (SV == ST_PUSH) {
            if (!tmp) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k3_set_post<ST_PULL, LV, T>), dim3(nb), dim3(256), 0, s, p, f, (T*)tmp);
            hipLaunchKernelGGL((k3_pull_to_push<LV, T>), dim3(blocks3(p.g.plane * p.g.nz, 256)), dim3(256), 0, s, p,
                               (const T*)tmp, (T*)lat);
        } else {
            hipLaunchKernelGGL((k3_set_post<SV, LV, T>), dim3(nb), dim3(256), 0, s, p, f, (T*)lat);
        }
        return hipGetLastError();
    });
}

hipError_t launch3_update(int scheme, int layout, int prec, const KParams3& p, int parity, const void* src, void* dst,
                          void* obuf, hipStream_t s)
{
    return dispatch3(ST_PULL, layout, prec, [&](auto, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        constexpr int LV = decltype(L)::value;
        const dim3 blk(p.g.tx, p.g.ty);
        if constexpr (LV == L_COLLISION) {
            if (aos3_staged(p.g.px, p.g.ny, p.g.tx, p.g.ty)) { // whole records staged through LDS
                const size_t sh = Aos3<T>::bytes(p.g.ty);
                if (scheme != S_AA) {
                    if constexpr (sizeof(T) == 4) {
                        const int zb = aos3_zb(p.g);
                        const uint32_t nb = (uint32_t)((int64_t)p.g.ntx * p.g.nty * ((p.g.nz + zb - 1) / zb));
                        hipLaunchKernelGGL((k3_pull_aos_z<T>), dim3(nb), blk, sh, s, p, (const T*)src, (T*)dst, zb);
                    } else {
                        hipLaunchKernelGGL((k3_pull_aos<T>), grid3(p.g), blk, sh, s, p, (const T*)src, (T*)dst);
                    }
                } else if (parity == 0)
                    hipLaunchKernelGGL((k3_aa_even_aos<T>), grid3(p.g), blk, sh, s, p, (T*)dst, (T*)obuf);
                else
                    hipLaunchKernelGGL((k3_aa_odd_aos<T>), grid3(p.g), blk, sh + (size_t)(p.g.ty + 2) * Aos3<T>::SEG, s,
                                       p, (T*)dst, (const T*)obuf);
                return hipGetLastError();
            }
        }
        if (scheme == S_AA) {
            if (parity == 0)
                hipLaunchKernelGGL((k3_aa_even<LV, T>), grid3(p.g), blk, 0, s, p, (T*)dst, (T*)obuf);
            else
                hipLaunchKernelGGL((k3_aa_odd<LV, T>), grid3(p.g), blk, 0, s, p, (T*)dst, (const T*)obuf);
        } else {
            hipLaunchKernelGGL((k3_pull<LV, T>), grid3(p.g), blk, 0, s, p, (const T*)src, (T*)dst);
        }
        return hipGetLastError();
    });
}

hipError_t launch3_aa_outlet_fill(int layout, int prec, const KParams3& p, const void* lat, void* obuf, hipStream_t s)
{
    return dispatch3(ST_SWAP, layout, prec, [&](auto, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k3_aa_outlet_fill<decltype(L)::value, T>), dim3(blocks3(p.g.ny * p.g.nz, 256)), dim3(256),
                           0, s, p, (const T*)lat, (T*)obuf);
        return hipGetLastError();
    });
}

hipError_t launch3_get_populations(int state, int layout, int prec, const KParams3& p, const void* lat, float* f,
                                   hipStream_t s)
{
    return dispatch3(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k3_get_pop<decltype(S)::value, decltype(L)::value, T>),
                           dim3(blocks3(p.g.nx * p.g.ny * p.g.nz, 256)), dim3(256), 0, s, p, (const T*)lat, f);
        return hipGetLastError();
    });
}

hipError_t launch3_diag(int state, int layout, int prec, const KParams3& p, const void* lat, double* u_prev,
                        int have_prev, double* partials, double* out, hipStream_t s)
{
    return dispatch3(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k3_diag<decltype(S)::value, decltype(L)::value, T>), dim3(DIAG3_BLOCKS),
                           dim3(DIAG3_THREADS), 0, s, p, (const T*)lat, u_prev, have_prev, partials);
        hipLaunchKernelGGL(k3_diag_final, dim3(1), dim3(DIAG3_THREADS), 0, s, (const double*)partials, out);
        return hipGetLastError();
    });
}

hipError_t launch3_macros(int state, int layout, int prec, const KParams3& p, const void* lat, float* rho, float* u,
                          hipStream_t s)
{
    return dispatch3(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k3_macros<decltype(S)::value, decltype(L)::value, T>),
                           dim3(blocks3(p.g.nx * p.g.ny * p.g.nz, 256)), dim3(256), 0, s, p, (const T*)lat, rho, u);
        return hipGetLastError();
    });
}

} // namespace lbm
