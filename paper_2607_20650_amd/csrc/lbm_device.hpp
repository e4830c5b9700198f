// lbm_device.hpp -- device building blocks shared by every update kernel:
// layout addressing (paper Section 3.2), the storage codec, the boundary
// classification of pull sources (Section 3.1, last paragraph) and the single
// BGK collision routine (Eq. 1-2).  Every scheme calls the same collide(), so
// all schemes and layouts of one precision give bitwise identical results.
#pragma once

#include <type_traits>
#include <utility>

#include "lbm_common.hpp"

namespace lbm {

// ------------------------------------------------------------------ dispatch
template <int V> using IC = std::integral_constant<int, V>;
template <class T> struct Tag { using type = T; };

// Storage type of each precision: the raw 16-bit codes of the formats with
// their own encoding each get a distinct scalar type.
//   FP32 float, FP16S _Float16, FP16S-SR uint16_t, FP16C int16_t, FP16C-SR char16_t
// Calls fn(Tag<storage>) for a runtime precision.
template <class Fn>
hipError_t with_storage(int prec, Fn&& fn)
{
    if (prec == P_FP32) return fn(Tag<float>{});
    if (prec == P_FP16S) return fn(Tag<_Float16>{});
    if (prec == P_FP16SR) return fn(Tag<uint16_t>{});
    if (prec == P_FP16C) return fn(Tag<int16_t>{});
    if (prec == P_FP16CSR) return fn(Tag<char16_t>{});
    return hipErrorInvalidValue;
}

// Calls fn(IC<layout>, Tag<storage>) for a runtime D2Q9 layout and precision.
template <class Fn>
hipError_t with_layout_storage(int layout, int prec, Fn&& fn)
{
    auto by_prec = [&](auto L) -> hipError_t { return with_storage(prec, [&](auto TT) { return fn(L, TT); }); };
    if (layout == L_STREAM) return by_prec(IC<L_STREAM>{});
    if (layout == L_BUNDLE) return by_prec(IC<L_BUNDLE>{});
    if (layout == L_COLLISION) return by_prec(IC<L_COLLISION>{});
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ layouts
// stream (SoA):        i * P + n
// bundle (SoAoS):      (i / 3) * 3P + 3 n + (i % 3)    (bundle = c_y + 1)
// collision (AoS):     9 n + i
template <int L>
__device__ __forceinline__ int64_t lat_at(int i, int64_t n, int64_t P)
{
    if constexpr (L == L_STREAM)
        return (int64_t)i * P + n;
    else if constexpr (L == L_BUNDLE)
        return (int64_t)(i / 3) * 3 * P + 3 * n + (i % 3);
    else
        return 9 * n + i;
}

// The same layouts split as  plane(i) + S * n + lane(i):  a per-direction
// base, a node stride S common to all directions, and a constant.
template <int L> constexpr int lat_stride() { return L == L_STREAM ? 1 : (L == L_BUNDLE ? 3 : 9); }
template <int L> constexpr int lat_lane(int i) { return L == L_STREAM ? 0 : (L == L_BUNDLE ? i % 3 : i); }
template <int L>
__device__ __forceinline__ int64_t lat_plane(int i, int64_t P)
{
    if constexpr (L == L_STREAM)
        return (int64_t)i * P;
    else if constexpr (L == L_BUNDLE)
        return (int64_t)(i / 3) * 3 * P;
    else
        return 0;
}

// Element at a 32-bit byte offset from a base pointer.  With the base uniform
// across the wavefront it stays in scalar registers and the offset takes one
// vector register: the scalar-base form of the global memory instructions.
template <class T> __device__ __forceinline__ const T& at_byte(const T* base, uint32_t off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <class T> __device__ __forceinline__ T& at_byte(T* base, uint32_t off)
{
    return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}

// ------------------------------------------------------------------ codec
// FP32 stores the shifted population as is; FP16S rounds it to binary16 with
// round-to-nearest-even and widens exactly on load (subnormals preserved).
__device__ __forceinline__ float ld(float v) { return v; }
__device__ __forceinline__ float ld(_Float16 v) { return (float)v; }
template <class T> __device__ __forceinline__ T st(float v);
template <> __device__ __forceinline__ float st<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 st<_Float16>(float v) { return (_Float16)v; }

// FP16S-SR: binary16 kept as raw bits (a distinct storage type); loads widen
// exactly, st<> rounds to nearest even, enc<> rounds stochastically.
__device__ __forceinline__ float ld(uint16_t v) { return (float)__builtin_bit_cast(_Float16, v); }
template <> __device__ __forceinline__ uint16_t st<uint16_t>(float v)
{
    return __builtin_bit_cast(uint16_t, (_Float16)v);
}

// FP16C: a custom 16-bit float for shifted populations, whose magnitudes stay
// below 1, trading binary16's unused top exponents for one more fraction bit:
// sign, 4 exponent bits e, 11 fraction bits m, bias 15.  Normal codes
// (e = 1..15) are 2^(e-15) (1 + m / 2^11), covering [2^-14, 2); subnormal
// codes (e = 0) are m 2^-25.  The top code 0x7fff (either sign) is NaN, and
// is what NaN, infinities and values that round to it encode to, so a run
// that blows up still ends in non-finite values.  The 15 low bits of a code
// are the bits of the FP32 number v 2^-112 shifted right by 12 (its exponent
// field is then e, or 0 below 2^-14), so:
//   decode: place the code 12 bits up, multiply by 2^112 (exact);
//   encode: scale by 2^-112 (exact above 2^-14; below it the FP32 subnormal
//           keeps 12 more bits than the code, rounded to nearest even), then
//           drop 12 bits with round-to-nearest-even (FP16C) or by adding 12
//           random bits (FP16C-SR, stochastic rounding); carries move into
//           the exponent as they should.
// Storage types: int16_t (FP16C) and char16_t (FP16C-SR) hold the raw codes.
// The top magnitude code scaled: FP32 bits 0x07fff000, 2 - 2^-11 after decoding.
constexpr float C16_TOP = 0x1.ffep-112f;

// h: the code sign-extended to 32 bits (what a signed 16-bit load yields).
// The extension fills bits 27..31, so one mask keeps the sign at bit 31 and
// the 15 magnitude bits at 12..26.
__device__ __forceinline__ float c16_decode(int32_t h)
{
    const float v = __builtin_bit_cast(float, ((uint32_t)h << 12) & 0x87fff000u) * 0x1p112f;
    return __builtin_fabsf(v) == 0x1.ffep0f ? __builtin_nanf("") : v;
}
// |v| 2^-112 as FP32 bits, clamped to the scaled top code: NaN (the minimum
// of a quiet NaN and a number is the number), infinities and everything that
// would round past the top code end in it, as every other magnitude rounds
// to at most it.
__device__ __forceinline__ uint32_t c16_scaled(float v)
{
    return __builtin_bit_cast(uint32_t, __builtin_fminf(__builtin_fabsf(v) * 0x1p-112f, C16_TOP));
}
// The code of v from a = c16_scaled(v) and rnd, the increment added below the
// 12 dropped bits (< 2^12).  The rounded magnitude is below 2^27, so shifted 4
// up its code bits land in 16..30 with the sign of v at 31: the code is the
// high half, which a 16-bit store takes without a further shift.
__device__ __forceinline__ uint16_t c16_pack(float v, uint32_t a, uint32_t rnd)
{
    return (uint16_t)((((a + rnd) << 4) | (__builtin_bit_cast(uint32_t, v) & 0x80000000u)) >> 16);
}
__device__ __forceinline__ uint16_t c16_encode(float v, uint32_t rnd) { return c16_pack(v, c16_scaled(v), rnd); }
__device__ __forceinline__ uint16_t c16_rne(float v)
{
    const uint32_t a = c16_scaled(v);
    return c16_pack(v, a, 0x7ff + ((a >> 12) & 1));
}

__device__ __forceinline__ float ld(int16_t v) { return c16_decode(v); }
__device__ __forceinline__ float ld(char16_t v) { return c16_decode((int16_t)v); }
template <> __device__ __forceinline__ int16_t st<int16_t>(float v) { return (int16_t)c16_rne(v); }
template <> __device__ __forceinline__ char16_t st<char16_t>(float v) { return (char16_t)c16_rne(v); }

// 32-bit integer mixing function "lowbias32" (C. Wellons, hash prospector).
__device__ __forceinline__ uint32_t mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

// Marsaglia's xorshift32 step.
__device__ __forceinline__ uint32_t xorshift32(uint32_t h)
{
    h ^= h << 13;
    h ^= h >> 17;
    h ^= h << 5;
    return h;
}

// Random bits for the stores of one node's post-collision values (used by
// the stochastically rounded formats, FP16S-SR and FP16C-SR), for Q
// directions.  One strong hash per node of its index and of the FP32 bits of
// three of its post-collision values (f*_0, f*_(Q/2), f*_(Q-1), folded by
// xor-rotate), stretched by xorshift to the 13 Q bits the draws need.  The
// draws change whenever the node's state changes, are independent of the bits
// a rounding drops (avalanche of the hash), and depend only on the node and
// its values, so every scheme rounds f*_i of a node identically, wherever the
// value lands.
template <int Q> struct NodeBits {
    static constexpr int NW = (13 * Q + 31) / 32; // words covering Q 13-bit fields
    uint32_t w[NW] = {};
    __device__ __forceinline__ NodeBits() {}
    __device__ __forceinline__ NodeBits(uint32_t node, const float* f)
    {
        const uint32_t b0 = __builtin_bit_cast(uint32_t, f[0]);
        const uint32_t b4 = __builtin_bit_cast(uint32_t, f[Q / 2]);
        const uint32_t b8 = __builtin_bit_cast(uint32_t, f[Q - 1]);
        w[0] = mix32(node ^ b0 ^ __builtin_amdgcn_alignbit(b4, b4, 21) ^ __builtin_amdgcn_alignbit(b8, b8, 10));
#pragma unroll
        for (int k = 1; k < NW; ++k) w[k] = xorshift32(w[k - 1]);
    }
    // 32 random bits for direction i, a window of the stream whose 13 high
    // bits are bits [13 i, 13 i + 13): disjoint between directions.  The
    // rounding reads the high bits first; in the binary16 normal range it
    // needs exactly those 13 (the bits an FP32 value loses; FP16C takes 12),
    // so the roundings of a node are independent.  With fewer fresh bits the
    // probability of rounding up would be quantised below the dropped
    // fraction, a bias toward zero that accumulates over thousands of updates.
    __device__ __forceinline__ uint32_t draw(int i) const
    {
        const int a = 13 * i - 19; // first bit of the window
        if (a < 0) return w[0] << -a;
        const int k = a >> 5, s = a & 31;
        return s == 0 ? w[k] : __builtin_amdgcn_alignbit(w[k + 1], w[k], s);
    }
};
template <class T, int Q = 9> struct NodeRng {
    __device__ __forceinline__ NodeRng() {}
    __device__ __forceinline__ NodeRng(uint32_t, const float*) {}
    __device__ __forceinline__ uint32_t draw(int) const { return 0; }
};
// the two stochastically rounded storage types draw the same bits
template <int Q> struct NodeRng<uint16_t, Q> : NodeBits<Q> {
    __device__ __forceinline__ NodeRng() {}
    __device__ __forceinline__ NodeRng(uint32_t node, const float* f) : NodeBits<Q>(node, f) {}
};
template <int Q> struct NodeRng<char16_t, Q> : NodeBits<Q> {
    __device__ __forceinline__ NodeRng() {}
    __device__ __forceinline__ NodeRng(uint32_t node, const float* f) : NodeBits<Q>(node, f) {}
};

// Encoding of a freshly computed post-collision value for storage.  FP32 and
// FP16S: as st<>.  FP16S-SR: the gfx950 conversion with stochastic rounding
// takes the binary16 neighbour of larger magnitude with probability equal to
// v's position between its two binary16 neighbours (binary16 subnormals
// included), decided by the high bits of r, so with uniform r the expected
// stored value is v.  Values representable in binary16 are kept exactly.
template <class T> __device__ __forceinline__ T enc(float v, uint32_t r)
{
    (void)r;
    return st<T>(v);
}
template <> __device__ __forceinline__ uint16_t enc<uint16_t>(float v, uint32_t r)
{
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    // the instruction writes the low half only; the high half passed through
    // (r's, unused) saves initialising a register
    const half2_t h = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2_t, r), v, r, false);
    return __builtin_bit_cast(uint16_t, h[0]);
}
// FP16C-SR: the 12 high bits of r added below the dropped bits round up with
// probability equal to the dropped fraction.
template <> __device__ __forceinline__ char16_t enc<char16_t>(float v, uint32_t r)
{
    return (char16_t)c16_encode(v, r >> 20);
}

// ------------------------------------------------------------------ vectors
// VX consecutive populations moved as one wide access.  Aligned accesses use
// the natural vector alignment; shifted ones (a +-1 node offset) only the
// element alignment, which the unaligned-access mode of gfx9 serves with the
// same wide instruction.
template <class T, int VX, bool ALIGNED>
__device__ __forceinline__ void vload(const T* __restrict__ p, float* out)
{
    if constexpr (VX == 1) {
        out[0] = ld(p[0]);
    } else {
        typedef T V __attribute__((ext_vector_type(VX), aligned(ALIGNED ? VX * sizeof(T) : sizeof(T))));
        const V v = *reinterpret_cast<const V*>(p);
#pragma unroll
        for (int k = 0; k < VX; ++k) out[k] = ld(v[k]);
    }
}

// VX already-encoded values stored as one wide access (natural alignment).
template <class T, int VX>
__device__ __forceinline__ void vstore_t(T* __restrict__ p, const T* in)
{
    if constexpr (VX == 1) {
        p[0] = in[0];
    } else {
        typedef T V __attribute__((ext_vector_type(VX), aligned(VX * sizeof(T))));
        V v;
#pragma unroll
        for (int k = 0; k < VX; ++k) v[k] = in[k];
        *reinterpret_cast<V*>(p) = v;
    }
}

// A run of NE contiguous elements whose start is a multiple of the run size
// in bytes, moved in the widest pieces (<= 16 bytes) that divide the run.
template <class T, int NE> constexpr int run_chunk()
{
    constexpr int bytes = NE * (int)sizeof(T);
    return (bytes % 16 == 0 ? 16 : bytes % 8 == 0 ? 8 : bytes % 4 == 0 ? 4 : (int)sizeof(T)) / (int)sizeof(T);
}

template <class T, int NE>
__device__ __forceinline__ void vload_run(const T* __restrict__ p, float* out)
{
    constexpr int C = run_chunk<T, NE>();
#pragma unroll
    for (int k = 0; k < NE; k += C) vload<T, C, true>(p + k, out + k);
}

template <class T, int NE>
__device__ __forceinline__ void vstore_run_t(T* __restrict__ p, const T* in)
{
    constexpr int C = run_chunk<T, NE>();
#pragma unroll
    for (int k = 0; k < NE; k += C) vstore_t<T, C>(p + k, in + k);
}

// ------------------------------------------------------------------ collision
// Weights of Eq. 2 and the first-moment constants t_i = 3 w_i.  t_axis is the
// float nearest 1/3 and t_diag = (1 - 2 t_axis) / 4 (exact), so that
// 2 t_axis + 4 t_diag == 1 exactly and the equilibrium carries the momentum j
// without a systematic rounding drift.
constexpr float W_REST = 4.0f / 9.0f;
constexpr float W_AXIS = 1.0f / 9.0f;
constexpr float W_DIAG = 1.0f / 36.0f;
constexpr float T_AXIS = 1.0f / 3.0f;
constexpr float T_DIAG = (1.0f - 2.0f * T_AXIS) / 4.0f;
// 9/2 w_i: exact in binary32 for both link kinds
constexpr float H_AXIS = 0.5f;
constexpr float H_DIAG = 0.125f;

template <int I>
__device__ __forceinline__ float c_dot(float jx, float jy)
{
    constexpr int X = dir_cx(I), Y = dir_cy(I);
    if constexpr (X == 0 && Y == 0)
        return 0.0f;
    else if constexpr (X == 0)
        return Y > 0 ? jy : -jy;
    else if constexpr (Y == 0)
        return X > 0 ? jx : -jx;
    else
        return (X > 0 ? jx : -jx) + (Y > 0 ? jy : -jy);
}

template <int I>
__device__ __forceinline__ float feq_shifted(float base, float jx, float jy)
{
    constexpr int X = dir_cx(I), Y = dir_cy(I);
    if constexpr (X == 0 && Y == 0) {
        return W_REST * base;
    } else if constexpr (X == 0 || Y == 0) {
        const float cu = c_dot<I>(jx, jy);
        return __builtin_fmaf(W_AXIS, base, cu * __builtin_fmaf(H_AXIS, cu, T_AXIS));
    } else {
        const float cu = c_dot<I>(jx, jy);
        return __builtin_fmaf(W_DIAG, base, cu * __builtin_fmaf(H_DIAG, cu, T_DIAG));
    }
}

template <int I>
__device__ __forceinline__ void relax_one(float* f, float base, float jx, float jy, float omc, const float* F)
{
    const float e = feq_shifted<I>(base, jx, jy);
    f[I] = e + __builtin_fmaf(omc, f[I] - e, F[I]);
}

// In: shifted incoming populations f~_in.  Out: shifted post-collision f~*.
//   rho~ = sum f~, j = sum f~ c,  feq~_i = w_i (rho~ - 3/2 j.j) + 9/2 w_i (c_i.j)^2 + t_i c_i.j
//   f~*_i = feq~_i + [ (1 - 1/tau)(f~_i - feq~_i) + F_i ]
__device__ __forceinline__ void collide(float* f, float omc, const float* F)
{
    const float rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const float jx = ((f[2] + f[5]) + f[8]) - ((f[0] + f[3]) + f[6]);
    const float jy = ((f[6] + f[7]) + f[8]) - ((f[0] + f[1]) + f[2]);
    const float jj = __builtin_fmaf(jx, jx, jy * jy);
    const float base = __builtin_fmaf(-1.5f, jj, rho);
    relax_one<0>(f, base, jx, jy, omc, F);
    relax_one<1>(f, base, jx, jy, omc, F);
    relax_one<2>(f, base, jx, jy, omc, F);
    relax_one<3>(f, base, jx, jy, omc, F);
    relax_one<4>(f, base, jx, jy, omc, F);
    relax_one<5>(f, base, jx, jy, omc, F);
    relax_one<6>(f, base, jx, jy, omc, F);
    relax_one<7>(f, base, jx, jy, omc, F);
    relax_one<8>(f, base, jx, jy, omc, F);
}

// Moments used by the readouts, summed in the same order as collide().
__device__ __forceinline__ void moments(const float* f, float& rho, float& jx, float& jy)
{
    rho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    jx = ((f[2] + f[5]) + f[8]) - ((f[0] + f[3]) + f[6]);
    jy = ((f[6] + f[7]) + f[8]) - ((f[0] + f[1]) + f[2]);
}

// ------------------------------------------------------------------ sources
enum SrcKind : int { K_NODE = 0, K_SOLID = 1, K_INLET = 2 };

// A node-type byte carries the NodeType in its low bits and, in bit 7, the
// IRREGULAR mark: set when the node or one of its 8 neighbours is not a plain
// fluid node, or the node lies on the domain border.  Nodes without the mark
// stream with fixed offsets and no boundary rule.
constexpr uint8_t TYPE_MASK = 0x7f;
constexpr uint8_t IRREGULAR = 0x80;

__device__ __forceinline__ uint8_t node_type(uint8_t t) { return t & TYPE_MASK; }
__device__ __forceinline__ bool updated(uint8_t t)
{
    const uint8_t k = node_type(t);
    return k == T_FLUID || k == T_OUTLET;
}

// The inlet equilibrium of direction i as a wavefront-uniform register value.
// Choosing between it and a loaded population by value keeps the compiler
// from turning the choice into a choice of addresses, which would copy the
// kernel argument to scratch and load through a flat pointer.
__device__ __forceinline__ float inlet_value(const KParams& p, int i)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, p.ph.ein[i])));
}

// Pull source of direction i for node (x, y): the node (x, y) - c_i after the
// axis rules.  Periodic axes wrap; outside a closed side counts as solid; past
// the outlet of an inflow/outflow x axis the last column is used (zero
// gradient, applied after the y shift).  Returns the kind of the source and,
// for K_NODE, its padded node index in sn.
__device__ __forceinline__ int pull_source(const Geometry& g, const uint8_t* __restrict__ types, int64_t x,
                                           int64_t y, int i, int64_t& sn, bool fullway = false)
{
    int64_t sx = x - dir_cx(i);
    int64_t sy = y - dir_cy(i);
    if (sy < 0 || sy >= g.ny) {
        if (g.ya != AX_PERIODIC) return K_SOLID;
        sy = sy < 0 ? sy + g.ny : sy - g.ny;
    }
    if (sx < 0 || sx >= g.nx) {
        if (g.xa == AX_PERIODIC)
            sx = sx < 0 ? sx + g.nx : sx - g.nx;
        else if (g.xa == AX_INOUT && sx >= g.nx)
            sx = g.nx - 1;
        else
            return K_SOLID;
    }
    sn = sy * g.px + sx;
    const uint8_t t = node_type(types[sn]);
    // with full-way bounce-back a solid node is a source like any other
    return t == T_SOLID ? (fullway ? K_NODE : K_SOLID) : (t == T_INLET ? K_INLET : K_NODE);
}

// Slot that holds the post-collision value of direction i in a given state kind.
template <int S>
__device__ __forceinline__ int post_slot(int i)
{
    return S == ST_SWAP ? dir_opp(i) : i;
}

// Pressure outlet (the Zou-He condition Section 3.1 adapts, in the
// incompressible model's momentum form): at an outlet node the three incoming
// values with c_x = -1 (directions 0, 3, 6) are rebuilt from the six others so
// that the incoming density is rho0 = 1 and the tangential momentum zero, the
// normal non-equilibrium part bouncing back.  In shifted storage (f~ = f - w)
// the relations keep their form with j_x = K~, K~ being the three c_x = 0
// values plus twice the three c_x = +1 values.
__device__ __forceinline__ void outlet_fix(const Geometry& g, int64_t x, float* f)
{
    if (!g.zh || x != g.nx - 1) return;
    const float jx = ((f[1] + f[4]) + f[7]) + 2.0f * ((f[2] + f[5]) + f[8]);
    const float h = 0.5f * (f[1] - f[7]);
    const float d = jx * (1.0f / 6.0f);
    f[3] = f[5] - jx * (2.0f / 3.0f);
    f[6] = (f[2] + h) - d;
    f[0] = (f[8] - h) - d;
}

// Weight w_i of Eq. 2.
__device__ __forceinline__ constexpr float weight(int i)
{
    return i == 4 ? W_REST : ((dir_cx(i) == 0 || dir_cy(i) == 0) ? W_AXIS : W_DIAG);
}

// Neumann inlet (Section 3.1): the inlet node (0, s) holds feq(rho_in, u_in)
// with rho_in the density its neighbour (1, s) had after the previous update
// (p.rin[s] = rho_in - 1).  In shifted storage that is the Dirichlet value plus
// w_i (rho_in - 1).  Only column 1 pulls from the inlet, in the three
// directions with c_x = +1, from row s = y - c_y.
__device__ __forceinline__ void neumann_inlet(const KParams& p, int64_t x, int64_t y, float* f)
{
    if (p.rin == nullptr || x != 1) return;
    // a loop (not unrolled) keeps this rare path from raising the register
    // count of the kernels it is inlined into
#pragma unroll 1
    for (int i = 2; i < 9; i += 3) {
        int64_t s = y - dir_cy(i);
        if (s < 0 || s >= p.g.ny) {
            if (p.g.ya != AX_PERIODIC) continue;
            s = s < 0 ? s + p.g.ny : s - p.g.ny;
        }
        if (node_type(p.types[s * p.g.px]) == T_INLET) f[i] = f[i] + weight(i) * p.rin[s];
    }
}

// The inlet and outlet rules on the incoming populations of an updated node at
// (x, y), after its sources were read (inlet sources at the Dirichlet value).
__device__ __forceinline__ void boundary_fix(const KParams& p, int64_t x, int64_t y, float* f)
{
    neumann_inlet(p, x, y, f);
    outlet_fix(p.g, x, f);
}

// An update records rho - 1 of the column-1 node of row y (the sum of its
// incoming values, which collision and force conserve) for the next update's
// Neumann inlet.
__device__ __forceinline__ void record_inlet_density(const KParams& p, int64_t x, int64_t y, const float* f)
{
    if (p.rout == nullptr || x != 1) return;
    p.rout[y] = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
}

// Shifted inlet value of direction i at the inlet node of row y.
__device__ __forceinline__ float inlet_node_value(const KParams& p, int i, int64_t y)
{
    const float e = inlet_value(p, i);
    return p.rin == nullptr ? e : e + weight(i) * p.rin[y];
}

// Gather the incoming populations of an updated node from a pull-like state
// (ST_PULL or ST_SWAP) held in one lattice: the definition every scheme's
// streaming reproduces.  Every direction issues one load from a valid lattice
// address (the source, or the node itself for bounce-back and inlet sources)
// and the inlet value is chosen afterwards by value, so no private array is
// ever addressed through memory.  NEU = false leaves the Neumann inlet out (for
// kernels instantiated separately for the Dirichlet inlet).  FW: full-way
// bounce-back never (0), always (1), or as the geometry says (2, readouts).
template <int L, int S, class T, bool NEU = true, int FW = 0>
__device__ __forceinline__ void gather_pull(const KParams& p, const T* __restrict__ lat, int64_t x, int64_t y,
                                            int64_t n, float* f)
{
    const bool fullway = FW == 1 || (FW == 2 && p.g.fw);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int64_t sn = n;
        const int k = pull_source(p.g, p.types, x, y, i, sn, fullway);
        const int64_t at = k == K_NODE ? lat_at<L>(post_slot<S>(i), sn, p.g.P)
                                       : lat_at<L>(post_slot<S>(dir_opp(i)), n, p.g.P);
        const float v = ld(lat[at]);
        f[i] = k == K_INLET ? p.ph.ein[i] : v;
    }
    if constexpr (NEU) neumann_inlet(p, x, y, f);
    outlet_fix(p.g, x, f);
}

// gather_pull from a pull-like state for a node with link word lk (no source
// across a periodic side): the kinds come from the word, so no neighbour type
// is read.  Same loads and values as gather_pull.
template <int L, int S, class T, bool NEU = true>
__device__ __forceinline__ void gather_linked(const KParams& p, const T* __restrict__ lat, int64_t x, int64_t y,
                                              int64_t n, uint32_t lk, float* f)
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const uint32_t k = (lk >> (2 * i)) & 3u;
        const int64_t sn = n - (k == LINK_CLAMP ? 0 : dir_cx(i)) - dir_cy(i) * p.g.px;
        const int64_t at = k == LINK_SOLID ? lat_at<L>(post_slot<S>(dir_opp(i)), n, p.g.P)
                                           : lat_at<L>(post_slot<S>(i), sn, p.g.P);
        const float v = ld(lat[at]);
        f[i] = k == LINK_INLET ? p.ph.ein[i] : v;
    }
    if constexpr (NEU) neumann_inlet(p, x, y, f);
    outlet_fix(p.g, x, f);
}

// Incoming populations of an updated node held in a push state: its own slots,
// except slots fed by an inlet, which take the inlet equilibrium.
template <int L, class T>
__device__ __forceinline__ void gather_push(const KParams& p, const T* __restrict__ lat, int64_t x, int64_t y,
                                            int64_t n, float* f)
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        int64_t sn = n;
        const int k = pull_source(p.g, p.types, x, y, i, sn);
        const float v = ld(lat[lat_at<L>(i, n, p.g.P)]);
        f[i] = k == K_INLET ? inlet_value(p, i) : v;
    }
    boundary_fix(p, x, y, f);
}

// The kind pull_source would return for direction i of a node with link word
// lk (no source across a periodic side), and that source's coordinates.
__device__ __forceinline__ int linked_source(uint32_t lk, int i, int x, int y, int& sx, int& sy)
{
    const uint32_t k = (lk >> (2 * i)) & 3u;
    sx = x - (k == LINK_CLAMP ? 0 : dir_cx(i));
    sy = y - dir_cy(i);
    return k == LINK_SOLID ? K_SOLID : (k == LINK_INLET ? K_INLET : K_NODE);
}

// gather_push for a node with link word lk (no source across a periodic
// side): inlet-fed slots from the word, no neighbour type read.
template <int L, class T>
__device__ __forceinline__ void gather_push_linked(const KParams& p, const T* __restrict__ lat, int64_t x, int64_t y,
                                                   int64_t n, uint32_t lk, float* f)
{
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const float v = ld(lat[lat_at<L>(i, n, p.g.P)]);
        f[i] = ((lk >> (2 * i)) & 3u) == LINK_INLET ? inlet_value(p, i) : v;
    }
    boundary_fix(p, x, y, f);
}

// Incoming populations of an updated node for any state kind.
template <int L, int S, class T>
__device__ __forceinline__ void gather_state(const KParams& p, const T* __restrict__ lat, int64_t x, int64_t y,
                                             int64_t n, float* f)
{
    if constexpr (S == ST_PUSH)
        gather_push<L>(p, lat, x, y, n, f);
    else
        gather_pull<L, S, T, true, 2>(p, lat, x, y, n, f);
}

// ------------------------------------------------------ LDS staging copies
// Copy `total` 16-byte pieces from global memory into LDS, all threads of the
// block taking part: piece k goes from global element e to LDS element o,
// which piece(k, e, o) fills in, returning false for a piece that is not
// copied.  Each thread issues the loads of up to CHUNK pieces before it
// writes any of them, so CHUNK requests per thread are in flight instead of
// one (a loop that writes each piece as it arrives waits a full memory round
// trip per piece).  Loads and LDS writes are unconditional (so the compiler
// cannot sink a load into a conditional write): a piece that is not copied loads from g itself (a valid
// address) and goes to the 16-byte LDS slot at element `dummy`, which nothing
// reads.
template <int CHUNK, class T, class F>
__device__ __forceinline__ void pieces_to_lds(const T* __restrict__ g, T* s, int total, int dummy, int tid, int nthr,
                                              F&& piece)
{
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    for (int base = 0; base < total; base += CHUNK * nthr) {
        u32x4 v[CHUNK];
        int so[CHUNK];
        // slot j is in use when some thread of the block has a piece for it
        // (a block-uniform test): only the last slot in use has threads
        // without a piece
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            if (base + j * nthr >= total) break;
            const int k = base + j * nthr + tid;
            int64_t e = 0;
            int o = 0;
            const bool ok = k < total && piece(k, e, o);
            so[j] = ok ? o : dummy;
            v[j] = *reinterpret_cast<const u32x4*>(g + (ok ? e : 0));
        }
        // an empty asm that takes every loaded value once all loads are
        // issued: the optimiser can no longer fuse each load with its write
        // into a 16-byte copy (which waits for that load alone)
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            if (base + j * nthr >= total) break;
            asm volatile("" : "+v"(v[j]));
        }
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            if (base + j * nthr >= total) break;
            *reinterpret_cast<u32x4*>(s + so[j]) = v[j];
        }
    }
}

// The reverse: piece k goes from LDS element o to global element e.
template <int CHUNK, class T, class F>
__device__ __forceinline__ void pieces_from_lds(T* __restrict__ g, const T* s, int total, int tid, int nthr, F&& piece)
{
    for (int base = 0; base < total; base += CHUNK * nthr) {
        uint4 v[CHUNK];
        int64_t ge[CHUNK];
        bool ok[CHUNK];
#pragma unroll
        for (int j = 0; j < CHUNK; ++j) {
            const int k = base + j * nthr + tid;
            int64_t e = 0;
            int o = 0;
            ok[j] = k < total && piece(k, e, o);
            ge[j] = e;
            v[j] = *reinterpret_cast<const uint4*>(s + (ok[j] ? o : 0));
        }
#pragma unroll
        for (int j = 0; j < CHUNK; ++j)
            if (ok[j]) *reinterpret_cast<uint4*>(g + ge[j]) = v[j];
    }
}

} // namespace lbm
