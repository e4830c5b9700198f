// k_aux.hip -- kernels around the update: node types, initial state, state
// load, edge-buffer fill, population / macroscopic readout and the FP64
// diagnostic reductions.  All readouts reconstruct the incoming populations
// with the same gather the update kernels use.
#include <algorithm>
#include <type_traits>

#include "lbm_device.hpp"
#include "lbm_edges.hpp"
#include "lbm_kernels.hpp"

namespace lbm {

// Calls fn(IC<state>, IC<layout>, Tag<storage>) for the runtime triple.
template <class Fn>
static hipError_t dispatch(int state, int layout, int prec, Fn&& fn)
{
    return with_layout_storage(layout, prec, [&](auto L, auto TT) -> hipError_t {
        if (state == ST_PULL) return fn(IC<ST_PULL>{}, L, TT);
        if (state == ST_PUSH) return fn(IC<ST_PUSH>{}, L, TT);
        if (state == ST_SWAP) return fn(IC<ST_SWAP>{}, L, TT);
        return hipErrorInvalidValue;
    });
}

static inline uint32_t blocks_for(int64_t n, int b) { return (uint32_t)((n + b - 1) / b); }

// ---------------------------------------------------------------- node types
__device__ __forceinline__ uint8_t derive_type(const Geometry& g, const uint8_t* __restrict__ flags, int64_t x,
                                               int64_t y)
{
    if (x < 0 || y < 0 || x >= g.nx || y >= g.ny) return T_SOLID; // row padding / outside
    if (flags[y * g.nx + x] != 0) return T_SOLID;
    if (g.xa == AX_INOUT && x == 0) return T_INLET;
    if (g.xa == AX_INOUT && x == g.nx - 1) return T_OUTLET;
    return T_FLUID;
}

// Node types [ny][px] from user flags [ny][nx], with the IRREGULAR mark.
__global__ void k_types(Geometry g, const uint8_t* __restrict__ flags, uint8_t* __restrict__ types)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.px * g.ny) return;
    const int64_t y = m / g.px, x = m - y * g.px;
    const uint8_t t = derive_type(g, flags, x, y);
    bool irr = t != T_FLUID || x == 0 || y == 0 || x >= g.nx - 1 || y == g.ny - 1;
    for (int dy = -1; dy <= 1 && !irr; ++dy)
        for (int dx = -1; dx <= 1 && !irr; ++dx)
            if (derive_type(g, flags, x + dx, y + dy) != T_FLUID) irr = true;
    types[m] = (uint8_t)(t | (irr ? IRREGULAR : 0));
}

// Link words from the node types: for every node that updates (with full-way
// bounce-back, solid nodes too), the kind of each direction's pull source
// under the rules of pull_source, so that irregular nodes gather without
// looking up their neighbours' types.
__global__ void k_links(Geometry g, const uint8_t* __restrict__ types, uint32_t* __restrict__ links)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= g.px * g.ny) return;
    const int64_t y = m / g.px, x = m - y * g.px;
    uint32_t w = 0;
    if (x < g.nx) {
        for (int i = 0; i < 9; ++i) {
            const int64_t sx = x - dir_cx(i), sy = y - dir_cy(i);
            const bool wrap = ((sy < 0 || sy >= g.ny) && g.ya == AX_PERIODIC) ||
                              ((sx < 0 || sx >= g.nx) && g.xa == AX_PERIODIC);
            if (wrap) {
                w |= LINK_GENERAL;
                continue;
            }
            int64_t sn = 0;
            const int k = pull_source(g, types, x, y, i, sn, g.fw != 0);
            uint32_t kind = LINK_PLAIN;
            if (k == K_SOLID)
                kind = LINK_SOLID;
            else if (k == K_INLET)
                kind = LINK_INLET;
            else if (sx >= g.nx)
                kind = LINK_CLAMP; // the outlet's zero-gradient source
            w |= kind << (2 * i);
        }
    }
    links[m] = w;
}

hipError_t launch_types(const Geometry& g, const uint8_t* flags, uint8_t* types, hipStream_t s)
{
    hipLaunchKernelGGL(k_types, dim3(blocks_for(g.px * g.ny, 256)), dim3(256), 0, s, g, flags, types);
    return hipGetLastError();
}

hipError_t launch_links(const Geometry& g, const uint8_t* types, uint32_t* links, hipStream_t s)
{
    hipLaunchKernelGGL(k_links, dim3(blocks_for(g.px * g.ny, 256)), dim3(256), 0, s, g, types, links);
    return hipGetLastError();
}

// ---------------------------------------------------------------- init
template <int S, int L, class T>
__global__ void k_init(KParams p, T* __restrict__ lat)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.g.px * p.g.ny) return;
    const int64_t y = n / p.g.px, x = n - y * p.g.px;
    const bool upd = updated(p.types[n]);
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        float v = 0.0f;
        if (upd) {
            if constexpr (S == ST_PULL) {
                v = p.ph.e0[j];
            } else if constexpr (S == ST_SWAP) {
                v = p.ph.e0[dir_opp(j)];
            } else { // push: incoming values of the initial pull state
                int64_t sn;
                const int k = pull_source(p.g, p.types, x, y, j, sn);
                v = k == K_NODE ? p.ph.e0[j] : (k == K_SOLID ? p.ph.e0[dir_opp(j)] : p.ph.ein[j]);
            }
        }
        lat[lat_at<L>(j, n, p.g.P)] = st<T>(v);
    }
}

hipError_t launch_init(int state, int layout, int prec, const KParams& p, void* lat, hipStream_t s)
{
    return dispatch(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k_init<decltype(S)::value, decltype(L)::value, T>), dim3(blocks_for(p.g.px * p.g.ny, 256)),
                           dim3(256), 0, s, p, (T*)lat);
        return hipGetLastError();
    });
}

// ---------------------------------------------------------------- state load
// Post-collision values f [9][ny][nx] -> slots of a pull or swap lattice.
template <int S, int L, class T>
__global__ void k_set_post(KParams p, const float* __restrict__ f, T* __restrict__ lat)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = p.g.nx * p.g.ny;
    if (m >= N) return;
    const int64_t y = m / p.g.nx, x = m - y * p.g.nx;
    const int64_t n = y * p.g.px + x;
    // solid nodes hold state under full-way bounce-back
    if (!updated(p.types[n]) && !(p.g.fw && node_type(p.types[n]) == T_SOLID)) return;
#pragma unroll
    for (int i = 0; i < 9; ++i) lat[lat_at<L>(post_slot<S>(i), n, p.g.P)] = st<T>(f[i * N + m]);
}

// Pull lattice -> push lattice: stream once without colliding.
template <int L, class T>
__global__ void k_pull_to_push(KParams p, const T* __restrict__ pull, T* __restrict__ push)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= p.g.px * p.g.ny) return;
    const int64_t y = n / p.g.px, x = n - y * p.g.px;
    if (!updated(p.types[n])) return;
    float f[9];
    gather_pull<L, ST_PULL>(p, pull, x, y, n, f);
#pragma unroll
    for (int i = 0; i < 9; ++i) push[lat_at<L>(i, n, p.g.P)] = st<T>(f[i]);
}

hipError_t launch_set_state(int state, int layout, int prec, const KParams& p, const float* f, void* lat, void* tmp,
                            hipStream_t s)
{
    return dispatch(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        constexpr int SV = decltype(S)::value, LV = decltype(L)::value;
        const uint32_t nb = blocks_for(p.g.nx * p.g.ny, 256);
        if constexpr (SV == ST_PUSH) {
            if (!tmp) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_set_post<ST_PULL, LV, T>), dim3(nb), dim3(256), 0, s, p, f, (T*)tmp);
            hipLaunchKernelGGL((k_pull_to_push<LV, T>), dim3(blocks_for(p.g.px * p.g.ny, 256)), dim3(256), 0, s, p,
                               (const T*)tmp, (T*)lat);
        } else {
            hipLaunchKernelGGL((k_set_post<SV, LV, T>), dim3(nb), dim3(256), 0, s, p, f, (T*)lat);
        }
        return hipGetLastError();
    });
}

// ------------------------------------------------------ Neumann inlet state
// rho - 1 of the node (1, y) of every row from shifted post-collision values
// f [9][ny][nx] (summed as an update sums its incoming values), 0 where that
// node is not updated.
__global__ void k_inlet_density_fill(KParams p, const float* __restrict__ f, float* __restrict__ rin)
{
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= p.g.ny) return;
    float r = 0.0f;
    if (p.g.nx > 1 && updated(p.types[y * p.g.px + 1])) {
        const int64_t N = p.g.nx * p.g.ny, m = y * p.g.nx + 1;
        float v[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = f[i * N + m];
        r = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])) + v[8];
    }
    rin[y] = r;
}

hipError_t launch_inlet_density_fill(const KParams& p, const float* f, float* rin, hipStream_t s)
{
    hipLaunchKernelGGL(k_inlet_density_fill, dim3(blocks_for(p.g.ny, 256)), dim3(256), 0, s, p, f, rin);
    return hipGetLastError();
}

// ---------------------------------------------------------- AA outlet buffer
template <int L, class T>
__global__ void k_aa_outlet_fill(KParams p, const T* __restrict__ lat, T* __restrict__ obuf)
{
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= p.g.ny) return;
    const int64_t n = y * p.g.px + (p.g.nx - 1);
    if (!updated(p.types[n])) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) obuf[3 * y + k] = lat[lat_at<L>(dir_opp(3 * k), n, p.g.P)];
}

hipError_t launch_aa_outlet_fill(int layout, int prec, const KParams& p, const void* lat, void* obuf, hipStream_t s)
{
    return dispatch(ST_SWAP, layout, prec, [&](auto, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        constexpr int LV = decltype(L)::value;
        hipLaunchKernelGGL((k_aa_outlet_fill<LV, T>), dim3(blocks_for(p.g.ny, 256)), dim3(256), 0, s, p,
                           (const T*)lat, (T*)obuf);
        return hipGetLastError();
    });
}

// ---------------------------------------------------------------- edge fill
template <int S, int L, class T>
__global__ void k_edge_fill(KParams p, const T* __restrict__ lat, T* __restrict__ edge)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= p.g.nx * p.g.ny) return;
    const int y = (int)(m / p.g.nx), x = (int)(m - (int64_t)y * p.g.nx);
    const int64_t n = (int64_t)y * p.g.px + x;
    if (!updated(p.types[n])) return;
    TileCoord c;
    c.bx = x / p.g.tx;
    c.by = y / p.g.ty;
    c.x0 = c.bx * p.g.tx;
    c.y0 = c.by * p.g.ty;
    c.x1 = (int)min((int64_t)(c.x0 + p.g.tx), p.g.nx);
    c.y1 = (int)min((int64_t)(c.y0 + p.g.ty), p.g.ny);
    float r[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) r[i] = ld(lat[lat_at<L>(post_slot<S>(i), n, p.g.P)]);
    edge_emit(p.g, c, x, y, r, edge);
}

hipError_t launch_edge_fill(int state, int layout, int prec, const KParams& p, const void* lat, void* edge,
                            hipStream_t s)
{
    return dispatch(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        constexpr int SV = decltype(S)::value;
        if constexpr (SV == ST_PUSH) {
            return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((k_edge_fill<SV, decltype(L)::value, T>), dim3(blocks_for(p.g.nx * p.g.ny, 256)),
                               dim3(256), 0, s, p, (const T*)lat, (T*)edge);
            return hipGetLastError();
        }
    });
}

// ---------------------------------------------------------------- readouts
template <int S, int L, class T>
__global__ void k_get_pop(KParams p, const T* __restrict__ lat, float* __restrict__ out)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = p.g.nx * p.g.ny;
    if (m >= N) return;
    const int64_t y = m / p.g.nx, x = m - y * p.g.nx;
    const int64_t n = y * p.g.px + x;
    const uint8_t t = p.types[n];
    const bool upd = updated(t), inlet = node_type(t) == T_INLET;
    float f[9];
    gather_state<L, S>(p, lat, x, y, upd ? n : 0, f); // in-bounds for every node
#pragma unroll
    for (int i = 0; i < 9; ++i) out[i * N + m] = upd ? f[i] : (inlet ? inlet_node_value(p, i, y) : 0.0f);
}

hipError_t launch_get_populations(int state, int layout, int prec, const KParams& p, const void* lat, float* f,
                                  hipStream_t s)
{
    return dispatch(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k_get_pop<decltype(S)::value, decltype(L)::value, T>),
                           dim3(blocks_for(p.g.nx * p.g.ny, 256)), dim3(256), 0, s, p, (const T*)lat, f);
        return hipGetLastError();
    });
}

template <int S, int L, class T>
__global__ void k_macros(KParams p, const T* __restrict__ lat, float* __restrict__ rho, float* __restrict__ u)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t N = p.g.nx * p.g.ny;
    if (m >= N) return;
    const int64_t y = m / p.g.nx, x = m - y * p.g.nx;
    const int64_t n = y * p.g.px + x;
    const uint8_t t = p.types[n];
    float r = 0.0f, ux = 0.0f, uy = 0.0f;
    if (updated(t)) {
        float f[9];
        gather_state<L, S>(p, lat, x, y, n, f);
        float rt, jx, jy;
        moments(f, rt, jx, jy);
        r = 1.0f + rt;
        ux = jx + p.ph.hg[0];
        uy = jy + p.ph.hg[1];
    } else if (node_type(t) == T_INLET) {
        r = p.rin ? 1.0f + p.rin[y] : 1.0f;
        ux = p.ph.u_in[0];
        uy = p.ph.u_in[1];
    }
    if (rho) rho[m] = r;
    if (u) {
        u[m] = ux;
        u[N + m] = uy;
    }
}

hipError_t launch_macros(int state, int layout, int prec, const KParams& p, const void* lat, float* rho, float* u,
                         hipStream_t s)
{
    return dispatch(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k_macros<decltype(S)::value, decltype(L)::value, T>),
                           dim3(blocks_for(p.g.nx * p.g.ny, 256)), dim3(256), 0, s, p, (const T*)lat, rho, u);
        return hipGetLastError();
    });
}

// ---------------------------------------------------------------- FP64 diagnostics
constexpr int DIAG_BLOCKS = 1024;
constexpr int DIAG_THREADS = 256;
constexpr int DIAG_VALUES = 5;

int diag_partials() { return DIAG_BLOCKS * DIAG_VALUES; }

// Fixed-shape block reduction (deterministic order).
__device__ __forceinline__ double block_sum(double v, double* sh)
{
    const int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int w = DIAG_THREADS / 2; w > 0; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <int S, int L, class T>
__global__ void __launch_bounds__(DIAG_THREADS)
    k_diag(KParams p, const T* __restrict__ lat, double* __restrict__ u_prev, int have_prev, double* __restrict__ part)
{
    __shared__ double sh[DIAG_THREADS];
    const int64_t N = p.g.nx * p.g.ny;
    double acc[DIAG_VALUES] = {0, 0, 0, 0, 0};
    for (int64_t m = (int64_t)blockIdx.x * DIAG_THREADS + threadIdx.x; m < N; m += (int64_t)DIAG_BLOCKS * DIAG_THREADS) {
        const int64_t y = m / p.g.nx, x = m - y * p.g.nx;
        const int64_t n = y * p.g.px + x;
        if (!updated(p.types[n])) continue;
        float f[9];
        gather_state<L, S>(p, lat, x, y, n, f);
        double r = 1.0, jx = 0.0, jy = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double v = (double)f[i];
            r += v;
            jx += dir_cx(i) * v;
            jy += dir_cy(i) * v;
        }
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        const double ux = jx + (double)p.ph.hg[0];
        const double uy = jy + (double)p.ph.hg[1];
        // previous velocities: 2 doubles per node, dense [ny][nx][2]
        if (u_prev) {
            if (have_prev) {
                const double dx = ux - u_prev[2 * m], dy = uy - u_prev[2 * m + 1];
                acc[3] += dx * dx + dy * dy;
            }
            u_prev[2 * m] = ux;
            u_prev[2 * m + 1] = uy;
        }
        acc[4] += ux * ux + uy * uy;
    }
    for (int k = 0; k < DIAG_VALUES; ++k) {
        const double t = block_sum(acc[k], sh);
        if (threadIdx.x == 0) part[blockIdx.x * DIAG_VALUES + k] = t;
    }
}

__global__ void __launch_bounds__(DIAG_THREADS) k_diag_final(const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double sh[DIAG_THREADS];
    for (int k = 0; k < DIAG_VALUES; ++k) {
        double a = 0.0;
        for (int b = threadIdx.x; b < DIAG_BLOCKS; b += DIAG_THREADS) a += part[b * DIAG_VALUES + k];
        const double t = block_sum(a, sh);
        if (threadIdx.x == 0) out[k] = t;
    }
}

// The four diagnostics from the five sums of k_diag_final: mass, momentum,
// and the residual sqrt(sum |du|^2) / sqrt(sum |u|^2) (-1 without a previous
// velocity field, 0 for a field at rest), written to out (device).
__global__ void k_diag_result(const double* __restrict__ sums, int have_prev, double* __restrict__ out)
{
    if (threadIdx.x != 0) return;
    out[0] = sums[0];
    out[1] = sums[1];
    out[2] = sums[2];
    out[3] = have_prev ? (sums[4] > 0 ? sqrt(sums[3]) / sqrt(sums[4]) : 0.0) : -1.0;
}

hipError_t launch_diag_result(const double* sums, int have_prev, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_diag_result, dim3(1), dim3(64), 0, s, sums, have_prev, out);
    return hipGetLastError();
}

hipError_t launch_diag(int state, int layout, int prec, const KParams& p, const void* lat, double* u_prev,
                       int have_prev, double* partials, double* out, hipStream_t s)
{
    return dispatch(state, layout, prec, [&](auto S, auto L, auto TT) {
        using T = typename decltype(TT)::type;
        hipLaunchKernelGGL((k_diag<decltype(S)::value, decltype(L)::value, T>), dim3(DIAG_BLOCKS), dim3(DIAG_THREADS),
                           0, s, p, (const T*)lat, u_prev, have_prev, partials);
        hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DIAG_THREADS), 0, s, (const double*)partials, out);
        return hipGetLastError();
    });
}

} // namespace lbm

// ---------------------------------------------------------------- bandwidth probe
// Plain streaming kernels of known byte counts: the practical HBM bandwidth
// and the calibration of the memory counters are measured with them.
namespace lbm {

// Each thread keeps U independent 16-byte accesses in flight per iteration;
// consecutive lanes touch consecutive 16-byte words (fully coalesced).
constexpr int PROBE_U = 4;

__global__ void __launch_bounds__(256) k_probe_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x * PROBE_U;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x * PROBE_U + threadIdx.x; k < n; k += step) {
        float4 v[PROBE_U];
#pragma unroll
        for (int u = 0; u < PROBE_U; ++u) {
            const int64_t j = k + (int64_t)u * blockDim.x;
            if (j < n) v[u] = src[j];
        }
#pragma unroll
        for (int u = 0; u < PROBE_U; ++u) {
            const int64_t j = k + (int64_t)u * blockDim.x;
            if (j < n) dst[j] = v[u];
        }
    }
}

__global__ void __launch_bounds__(256) k_probe_read(const float4* __restrict__ src, int64_t n, float* __restrict__ sink)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x * PROBE_U;
    float acc = 0.0f;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x * PROBE_U + threadIdx.x; k < n; k += step) {
#pragma unroll
        for (int u = 0; u < PROBE_U; ++u) {
            const int64_t j = k + (int64_t)u * blockDim.x;
            if (j < n) {
                const float4 v = src[j];
                acc += (v.x + v.y) + (v.z + v.w);
            }
        }
    }
    if (acc == 1.2345e-30f) sink[0] = acc; // keeps the loads alive; practically never true
}

__global__ void __launch_bounds__(256) k_probe_write(float4* __restrict__ dst, int64_t n)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x * PROBE_U;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x * PROBE_U + threadIdx.x; k < n; k += step)
#pragma unroll
        for (int u = 0; u < PROBE_U; ++u) {
            const int64_t j = k + (int64_t)u * blockDim.x;
            if (j < n) dst[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
}

// Copy with non-temporal loads and stores and PROBE_NT_U independent 16-byte
// pieces in flight per lane: the source is read once and the destination is
// not read again, so neither needs to stay in the caches.
constexpr int PROBE_NT_U = 8;

typedef float probe_v4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_probe_copy_nt(const probe_v4* __restrict__ src, probe_v4* __restrict__ dst,
                                                       int64_t n)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x * PROBE_NT_U;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x * PROBE_NT_U + threadIdx.x; k < n; k += step) {
        probe_v4 v[PROBE_NT_U];
#pragma unroll
        for (int u = 0; u < PROBE_NT_U; ++u) {
            const int64_t j = k + (int64_t)u * blockDim.x;
            if (j < n) v[u] = __builtin_nontemporal_load(src + j);
        }
#pragma unroll
        for (int u = 0; u < PROBE_NT_U; ++u) {
            const int64_t j = k + (int64_t)u * blockDim.x;
            if (j < n) __builtin_nontemporal_store(v[u], dst + j);
        }
    }
}

hipError_t launch_probe(int mode, void* dst, const void* src, int64_t bytes, hipStream_t s)
{
    const int64_t n = bytes / 16;
    if (mode == 3) {
        const uint32_t nb = (uint32_t)std::min<int64_t>((n + 256 * PROBE_NT_U - 1) / (256 * PROBE_NT_U), 256 * 16);
        hipLaunchKernelGGL(k_probe_copy_nt, dim3(nb), dim3(256), 0, s, (const probe_v4*)src, (probe_v4*)dst, n);
        return hipGetLastError();
    }
    const uint32_t blocks = (uint32_t)std::min<int64_t>((n + 256 * PROBE_U - 1) / (256 * PROBE_U), 256 * 32);
    if (mode == 0)
        hipLaunchKernelGGL(k_probe_copy, dim3(blocks), dim3(256), 0, s, (const float4*)src, (float4*)dst, n);
    else if (mode == 1)
        hipLaunchKernelGGL(k_probe_read, dim3(blocks), dim3(256), 0, s, (const float4*)src, n, (float*)dst);
    else
        hipLaunchKernelGGL(k_probe_write, dim3(blocks), dim3(256), 0, s, (float4*)dst, n);
    return hipGetLastError();
}

} // namespace lbm
