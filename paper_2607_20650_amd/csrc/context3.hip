// context3.hip -- the lbm3_* entry points of include/lbm.h: one D3Q19
// simulation (the 3-D extension Section 6 of the paper names) owned by the
// library, its validation, allocation, state bookkeeping and readouts.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "lbm.h"
#include "lbm3.hpp"
#include "lbm3_kernels.hpp"

using namespace lbm;

namespace {

thread_local std::string g_create3_error;

int64_t round_up3(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Shifted equilibrium feq(1, u) - w of the 19 directions, in FP64 then rounded.
void feq3_shifted(const double u[3], float* out)
{
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q3; ++i) {
        const int c2 = q3_c2(i);
        const double w = c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        const double cu = q3_cx(i) * u[0] + q3_cy(i) * u[1] + q3_cz(i) * u[2];
        out[i] = (float)(w * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

} // namespace

struct lbm3_ctx {
    lbm3_grid grid{};
    KParams3 kp{};
    int elem = 4;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* lat[2] = {nullptr, nullptr};
    void* obuf = nullptr; // AA with an outlet: 5 values per (y, z) row
    uint8_t* types = nullptr;
    float* readout = nullptr; // 19 * N floats, lazily
    double* u_prev = nullptr; // 3 * padded nodes, lazily (diagnostics)
    double* partials = nullptr;
    double* dout = nullptr;
    bool have_prev = false;
    int64_t lat_elems = 0;
    int64_t t = 0;
    bool poisoned = false;
    std::string err;

    lbm_status fail(lbm_status s, const std::string& msg)
    {
        err = msg;
        if (s == LBM_EDEVICE) poisoned = true;
        return s;
    }
    lbm_status check(hipError_t e, const char* what)
    {
        if (e == hipSuccess) return LBM_OK;
        return fail(LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
    bool aa() const { return grid.scheme == LBM_AA; }
    // AA holds the push form at even update counts, the swap form at odd ones
    int state() const { return aa() ? ((t & 1) ? ST_SWAP : ST_PUSH) : ST_PULL; }
    void* cur() const { return aa() ? lat[0] : lat[t & 1]; }
    int64_t nodes() const { return grid.nx * grid.ny * grid.nz; }
};

namespace {

void free3(lbm3_ctx* c)
{
    for (void* p : {c->lat[0], c->lat[1], c->obuf, (void*)c->types, (void*)c->readout, (void*)c->u_prev,
                    (void*)c->partials, (void*)c->dout})
        if (p) (void)hipFree(p);
    c->u_prev = nullptr;
    c->partials = c->dout = nullptr;
    c->lat[0] = c->lat[1] = c->obuf = nullptr;
    c->types = nullptr;
    c->readout = nullptr;
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
}

lbm_status create3_error(lbm_status s, const std::string& msg)
{
    g_create3_error = msg;
    return s;
}

lbm_status ensure_readout3(lbm3_ctx* c)
{
    if (c->readout) return LBM_OK;
    if (hipMalloc((void**)&c->readout, (size_t)c->nodes() * Q3 * sizeof(float)) != hipSuccess) {
        c->readout = nullptr;
        (void)hipGetLastError();
        return c->fail(LBM_ENOMEM, "readout buffer allocation failed");
    }
    return LBM_OK;
}

} // namespace

extern "C" {

lbm_status lbm3_create(const lbm3_grid* grid, const uint8_t* flags, double tau, const lbm3_bc* bc, void* stream,
                       lbm3_ctx** out)
{
    if (out) *out = nullptr;
    auto bad = [](const char* m) { return create3_error(LBM_EINVAL, m); };
    if (!grid || !flags || !bc || !out) return bad("grid, flags, bc and out must be non-NULL");
    const int64_t nx = grid->nx, ny = grid->ny, nz = grid->nz;
    if (nx < 1 || ny < 1 || nz < 1) return bad("nx, ny and nz must be >= 1");
    if (nx > (1ll << 20) || ny > (1ll << 20) || nz > (1ll << 20)) return bad("nx, ny and nz must be <= 2^20");
    if (nx * ny * nz > (1ll << 40)) return bad("the grid must hold at most 2^40 nodes");
    if (grid->scheme != LBM_NPTL && grid->scheme != LBM_AA) return bad("D3Q19 scheme must be LBM_NPTL or LBM_AA");
    if (grid->layout != LBM_STREAM && grid->layout != LBM_COLLISION && grid->layout != LBM_BLOCKED)
        return bad("D3Q19 layout must be LBM_STREAM, LBM_COLLISION or LBM_BLOCKED");
    if (grid->precision < LBM_FP32 || grid->precision > LBM_FP16C_SR) return bad("unknown precision");
    if (bc->x_axis != LBM_PERIODIC && bc->x_axis != LBM_CLOSED && bc->x_axis != LBM_INFLOW_OUTFLOW)
        return bad("bad x axis (periodic, closed or inflow/outflow)");
    if (bc->y_axis != LBM_PERIODIC && bc->y_axis != LBM_CLOSED) return bad("y axis must be periodic or closed");
    if (bc->z_axis != LBM_PERIODIC && bc->z_axis != LBM_CLOSED) return bad("z axis must be periodic or closed");
    if (bc->x_axis == LBM_INFLOW_OUTFLOW && nx < 2) return bad("inflow/outflow needs nx >= 2");
    if (!std::isfinite(tau) || tau <= 0.5) return bad("tau must be finite and > 1/2");
    if (bc->rho0 != 1.0) return bad("rho0 must be 1 (shifted storage assumes it)");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(bc->u_in[a]) || !std::isfinite(bc->g[a]) || !std::isfinite(bc->u0[a]))
            return bad("u_in, g and u0 must be finite");
    int32_t tx = grid->tile_x, ty = grid->tile_y;
    if (tx < 0 || ty < 0 || (tx == 0) != (ty == 0)) return bad("tile_x and tile_y must both be 0 or both positive");
    const int64_t px3 = (nx + 15) / 16 * 16;
    if (tx == 0 && grid->layout == LBM_COLLISION && nx >= 64 && aos3_staged(px3, ny, 64, 8)) {
        // whole records staged through LDS (measured on the 256^3 sphere
        // array): 64 x 8 patches (taller tiles cut the halo rows each staged
        // plane carries: FP32 +12% over 64 x 2, 16-bit pull +4-5% over
        // 64 x 4), except the 16-bit AA pair at 64 x 4 (more blocks per CU:
        // +5-11% over 64 x 8)
        tx = 64;
        ty = grid->precision != LBM_FP32 && grid->scheme == LBM_AA ? 4 : 8;
    } else if (tx == 0) {
        // one block covers 256 nodes of a row where the row is long enough:
        // the longest contiguous runs per direction (measured on a 256^3
        // sphere array: 256 x 1 and 128 x 2 beat 64 x 4 by 8-15%)
        tx = nx >= 256 ? 256 : (nx >= 128 ? 128 : (nx >= 64 ? 64 : (nx >= 32 ? 32 : 16)));
        ty = 256 / tx;
    }
    // the staged collision-layout kernels take 64 x ty tiles up to 512 threads
    const int64_t max_threads = grid->layout == LBM_COLLISION && aos3_staged(px3, ny, tx, ty) ? 512 : 256;
    if ((int64_t)tx * ty > max_threads) return bad("tile needs more than 256 threads (512 for 64-wide collision-layout tiles)");
    const int64_t N = nx * ny * nz;
    for (int64_t k = 0; k < N; ++k)
        if (flags[k] > 1) return bad("flags must be 0 (fluid) or 1 (solid)");

    lbm3_ctx* c = new (std::nothrow) lbm3_ctx();
    if (!c) return create3_error(LBM_ENOMEM, "host allocation failed");
    c->grid = *grid;
    c->grid.tile_x = tx;
    c->grid.tile_y = ty;
    Geometry3& g = c->kp.g;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.px = round_up3(nx, grid->layout == LBM_BLOCKED ? 64 : 16);
    g.plane = g.px * ny;
    g.P = round_up3(g.plane * nz, 64);
    g.rstep = (g.px / 64) * (Q3 * 64); // used by the blocked layout only,
    g.pstep = (g.plane / 64) * (Q3 * 64); // where px is a multiple of 64
    g.yspan = ny * g.rstep;
    g.zspan = nz * g.pstep;
    g.xa = bc->x_axis == LBM_INFLOW_OUTFLOW ? (int32_t)AX_INOUT : bc->x_axis;
    g.ya = bc->y_axis;
    g.za = bc->z_axis;
    g.tx = tx;
    g.ty = ty;
    g.ntx = (int32_t)((nx + tx - 1) / tx);
    g.nty = (int32_t)((ny + ty - 1) / ty);
    if ((int64_t)g.ntx * g.nty * nz >= (1ll << 31)) {
        delete c;
        return bad("grid needs more than 2^31 blocks");
    }
    Physics3& ph = c->kp.ph;
    ph.omc = (float)(1.0 - 1.0 / tau);
    for (int i = 0; i < Q3; ++i) {
        const int c2 = q3_c2(i);
        const double w = c2 == 0 ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        ph.F[i] = (float)(3.0 * w * (q3_cx(i) * bc->g[0] + q3_cy(i) * bc->g[1] + q3_cz(i) * bc->g[2]));
    }
    feq3_shifted(bc->u_in, ph.ein);
    feq3_shifted(bc->u0, ph.e0);
    for (int a = 0; a < 3; ++a) {
        ph.hg[a] = (float)(0.5 * bc->g[a]);
        ph.u_in[a] = (float)bc->u_in[a];
    }
    c->elem = grid->precision == LBM_FP32 ? 4 : 2;
    c->lat_elems = grid->layout == LBM_STREAM ? (int64_t)Q3 * g.P : (int64_t)Q3 * g.plane * nz;

    if (stream) {
        c->stream = (hipStream_t)stream;
    } else if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return create3_error(LBM_EDEVICE, "hipStreamCreate failed");
    } else {
        c->own_stream = true;
    }
    const size_t lat_bytes = (size_t)c->lat_elems * c->elem;
    bool ok = hipMalloc(&c->lat[0], lat_bytes) == hipSuccess;
    if (ok && grid->scheme == LBM_NPTL) ok = hipMalloc(&c->lat[1], lat_bytes) == hipSuccess;
    if (ok && grid->scheme == LBM_AA && g.xa == AX_INOUT)
        ok = hipMalloc(&c->obuf, (size_t)(5 * ny * nz) * c->elem) == hipSuccess;
    if (ok) ok = hipMalloc((void**)&c->types, (size_t)(g.plane * nz)) == hipSuccess;
    uint8_t* dflags = nullptr;
    if (ok) ok = hipMalloc((void**)&dflags, (size_t)N) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        if (dflags) (void)hipFree(dflags);
        free3(c);
        delete c;
        return create3_error(LBM_ENOMEM, "device memory exhausted");
    }
    c->kp.types = c->types;
    hipError_t e = hipMemcpyAsync(dflags, flags, (size_t)N, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch3_types(g, dflags, c->types, c->stream);
    for (int k = 0; k < 2; ++k)
        if (e == hipSuccess && c->lat[k]) e = hipMemsetAsync(c->lat[k], 0, lat_bytes, c->stream);
    if (e == hipSuccess) e = launch3_init(c->state(), grid->layout, grid->precision, c->kp, c->lat[0], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dflags);
    if (e != hipSuccess) {
        std::string msg = std::string("initialisation failed: ") + hipGetErrorString(e);
        free3(c);
        delete c;
        return create3_error(LBM_EDEVICE, msg);
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm3_step(lbm3_ctx* c, int64_t n)
{
    if (!c) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    if (n < 0) return c->fail(LBM_EINVAL, "negative step count");
    for (int64_t k = 0; k < n; ++k) {
        const int parity = (int)(c->t & 1);
        const hipError_t e =
            c->aa() ? launch3_update(LBM_AA, c->grid.layout, c->grid.precision, c->kp, parity, nullptr, c->lat[0],
                                     c->obuf, c->stream)
                    : launch3_update(LBM_NPTL, c->grid.layout, c->grid.precision, c->kp, parity, c->lat[parity],
                                     c->lat[parity ^ 1], nullptr, c->stream);
        if (e != hipSuccess) return c->check(e, "update launch");
        ++c->t;
    }
    return LBM_OK;
}

lbm_status lbm3_macros(lbm3_ctx* c, float* rho, float* u, int on_device)
{
    if (!c) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    if (on_device)
        return c->check(launch3_macros(c->state(), c->grid.layout, c->grid.precision, c->kp, c->cur(), rho, u,
                                       c->stream),
                        "macros launch");
    lbm_status st = ensure_readout3(c);
    if (st != LBM_OK) return st;
    const int64_t N = c->nodes();
    float* dr = c->readout;
    float* du = c->readout + N;
    hipError_t e = launch3_macros(c->state(), c->grid.layout, c->grid.precision, c->kp, c->cur(), dr, du, c->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, dr, N * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, du, 3 * N * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return c->check(e, "macros readout");
}

lbm_status lbm3_get_populations(lbm3_ctx* c, float* f, int on_device)
{
    if (!c || !f) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    if (on_device)
        return c->check(launch3_get_populations(c->state(), c->grid.layout, c->grid.precision, c->kp, c->cur(), f,
                                                c->stream),
                        "populations launch");
    lbm_status st = ensure_readout3(c);
    if (st != LBM_OK) return st;
    hipError_t e = launch3_get_populations(c->state(), c->grid.layout, c->grid.precision, c->kp, c->cur(),
                                           c->readout, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(f, c->readout, (size_t)c->nodes() * Q3 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return c->check(e, "populations readout");
}

lbm_status lbm3_set_state(lbm3_ctx* c, const float* f, int on_device)
{
    if (!c || !f) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    const float* src = f;
    if (!on_device) {
        lbm_status st = ensure_readout3(c);
        if (st != LBM_OK) return st;
        const hipError_t e = hipMemcpyAsync(c->readout, f, (size_t)c->nodes() * Q3 * sizeof(float),
                                            hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return c->check(e, "state upload");
        src = c->readout;
    }
    // the push form is built from the pull form through a temporary lattice
    void* tmp = nullptr;
    if (c->state() == ST_PUSH && hipMalloc(&tmp, (size_t)c->lat_elems * c->elem) != hipSuccess) {
        (void)hipGetLastError();
        return c->fail(LBM_ENOMEM, "temporary lattice for the state load");
    }
    hipError_t e = launch3_set_state(c->state(), c->grid.layout, c->grid.precision, c->kp, src, c->cur(), tmp,
                                     c->stream);
    if (e == hipSuccess && c->obuf && c->state() == ST_SWAP)
        e = launch3_aa_outlet_fill(c->grid.layout, c->grid.precision, c->kp, c->cur(), c->obuf, c->stream);
    if (tmp) {
        const hipError_t e2 = hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->stream);
    c->have_prev = false;
    return c->check(e, "state load");
}

lbm_status lbm3_diag(lbm3_ctx* c, double out[5])
{
    if (!c || !out) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    const Geometry3& g = c->kp.g;
    auto get = [&](void** p, size_t bytes) {
        if (*p) return true;
        if (hipMalloc(p, bytes) == hipSuccess) return true;
        *p = nullptr;
        (void)hipGetLastError();
        return false;
    };
    if (!get((void**)&c->u_prev, (size_t)(3 * g.plane * g.nz) * sizeof(double)) ||
        !get((void**)&c->partials, (size_t)diag3_partials() * sizeof(double)) ||
        !get((void**)&c->dout, 8 * sizeof(double)))
        return c->fail(LBM_ENOMEM, "diagnostics buffer allocation failed");
    double h[6];
    hipError_t e = launch3_diag(c->state(), c->grid.layout, c->grid.precision, c->kp, c->cur(), c->u_prev,
                                c->have_prev ? 1 : 0, c->partials, c->dout, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h, c->dout, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    const lbm_status st = c->check(e, "diagnostics");
    if (st != LBM_OK) return st;
    for (int k = 0; k < 4; ++k) out[k] = h[k];
    out[4] = c->have_prev ? (h[5] > 0 ? std::sqrt(h[4]) / std::sqrt(h[5]) : 0.0) : -1.0;
    c->have_prev = true;
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(h[k])) {
            c->err = "non-finite mass or momentum";
            return LBM_EUNSTABLE;
        }
    return LBM_OK;
}

lbm_status lbm3_sync(lbm3_ctx* c)
{
    if (!c) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    return c->check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

const char* lbm3_last_error(const lbm3_ctx* c)
{
    if (!c) return g_create3_error.c_str();
    return c->err.c_str();
}

void lbm3_destroy(lbm3_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free3(c);
    delete c;
}

int32_t lbm3_bytes_per_update(int32_t precision) { return precision == LBM_FP32 ? 2 * Q3 * 4 : 2 * Q3 * 2; }

} // extern "C"
