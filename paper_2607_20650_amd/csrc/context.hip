// context.hip -- host runtime behind the C ABI of include/lbm.h: validation,
// all-or-nothing allocation, the tile chooser, per-step launch bookkeeping,
// cached HIP graphs of K-update bundles, readouts and FP64 diagnostics.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "lbm.h"
#include "lbm_common.hpp"
#include "lbm_host.hpp"
#include "lbm_kernels.hpp"

using namespace lbm;

namespace {

thread_local std::string g_create_error;

// Eq. 2 weights and velocity set, for the host-side constants below.
constexpr double kW[9] = {1.0 / 36, 1.0 / 9, 1.0 / 36, 1.0 / 9, 4.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 9, 1.0 / 36};

// Shifted equilibrium feq_i(1, u) - w_i of Eq. 2, in FP64.
void shifted_feq(double ux, double uy, float out[9])
{
    const double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        const double cu = dir_cx(i) * ux + dir_cy(i) * uy;
        out[i] = (float)(kW[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

bool is_two_lattice(int scheme) { return scheme == S_LPTL || scheme == S_NPTL || scheme == S_PUSH; }

// x-axis kinds with an inlet column and an outlet column.
bool is_inout(int axis) { return axis >= LBM_INFLOW_OUTFLOW && axis <= LBM_NEUMANN_PRESSURE; }
bool is_pressure_outlet(int axis) { return axis == LBM_INFLOW_PRESSURE || axis == LBM_NEUMANN_PRESSURE; }
bool is_neumann_inlet(int axis) { return axis == LBM_NEUMANN_OUTFLOW || axis == LBM_NEUMANN_PRESSURE; }

// One-lattice schemes that exchange through the tile buffer grid.
bool has_buffer_grid(int scheme) { return scheme == S_NPOL || scheme == S_NSOL; }

int state_of(int scheme)
{
    if (scheme == S_PUSH || scheme == S_AA) return ST_PUSH; // AA: at even update counts
    if (scheme == S_NSOL) return ST_SWAP;
    return ST_PULL;
}

} // namespace

struct lbm_ctx {
    lbm_grid grid{};
    lbm_bc bc{};
    double tau = 0;
    KParams kp{};
    int state = ST_PULL;
    int elem = 4; // bytes per stored population
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap = nullptr; // private stream used only to capture graphs
    void* lat[2] = {nullptr, nullptr};     // first element of each lattice
    void* lat_raw[2] = {nullptr, nullptr}; // allocations: guard, lattice, guard
    int64_t guard = 0;                     // guard elements on each side
    void* edge[2] = {nullptr, nullptr};
    void* obuf = nullptr; // AA outlet side buffer (3 values per row)
    float* rin = nullptr; // Neumann inlet: rho - 1 of column 1 per row, two halves by update parity
    uint8_t* types = nullptr;
    uint32_t* links = nullptr; // link words [ny][px]
    float* readout = nullptr; // 9 * nx * ny floats, lazily
    double* u_prev = nullptr; // 2 * px * ny doubles, lazily
    double* partials = nullptr;
    double* dout = nullptr;
    int64_t lat_elems = 0, edge_elems = 0;
    int64_t t = 0;
    int32_t bundle = 32;
    int32_t block = 256;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    bool have_prev = false;
    bool poisoned = false;
    std::string err;
    int64_t bytes = 0;
    int64_t fluid = 0;
    int device = 0; // device current at lbm_create

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
    void* cur_lat() const { return is_two_lattice(grid.scheme) ? lat[t & 1] : lat[0]; }
    // State kind of the current lattice: AA alternates push (even t) and swap (odd t).
    int state_now() const { return grid.scheme == S_AA ? ((t & 1) ? ST_SWAP : ST_PUSH) : state; }
    void* other_lat() const { return is_two_lattice(grid.scheme) ? lat[(t + 1) & 1] : nullptr; }
    // Kernel parameters of the update of the given parity (update: it records
    // the Neumann inlet densities for the next one) or of a readout.
    KParams at(int parity, bool update) const
    {
        KParams p = kp;
        if (rin) {
            p.rin = rin + (int64_t)parity * grid.ny;
            p.rout = update ? rin + (int64_t)(parity ^ 1) * grid.ny : nullptr;
        }
        return p;
    }
    KParams view() const { return at((int)(t & 1), false); }
};

namespace {

void free_all(lbm_ctx* c)
{
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
        c->gexec[k] = nullptr;
        c->graph[k] = nullptr;
        if (c->lat_raw[k]) (void)hipFree(c->lat_raw[k]);
        if (c->edge[k]) (void)hipFree(c->edge[k]);
        c->lat[k] = c->lat_raw[k] = c->edge[k] = nullptr;
    }
    if (c->obuf) (void)hipFree(c->obuf);
    c->obuf = nullptr;
    if (c->rin) (void)hipFree(c->rin);
    c->rin = nullptr;
    void* ptrs[] = {c->types, c->links, c->readout, c->u_prev, c->partials, c->dout};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    c->types = nullptr;
    c->links = nullptr;
    c->readout = nullptr;
    c->u_prev = nullptr;
    c->partials = c->dout = nullptr;
    if (c->cap) (void)hipStreamDestroy(c->cap);
    c->cap = nullptr;
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
}

lbm_status create_error(lbm_status s, const std::string& msg)
{
    g_create_error = msg;
    return s;
}

// Tile chooser (the paper's work-group decomposition): for a block of
// `threads` threads, each updating `vx` consecutive nodes of a row, the tile
// width is a multiple of one 64-wide wavefront row (64 * vx nodes) and the
// arrangement minimises the tile perimeter, i.e. the interface between tiles.
void choose_tile(int64_t nx, int threads, int vx, int32_t& tx, int32_t& ty)
{
    int best_x = 64 * vx, best_y = threads / 64;
    int64_t best = INT64_MAX;
    for (int w = 64; w <= threads; w += 64) {
        if (threads % w) continue;
        const int h = threads / w;
        const int64_t per = 2 * (int64_t)(w * vx + h);
        if (per < best) {
            best = per;
            best_x = w * vx;
            best_y = h;
        }
    }
    tx = best_x;
    ty = best_y;
    if (nx < tx) { // narrow grids: keep the block but use fewer columns
        int w = vx;
        while (w < nx) w <<= 1;
        tx = w;
        ty = threads / (w / vx);
    }
}

// Nodes per thread of the tiled pull, per layout and storage precision: the
// fastest setting measured on MI355X for the 4096 x 1024 Karman case (one
// node per thread keeps the most waves resident; only FP16 bundle runs gain
// from pairs of nodes).
int pull_nodes_per_thread(int layout, int prec) { return (prec != LBM_FP32 && layout == LBM_BUNDLE) ? 2 : 1; }

// Default tiles measured on MI355X (4096 x 1024 Karman case, tile sweeps):
// NPOL 64 x 8 (FP32 stream / bundle) and 64 x 4 (FP32 collision, binary16),
// NSOL 64 x 8 (FP32) and 32 x 8 (binary16: squarer tiles, fewer edge values;
// +3% over 64 x 4); for binary16 storage NPTL 32 x 2
// (stream) or 32 x 4 and AA 32 x 4.  Wider or taller one-lattice tiles cut
// buffer-grid traffic but leave fewer blocks to hide latency.  Other cases use
// choose_tile.
bool measured_tile(int scheme, int layout, int prec, int64_t nx, int32_t& tx, int32_t& ty)
{
    if (scheme == LBM_NPOL) {
        tx = 64;
        ty = prec == LBM_FP32 && layout != LBM_COLLISION ? 8 : 4;
    } else if (scheme == LBM_NSOL) {
        tx = prec == LBM_FP32 ? 64 : 32;
        ty = 8;
    } else if ((scheme == LBM_NPTL || scheme == LBM_AA || scheme == LBM_TL_PUSH) && layout == LBM_COLLISION &&
               prec == LBM_FP32) {
        // FP32 records staged through LDS (one node per thread, 64-wide
        // tiles): 64 x 8 for the pull and the push (fewer halo rows per staged
        // tile: +1.4% and +8% over 64 x 4), 64 x 4 for AA; binary16 records run
        // unstaged on the smaller tiles below, where the staged kernels gain
        // little, bound by their 2-byte LDS accesses
        tx = 64;
        ty = scheme == LBM_AA ? 4 : 8;
    } else if (scheme == LBM_NPTL && prec != LBM_FP32) {
        // binary16 moves half the bytes per node: small blocks (one or two
        // wavefronts) keep more of them in flight per CU
        tx = 32;
        ty = layout == LBM_STREAM ? 2 : 4;
    } else if (scheme == LBM_AA && prec != LBM_FP32) {
        tx = 32;
        ty = 4;
    } else if (scheme == LBM_TL_PUSH && layout != LBM_COLLISION) {
        // direct scattered stores: binary16 on one-wavefront 32 x 2 tiles
        // (+12% stream, +5% bundle over 64 x 4), FP32 on 128 x 2 (+1-2%)
        tx = prec == LBM_FP32 ? 128 : 32;
        ty = 2;
    } else {
        return false;
    }
    return nx >= tx;
}

// Threads per block of a tiled update kernel for a tile of tx * ty nodes.
int tile_threads(int scheme, int layout, int prec, int tx, int ty)
{
    const int vx = scheme == LBM_NPTL ? pull_nodes_per_thread(layout, prec) : 1;
    if (tx % vx == 0) return (tx / vx) * ty;
    return tx * ty;
}

lbm_status alloc(lbm_ctx* c, void** p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return LBM_ENOMEM;
    }
    c->bytes += (int64_t)bytes;
    return LBM_OK;
}

lbm_status launch_one(lbm_ctx* c, int parity, hipStream_t s)
{
    const KParams p = c->at(parity, true);
    hipError_t e;
    if (c->grid.scheme == S_AA)
        e = launch_aa(c->grid.layout, c->grid.precision, p, parity, c->lat[0], c->obuf, s);
    else if (is_two_lattice(c->grid.scheme))
        e = launch_update(c->grid.scheme, c->grid.layout, c->grid.precision, p, c->block, c->lat[parity],
                          c->lat[parity ^ 1], nullptr, nullptr, s);
    else
        e = launch_update(c->grid.scheme, c->grid.layout, c->grid.precision, p, c->block, nullptr, c->lat[0],
                          c->edge[parity], c->edge[parity ^ 1], s);
    return c->check(e, "update launch");
}

lbm_status build_graph(lbm_ctx* c, int parity)
{
    hipError_t e = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return c->check(e, "hipStreamBeginCapture");
    lbm_status st = LBM_OK;
    for (int k = 0; k < c->bundle && st == LBM_OK; ++k) st = launch_one(c, (parity + k) & 1, c->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap, &g);
    if (st != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return c->check(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return c->check(e, "hipGraphInstantiate");
    }
    c->graph[parity] = g;
    c->gexec[parity] = x;
    return LBM_OK;
}

void drop_graphs(lbm_ctx* c)
{
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        if (c->graph[k]) (void)hipGraphDestroy(c->graph[k]);
        c->gexec[k] = nullptr;
        c->graph[k] = nullptr;
    }
}

lbm_status ensure_readout(lbm_ctx* c)
{
    if (c->readout) return LBM_OK;
    const int64_t N = c->grid.nx * c->grid.ny;
    if (alloc(c, (void**)&c->readout, (size_t)N * 9 * sizeof(float)) != LBM_OK)
        return c->fail(LBM_ENOMEM, "readout buffer allocation failed");
    return LBM_OK;
}

} // namespace

// ------------------------------------------------------------ shared setup
// Validation and constants shared by simulations and served requests.
lbm_status lbm::setup_params(const lbm_grid* grid, const uint8_t* flags, double tau, const lbm_bc* bc, KParams& kp,
                             std::string& err)
{
    auto bad = [&](const char* m) {
        err = m;
        return LBM_EINVAL;
    };
    if (!grid || !flags || !bc) return bad("grid, flags and bc must be non-NULL");
    const int64_t nx = grid->nx, ny = grid->ny;
    if (nx < 1 || ny < 1) return bad("nx and ny must be >= 1");
    if (nx > (1ll << 30) || ny > (1ll << 30)) return bad("nx and ny must be <= 2^30");
    if (nx * ny > (1ll << 40)) return bad("the grid must hold at most 2^40 nodes");
    if (grid->scheme < LBM_LPTL || grid->scheme > LBM_AA) return bad("unknown scheme");
    if (grid->layout < LBM_STREAM || grid->layout > LBM_COLLISION) return bad("unknown layout");
    if (grid->precision < LBM_FP32 || grid->precision > LBM_FP16C_SR) return bad("unknown precision");
    if (bc->x_axis < LBM_PERIODIC || bc->x_axis > LBM_NEUMANN_PRESSURE) return bad("bad x axis");
    if (bc->y_axis != LBM_PERIODIC && bc->y_axis != LBM_CLOSED) return bad("y axis must be periodic or closed");
    if (is_inout(bc->x_axis) && nx < 2) return bad("inflow/outflow needs nx >= 2");
    if (!std::isfinite(tau) || tau <= 0.5) return bad("tau must be finite and > 1/2");
    if (bc->rho0 != 1.0) return bad("rho0 must be 1 (shifted storage assumes it)");
    if (bc->bounce != LBM_HALFWAY && bc->bounce != LBM_FULLWAY) return bad("bounce must be halfway or full-way");
    if (bc->bounce == LBM_FULLWAY && grid->scheme != LBM_LPTL && grid->scheme != LBM_NPTL)
        return bad("full-way bounce-back is built for the two-lattice pull schemes (LPTL, NPTL)");
    if (bc->bounce == LBM_FULLWAY && bc->x_axis > LBM_INFLOW_OUTFLOW)
        return bad("full-way bounce-back takes a periodic, closed or inflow/outflow x axis");
    const double vals[] = {bc->u_in[0], bc->u_in[1], bc->g[0], bc->g[1], bc->u0[0], bc->u0[1]};
    for (double v : vals)
        if (!std::isfinite(v)) return bad("u_in, g and u0 must be finite");
    const bool tiled = grid->scheme != LBM_LPTL;
    if (grid->tile_x < 0 || grid->tile_y < 0) return bad("negative tile size");
    if ((grid->tile_x == 0) != (grid->tile_y == 0))
        return bad("tile_x and tile_y must both be 0 (automatic) or both set");
    const int max_threads = (grid->scheme == LBM_NPOL || grid->scheme == LBM_NSOL) ? 1024 : 256;
    // the LDS-staged collision-layout kernels (64-wide tiles) take up to 512
    // (the full-way pull keeps the direct kernel)
    const bool staged_aos = grid->layout == LBM_COLLISION && grid->tile_x == 64 &&
                            ((grid->scheme == LBM_NPTL && bc->bounce == LBM_HALFWAY) || grid->scheme == LBM_AA ||
                             (grid->scheme == LBM_TL_PUSH && grid->precision == LBM_FP32));
    const int max_user_threads = staged_aos ? 512 : max_threads;
    if (grid->tile_x > 0 && ((int64_t)grid->tile_x * grid->tile_y > (1 << 16) ||
                             tile_threads(grid->scheme, grid->layout, grid->precision, grid->tile_x, grid->tile_y) >
                                 max_user_threads))
        return bad("tile needs more threads than a block of the scheme allows (256; 1024 for the one-lattice "
                   "schemes; 512 for 64-wide collision-layout tiles of the staged kernels)");
    const int64_t N = nx * ny;
    for (int64_t k = 0; k < N; ++k)
        if (flags[k] > 1) return bad("flags must be 0 (fluid) or 1 (solid)");

    kp.rin = nullptr;
    kp.rout = nullptr;
    kp.links = nullptr;
    Geometry& g = kp.g;
    g = Geometry{};
    g.nx = nx;
    g.ny = ny;
    g.px = round_up(nx, 16);
    g.P = round_up(g.px * ny, 64);
    g.xa = is_inout(bc->x_axis) ? (int32_t)AX_INOUT : bc->x_axis;
    g.zh = is_pressure_outlet(bc->x_axis) ? 1 : 0;
    g.fw = bc->bounce == LBM_FULLWAY ? 1 : 0;
    g.ya = bc->y_axis;
    g.vx = grid->scheme == LBM_NPTL ? pull_nodes_per_thread(grid->layout, grid->precision) : 1;
    if (tiled) {
        int32_t tx = grid->tile_x, ty = grid->tile_y;
        if (tx % g.vx) g.vx = 1;
        if (tx == 0 && !measured_tile(grid->scheme, grid->layout, grid->precision, nx, tx, ty))
            choose_tile(nx, max_threads, g.vx, tx, ty);
        if (grid->tile_x == 0 && g.fw && tx * ty > 256) ty = 256 / tx; // the full-way pull's direct kernel
        g.tx = tx;
        g.ty = ty;
    } else {
        g.tx = g.ty = 1;
    }
    g.ntx = (int32_t)((nx + g.tx - 1) / g.tx);
    g.nty = (int32_t)((ny + g.ty - 1) / g.ty);
    if (tiled && (int64_t)g.ntx * g.nty > 0x7fffffffll) return bad("too many tiles");
    // t / ntx == umulhi(t, ceil(2^32 / ntx)) whenever t * (ntx - 1) < 2^32
    g.ntx_rcp = 0;
    if (g.ntx >= 2 && ((uint64_t)g.ntx * g.nty - 1) * (uint64_t)(g.ntx - 1) < ((uint64_t)1 << 32))
        g.ntx_rcp = (uint32_t)((((uint64_t)1 << 32) + g.ntx - 1) / g.ntx);
    if (lattice_elems(g, grid->layout) > (int64_t)(SIZE_MAX / 8)) return bad("lattice size overflows");

    Physics& ph = kp.ph;
    ph.omc = (float)(1.0 - 1.0 / tau);
    for (int i = 0; i < 9; ++i)
        ph.F[i] = (float)(3.0 * kW[i] * (dir_cx(i) * bc->g[0] + dir_cy(i) * bc->g[1]));
    shifted_feq(bc->u_in[0], bc->u_in[1], ph.ein);
    shifted_feq(bc->u0[0], bc->u0[1], ph.e0);
    ph.hg[0] = (float)(0.5 * bc->g[0]);
    ph.hg[1] = (float)(0.5 * bc->g[1]);
    ph.u_in[0] = (float)bc->u_in[0];
    ph.u_in[1] = (float)bc->u_in[1];
    kp.types = nullptr;
    return LBM_OK;
}

int64_t lbm::lattice_elems(const Geometry& g, int layout)
{
    return layout == LBM_COLLISION ? 9 * g.px * g.ny : 9 * g.P;
}

// ------------------------------------------------ fixed scratch (no allocation)
// Device memory for lbm_diag_noalloc: the reduction partials and sums of the
// diagnostics (diag_partials() + 8 doubles, 41 KB), a file-scope array that
// each GPU holds for the life of the process.  Host code never passes the
// array's name to a kernel: on the host it stands for the symbol, not for a
// device address.  Each device's address is looked up once, with that device
// current, and kept.  Every call on a device shares its array, so calls that
// overlap on one device race on it.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = 5120 + 8;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

lbm_status noalloc_scratch(lbm_ctx* c, double** out)
{
    if (c->device < 0 || c->device >= NOALLOC_MAX_DEVICES) return c->fail(LBM_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess) return c->fail(LBM_EDEVICE, "hipGetDevice failed");
        if (cur != c->device && hipSetDevice(c->device) != hipSuccess)
            return c->fail(LBM_EDEVICE, "hipSetDevice failed");
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != c->device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return c->fail(LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[c->device] = (double*)p;
    }
    *out = g_scratch_ptr[c->device];
    return LBM_OK;
}
} // namespace

int64_t lbm::count_updated(const lbm_grid* grid, const uint8_t* flags, const lbm_bc* bc)
{
    int64_t n = 0;
    for (int64_t y = 0; y < grid->ny; ++y)
        for (int64_t x = 0; x < grid->nx; ++x)
            if (!flags[y * grid->nx + x] && !(is_inout(bc->x_axis) && x == 0)) ++n;
    return n;
}

extern "C" {

int32_t lbm_bytes_per_update(int32_t precision) { return precision == LBM_FP32 ? 72 : 36; }

lbm_status lbm_create(const lbm_grid* grid, const uint8_t* flags, double tau, const lbm_bc* bc, void* stream,
                      lbm_ctx** out)
{
    if (!out) return create_error(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    KParams kp{};
    std::string why;
    lbm_status vs = setup_params(grid, flags, tau, bc, kp, why);
    if (vs != LBM_OK) return create_error(vs, why);
    const int64_t nx = grid->nx, ny = grid->ny;
    const int64_t N = nx * ny;
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return create_error(LBM_ENOMEM, "host allocation failed");
    (void)hipGetDevice(&c->device);
    c->grid = *grid;
    c->bc = *bc;
    c->tau = tau;
    c->state = state_of(grid->scheme);
    c->elem = grid->precision == LBM_FP32 ? 4 : 2;
    c->kp = kp;
    const Geometry& g = c->kp.g;
    c->lat_elems = lattice_elems(g, grid->layout);
    c->edge_elems = has_buffer_grid(grid->scheme) ? edge_x_elems(g) + edge_y_elems(g) : 0;
    c->fluid = count_updated(grid, flags, bc);

    // streams
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return create_error(LBM_EDEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        free_all(c);
        delete c;
        return create_error(LBM_EDEVICE, "hipStreamCreate failed");
    }

    // all-or-nothing allocation
    const size_t lat_bytes = (size_t)c->lat_elems * c->elem;
    c->guard = lattice_guard(g);
    const size_t raw_bytes = lat_bytes + 2 * (size_t)c->guard * c->elem;
    lbm_status st = alloc(c, &c->lat_raw[0], raw_bytes);
    if (st == LBM_OK && is_two_lattice(grid->scheme)) st = alloc(c, &c->lat_raw[1], raw_bytes);
    for (int k = 0; k < 2; ++k)
        if (c->lat_raw[k]) c->lat[k] = (char*)c->lat_raw[k] + (size_t)c->guard * c->elem;
    if (st == LBM_OK && c->edge_elems) st = alloc(c, &c->edge[0], (size_t)c->edge_elems * c->elem);
    if (st == LBM_OK && c->edge_elems) st = alloc(c, &c->edge[1], (size_t)c->edge_elems * c->elem);
    if (st == LBM_OK && grid->scheme == S_AA && is_inout(bc->x_axis))
        st = alloc(c, &c->obuf, (size_t)(3 * ny) * c->elem);
    if (st == LBM_OK && is_neumann_inlet(bc->x_axis)) st = alloc(c, (void**)&c->rin, (size_t)(2 * ny) * sizeof(float));
    if (st == LBM_OK) st = alloc(c, (void**)&c->types, (size_t)(g.px * ny));
    if (st == LBM_OK) st = alloc(c, (void**)&c->links, (size_t)(g.px * ny) * sizeof(uint32_t));
    uint8_t* dflags = nullptr;
    if (st == LBM_OK && hipMalloc(&dflags, (size_t)N) != hipSuccess) {
        dflags = nullptr;
        st = LBM_ENOMEM;
    }
    if (st != LBM_OK) {
        free_all(c);
        delete c;
        return create_error(LBM_ENOMEM, "device memory exhausted");
    }
    c->kp.types = c->types;
    c->kp.links = c->links;

    hipError_t e = hipMemcpyAsync(dflags, flags, (size_t)N, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_types(g, dflags, c->types, c->stream);
    if (e == hipSuccess) e = launch_links(g, c->types, c->links, c->stream);
    for (int k = 0; k < 2; ++k) // guards included: what a speculative load reads there is defined
        if (e == hipSuccess && c->lat_raw[k]) e = hipMemsetAsync(c->lat_raw[k], 0, raw_bytes, c->stream);
    if (e == hipSuccess) e = launch_init(c->state, grid->layout, grid->precision, c->kp, c->lat[0], c->stream);
    if (e == hipSuccess && c->edge_elems) {
        e = launch_edge_fill(c->state, grid->layout, grid->precision, c->kp, c->lat[0], c->edge[0], c->stream);
        if (e == hipSuccess) e = hipMemsetAsync(c->edge[1], 0, (size_t)c->edge_elems * c->elem, c->stream);
    }
    if (e == hipSuccess && c->rin) e = hipMemsetAsync(c->rin, 0, (size_t)(2 * ny) * sizeof(float), c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    (void)hipFree(dflags);
    if (e != hipSuccess) {
        std::string msg = std::string("initialisation failed: ") + hipGetErrorString(e);
        free_all(c);
        delete c;
        return create_error(LBM_EDEVICE, msg);
    }
    c->block = grid->scheme == LBM_LPTL ? lptl_block_size(grid->layout, grid->precision)
                                        : (g.tx / g.vx) * g.ty;
    *out = c;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n)
{
    if (!c) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    if (n < 0) return c->fail(LBM_EINVAL, "negative step count");
    while (n > 0) {
        const int parity = (int)(c->t & 1);
        if (c->bundle > 0 && n >= c->bundle) {
            if (!c->gexec[parity]) {
                lbm_status st = build_graph(c, parity);
                if (st != LBM_OK) return st;
            }
            lbm_status st = c->check(hipGraphLaunch(c->gexec[parity], c->stream), "hipGraphLaunch");
            if (st != LBM_OK) return st;
            c->t += c->bundle;
            n -= c->bundle;
        } else {
            lbm_status st = launch_one(c, parity, c->stream);
            if (st != LBM_OK) return st;
            c->t += 1;
            n -= 1;
        }
    }
    return LBM_OK;
}

lbm_status lbm_set_bundle(lbm_ctx* c, int32_t k)
{
    if (!c) return LBM_EINVAL;
    if (k < 0 || k > 4096) return c->fail(LBM_EINVAL, "bundle must be in [0, 4096]");
    if (k != c->bundle) {
        lbm_status st = c->check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
        if (st != LBM_OK) return st;
        drop_graphs(c);
        c->bundle = k;
    }
    return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx* c)
{
    if (!c) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    return c->check(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
}

lbm_status lbm_macros(lbm_ctx* c, float* rho, float* u, int on_device)
{
    if (!c) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    if (!rho && !u) return LBM_OK;
    const int64_t N = c->grid.nx * c->grid.ny;
    if (on_device) {
        return c->check(launch_macros(c->state_now(), c->grid.layout, c->grid.precision, c->view(), c->cur_lat(), rho, u,
                                      c->stream),
                        "macros launch");
    }
    lbm_status st = ensure_readout(c);
    if (st != LBM_OK) return st;
    float* drho = c->readout;
    float* du = c->readout + N;
    hipError_t e = launch_macros(c->state_now(), c->grid.layout, c->grid.precision, c->view(), c->cur_lat(), drho, du, c->stream);
    if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, drho, N * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && u) e = hipMemcpyAsync(u, du, 2 * N * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return c->check(e, "macros readout");
}

lbm_status lbm_get_populations(lbm_ctx* c, float* f, int on_device)
{
    if (!c || !f) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    const int64_t N = c->grid.nx * c->grid.ny;
    if (on_device)
        return c->check(launch_get_populations(c->state_now(), c->grid.layout, c->grid.precision, c->view(), c->cur_lat(), f,
                                               c->stream),
                        "populations launch");
    lbm_status st = ensure_readout(c);
    if (st != LBM_OK) return st;
    hipError_t e = launch_get_populations(c->state_now(), c->grid.layout, c->grid.precision, c->view(), c->cur_lat(),
                                          c->readout, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(f, c->readout, 9 * N * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return c->check(e, "populations readout");
}

lbm_status lbm_set_state(lbm_ctx* c, const float* f, int on_device)
{
    if (!c || !f) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    const int64_t N = c->grid.nx * c->grid.ny;
    const float* src = f;
    if (!on_device) {
        lbm_status st = ensure_readout(c);
        if (st != LBM_OK) return st;
        hipError_t e = hipMemcpyAsync(c->readout, f, 9 * N * sizeof(float), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return c->check(e, "state upload");
        src = c->readout;
    }
    // the push state is built from the pull form through a second lattice;
    // AA, which has one, borrows a temporary one
    void* tmp = c->other_lat();
    const bool borrow = c->state_now() == ST_PUSH && !tmp;
    if (borrow && hipMalloc(&tmp, (size_t)c->lat_elems * c->elem) != hipSuccess)
        return c->fail(LBM_ENOMEM, "temporary lattice for the state load");
    hipError_t e = hipSuccess;
    if (c->rin) e = launch_inlet_density_fill(c->kp, src, c->rin + (c->t & 1) * c->grid.ny, c->stream);
    if (e == hipSuccess)
        e = launch_set_state(c->state_now(), c->grid.layout, c->grid.precision, c->view(), src, c->cur_lat(), tmp,
                             c->stream);
    if (e == hipSuccess && c->edge_elems)
        e = launch_edge_fill(c->state_now(), c->grid.layout, c->grid.precision, c->view(), c->cur_lat(),
                             c->edge[c->t & 1], c->stream);
    if (e == hipSuccess && c->obuf && c->state_now() == ST_SWAP)
        e = launch_aa_outlet_fill(c->grid.layout, c->grid.precision, c->view(), c->cur_lat(), c->obuf, c->stream);
    if (borrow) {
        const hipError_t e2 = hipStreamSynchronize(c->stream);
        (void)hipFree(tmp);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->stream);
    c->have_prev = false;
    return c->check(e, "state load");
}

lbm_status lbm_diag(lbm_ctx* c, double out[4])
{
    if (!c || !out) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    const Geometry& g = c->kp.g;
    if (!c->u_prev) {
        if (alloc(c, (void**)&c->u_prev, (size_t)(2 * g.px * g.ny) * sizeof(double)) != LBM_OK)
            return c->fail(LBM_ENOMEM, "diagnostics buffer allocation failed");
    }
    if (!c->partials) {
        if (alloc(c, (void**)&c->partials, (size_t)diag_partials() * sizeof(double)) != LBM_OK)
            return c->fail(LBM_ENOMEM, "diagnostics buffer allocation failed");
    }
    if (!c->dout) {
        if (alloc(c, (void**)&c->dout, 8 * sizeof(double)) != LBM_OK)
            return c->fail(LBM_ENOMEM, "diagnostics buffer allocation failed");
    }
    double h[5];
    hipError_t e = launch_diag(c->state_now(), c->grid.layout, c->grid.precision, c->view(), c->cur_lat(), c->u_prev,
                               c->have_prev ? 1 : 0, c->partials, c->dout, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h, c->dout, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    lbm_status st = c->check(e, "diagnostics");
    if (st != LBM_OK) return st;
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[2];
    out[3] = c->have_prev ? (h[4] > 0 ? std::sqrt(h[3]) / std::sqrt(h[4]) : 0.0) : -1.0;
    c->have_prev = true;
    if (!std::isfinite(h[0]) || !std::isfinite(h[1]) || !std::isfinite(h[2])) {
        c->err = "non-finite mass or momentum";
        return LBM_EUNSTABLE;
    }
    return LBM_OK;
}

lbm_status lbm_diag_noalloc(lbm_ctx* c, double* u_prev, int32_t have_prev, double* out)
{
    if (!c || !out || (have_prev && !u_prev)) return LBM_EINVAL;
    if (c->poisoned) return LBM_EDEVICE;
    const size_t need = (size_t)diag_partials() + 8;
    if (need > NOALLOC_SCRATCH_DOUBLES)
        return c->fail(LBM_EINVAL, "diagnostics need " + std::to_string(need) + " doubles of scratch, the fixed "
                                       "array holds " + std::to_string(NOALLOC_SCRATCH_DOUBLES));
    double* scr = nullptr;
    lbm_status st = noalloc_scratch(c, &scr);
    if (st != LBM_OK) return st;
    double* sums = scr + diag_partials(); // 5 sums after the partials
    hipError_t e = launch_diag(c->state_now(), c->grid.layout, c->grid.precision, c->view(), c->cur_lat(), u_prev,
                               have_prev ? 1 : 0, scr, sums, c->stream);
    if (e == hipSuccess) e = launch_diag_result(sums, have_prev ? 1 : 0, out, c->stream);
    return c->check(e, "diagnostics launch");
}

lbm_status lbm_get_info(const lbm_ctx* c, lbm_info* info)
{
    if (!c || !info) return LBM_EINVAL;
    info->steps = c->t;
    info->nx = c->grid.nx;
    info->ny = c->grid.ny;
    info->pitch = c->kp.g.px;
    info->scheme = c->grid.scheme;
    info->layout = c->grid.layout;
    info->precision = c->grid.precision;
    info->tile_x = c->grid.scheme == LBM_LPTL ? 0 : c->kp.g.tx;
    info->tile_y = c->grid.scheme == LBM_LPTL ? 0 : c->kp.g.ty;
    info->block = c->block;
    info->bundle = c->bundle;
    info->device_bytes = c->bytes;
    info->fluid_nodes = c->fluid;
    return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

lbm_status lbm_bandwidth_probe(int32_t mode, void* dst, const void* src, int64_t bytes, void* stream)
{
    if (mode < 0 || mode > 3 || bytes <= 0 || (bytes % 16) != 0) return LBM_EINVAL;
    if ((mode != 1 && (!dst || ((uintptr_t)dst % 16))) || (mode != 2 && (!src || ((uintptr_t)src % 16))))
        return LBM_EINVAL;
    if (mode == 1 && !dst) return LBM_EINVAL;
    hipError_t e = launch_probe(mode, dst, src, bytes, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

} // extern "C"
