// server.hip -- continuous-batching serving engine behind lbm_server_*.
//
// Independent simulation requests of different grid sizes share one GPU:
//   - memory: one pool of the HBM budget, carved first-fit per request
//     (two lattices + node types + flag staging + Neumann inlet densities);
//   - admission: at every bundle boundary, queued requests are admitted in
//     arrival order while a slot and pool space are free; a request that does
//     not fit yet lets later, smaller ones pass (backfill);
//   - compute: every bundle replays one captured HIP graph of K launches of
//     the batched kernel; the kernel reads the device descriptor table and
//     work list that the host rewrites between bundles, so the graph stays
//     valid while membership changes;
//   - retirement: the host knows at launch which requests a bundle finishes
//     (step counts are exact), so their readouts (macroscopic fields into a
//     pinned result arena) are enqueued right behind the bundle and their slots
//     and memory are free for the next admission at once -- stream order keeps
//     the readout ahead of any reuse.  A request is reported by poll once the
//     event after its bundle has passed.
//   - pipelining: up to two bundles are in flight; the host retires, admits and
//     writes the next descriptor table (double-buffered pinned staging) while
//     the device runs the previous bundle.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "lbm.h"
#include "lbm_batched.hpp"
#include "lbm_host.hpp"
#include "lbm_kernels.hpp"

using namespace lbm;

namespace {

enum ReqState { Q_QUEUED = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Request {
    uint64_t id = 0;
    lbm_grid grid{};
    lbm_bc bc{};
    double tau = 0;
    std::vector<uint8_t> flags;
    int64_t steps = 0;
    KParams kp{};
    float* rin2 = nullptr; // Neumann inlet: rho - 1 of column 1 per row, two halves by update parity
    int64_t lat_bytes = 0, footprint = 0;
    int64_t guard_bytes = 0; // zone before, between and after the two lattices (see lat_ptr)
    int32_t tiles = 0;
    int state = Q_QUEUED;
    int slot = -1;
    int64_t off = -1;
    int64_t steps_done = 0;
    int64_t res_off = -1; // its readout in the pinned result arena (while in flight)
    int32_t status = LBM_OK;
    std::vector<float> rho, u;
};

// A bundle in flight: its completion event, the requests it finishes (whose
// readouts follow it in the stream) and their region of the result arena.
struct InFlight {
    hipEvent_t ev = nullptr;
    std::vector<Request*> finishing;
    int64_t res_off = 0, res_bytes = 0;
    int64_t updates = 0; // node updates the bundle performs
};

constexpr int MAX_IN_FLIGHT = 2;

constexpr int64_t ALIGN = 256;
int64_t align_up(int64_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// A request's memory: guard, lattice 0, guard, lattice 1, guard, node types,
// flag staging, link words, Neumann inlet densities.  The guards (the
// lattice_guard of its geometry) keep every plain-neighbour load of an
// in-domain node inside the request's memory, so the batched kernel issues
// those loads before it knows whether the node is regular.
char* lat_ptr(char* pool, const Request* r, int k)
{
    return pool + r->off + r->guard_bytes + k * (r->lat_bytes + r->guard_bytes);
}

} // namespace

struct lbm_server {
    int32_t layout = 0, precision = 0, elem = 4;
    int32_t max_slots = 0, K = 0;
    int64_t budget = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap = nullptr;
    char* pool = nullptr;
    std::map<int64_t, int64_t> free_list; // offset -> size
    int64_t pool_used = 0;
    SlotDesc* d_slots = nullptr;
    WorkItem* d_work = nullptr;
    int32_t* d_nwork = nullptr;
    // pinned staging of the descriptor tables, two sets used by alternate
    // bundles (a set is rewritten only after the bundle that read it is done)
    SlotDesc* h_slots[2] = {nullptr, nullptr};
    WorkItem* h_work[2] = {nullptr, nullptr};
    int32_t* h_nwork[2] = {nullptr, nullptr};
    int stage = 0;
    std::deque<InFlight> flight; // oldest first
    std::vector<hipEvent_t> free_events;
    // pinned result arena, a ring of per-bundle regions freed in bundle order
    char* h_res = nullptr;
    int64_t res_cap = 0, res_head = 0, res_used = 0;
    int32_t finishing_pending = 0; // requests whose readout is in flight
    int64_t work_cap = 0;
    int64_t tiles_resident = 0;
    std::vector<Request*> slot_req;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> reqs;
    std::vector<uint64_t> unreported;
    uint64_t next_id = 1;
    // one captured bundle per persistent grid size: the full grid (resident
    // blocks on the device) and smaller ones down to 1/32 of it, so that a
    // bundle over few work items launches few blocks
    static constexpr int NGRIDS = 6;
    hipGraph_t graph[NGRIDS] = {};
    hipGraphExec_t gexec[NGRIDS] = {};
    int grid_blocks[NGRIDS] = {};
    int blocks = 0;
    bool poisoned = false;
    std::string err;
    int64_t bundles = 0, node_updates = 0;

    lbm_status fail(lbm_status s, const std::string& m)
    {
        err = m;
        if (s == LBM_EDEVICE) poisoned = true;
        return s;
    }
    lbm_status check(hipError_t e, const char* what)
    {
        if (e == hipSuccess) return LBM_OK;
        return fail(LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
};

namespace {

thread_local std::string g_server_create_error;

int64_t pool_alloc(lbm_server* s, int64_t bytes)
{
    bytes = align_up(bytes);
    for (auto it = s->free_list.begin(); it != s->free_list.end(); ++it) {
        if (it->second >= bytes) {
            const int64_t off = it->first, rest = it->second - bytes;
            s->free_list.erase(it);
            if (rest > 0) s->free_list[off + bytes] = rest;
            s->pool_used += bytes;
            return off;
        }
    }
    return -1;
}

void pool_free(lbm_server* s, int64_t off, int64_t bytes)
{
    bytes = align_up(bytes);
    s->pool_used -= bytes;
    auto it = s->free_list.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != s->free_list.end() && it->first + it->second == next->first) {
        it->second += next->second;
        s->free_list.erase(next);
    }
    if (it != s->free_list.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            s->free_list.erase(it);
        }
    }
}

void release(lbm_server* s, Request* r)
{
    if (r->off >= 0) pool_free(s, r->off, r->footprint);
    r->off = -1;
    if (r->slot >= 0) {
        s->slot_req[r->slot] = nullptr;
        s->tiles_resident -= r->tiles;
    }
    r->slot = -1;
    r->flags.clear();
    r->flags.shrink_to_fit();
}

// Enqueue the readout of a request that the bundle just enqueued finishes:
// rho and u into its other lattice (free at this point), then into the pinned
// result arena at r->res_off; its slot and memory are released at once.
lbm_status enqueue_readout(lbm_server* s, Request* r)
{
    const Geometry& g = r->kp.g;
    const int64_t N = g.nx * g.ny;
    void* cur = lat_ptr(s->pool, r, (int)(r->steps & 1));
    float* scratch = (float*)lat_ptr(s->pool, r, (int)((r->steps & 1) ^ 1)); // the other lattice
    KParams p = r->kp;
    if (r->rin2) p.rin = r->rin2 + (r->steps & 1) * g.ny;
    hipError_t e = launch_macros(ST_PULL, s->layout, s->precision, p, cur, scratch, scratch + N, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_res + r->res_off, scratch, 3 * N * sizeof(float), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return s->check(e, "request readout");
    release(s, r);
    ++s->finishing_pending;
    return LBM_OK;
}

// Retire the oldest bundle in flight: wait for it (blocking) or return
// LBM_EBUSY if it is still running; move the results of the requests it
// finished out of the arena and report them.
lbm_status finish_oldest(lbm_server* s, bool blocking)
{
    if (s->flight.empty()) return LBM_OK;
    InFlight& b = s->flight.front();
    if (blocking) {
        lbm_status st = s->check(hipEventSynchronize(b.ev), "hipEventSynchronize");
        if (st != LBM_OK) return st;
    } else {
        const hipError_t q = hipEventQuery(b.ev);
        if (q == hipErrorNotReady) return LBM_EBUSY;
        if (q != hipSuccess) return s->check(q, "hipEventQuery");
    }
    for (Request* r : b.finishing) {
        const int64_t N = r->kp.g.nx * r->kp.g.ny;
        const float* res = (const float*)(s->h_res + r->res_off);
        r->rho.assign(res, res + N);
        r->u.assign(res + N, res + 3 * N);
        r->status = LBM_OK;
        for (int64_t k = 0; k < 2 * N && r->status == LBM_OK; ++k)
            if (!std::isfinite(r->u[k])) r->status = LBM_EUNSTABLE;
        r->res_off = -1;
        r->state = Q_DONE;
        s->unreported.push_back(r->id);
        --s->finishing_pending;
    }
    s->node_updates += b.updates;
    s->res_used -= b.res_bytes;
    s->free_events.push_back(b.ev);
    s->flight.pop_front();
    if (s->res_used == 0) s->res_head = 0;
    return LBM_OK;
}

// Retire every bundle that has completed, oldest first, without blocking.
lbm_status drain(lbm_server* s)
{
    while (!s->flight.empty()) {
        const lbm_status st = finish_oldest(s, false);
        if (st == LBM_EBUSY) return LBM_OK;
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

// A region of `bytes` in the result arena after the regions of the bundles in
// flight (a ring: regions are freed in the order they were taken).
bool res_take(lbm_server* s, int64_t bytes, int64_t& off)
{
    if (bytes == 0) {
        off = s->res_head;
        return true;
    }
    if (s->res_used + bytes > s->res_cap) return false;
    if (s->res_used == 0) {
        off = 0;
        s->res_head = bytes;
        s->res_used = bytes;
        return true;
    }
    int64_t tail = s->res_head; // start of the oldest region still in use
    for (const InFlight& b : s->flight)
        if (b.res_bytes > 0) {
            tail = b.res_off;
            break;
        }
    if (s->res_head > tail) { // in use: [tail, head)
        if (s->res_cap - s->res_head >= bytes) {
            off = s->res_head;
        } else if (tail >= bytes) {
            off = 0;
        } else {
            return false;
        }
    } else { // in use: [tail, cap) and [0, head)
        if (tail - s->res_head < bytes) return false;
        off = s->res_head;
    }
    s->res_head = off + bytes;
    s->res_used += bytes;
    return true;
}

// Host side of an admission: the request takes a slot; its memory was taken
// from the pool by the caller.
void claim(lbm_server* s, Request* r, int slot)
{
    const Geometry& g = r->kp.g;
    uint8_t* types = (uint8_t*)(lat_ptr(s->pool, r, 1) + r->lat_bytes + r->guard_bytes);
    uint8_t* dflags = types + align_up(g.px * g.ny);
    r->kp.types = types;
    // link words after the flag staging, then the Neumann inlet densities
    r->kp.links = (const uint32_t*)(dflags + align_up(g.nx * g.ny));
    const bool neumann = r->bc.x_axis == LBM_NEUMANN_OUTFLOW || r->bc.x_axis == LBM_NEUMANN_PRESSURE;
    r->rin2 = neumann ? (float*)((char*)r->kp.links + align_up(g.px * g.ny * (int64_t)sizeof(uint32_t))) : nullptr;
    r->slot = slot;
    r->state = Q_RUNNING;
    s->slot_req[slot] = r;
    s->tiles_resident += r->tiles;
}

// Device side of an admission, enqueued ahead of the request's first bundle:
// flags (staged in the pinned arena at `staged`) -> node types, initial state.
lbm_status upload(lbm_server* s, Request* r, char* staged)
{
    const Geometry& g = r->kp.g;
    uint8_t* dflags = (uint8_t*)r->kp.types + align_up(g.px * g.ny);
    std::memcpy(staged, r->flags.data(), (size_t)(g.nx * g.ny));
    r->flags.clear();
    r->flags.shrink_to_fit();
    hipError_t e = hipMemcpyAsync(dflags, staged, (size_t)(g.nx * g.ny), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && r->rin2) e = hipMemsetAsync(r->rin2, 0, (size_t)(2 * g.ny) * sizeof(float), s->stream);
    if (e == hipSuccess) e = launch_types(g, dflags, (uint8_t*)r->kp.types, s->stream);
    if (e == hipSuccess) e = launch_links(g, r->kp.types, (uint32_t*)r->kp.links, s->stream);
    if (e == hipSuccess) e = launch_init(ST_PULL, s->layout, s->precision, r->kp, lat_ptr(s->pool, r, 0), s->stream);
    return s->check(e, "request initialisation");
}

} // namespace

extern "C" {

lbm_status lbm_server_create(int64_t hbm_budget_bytes, int32_t max_slots, int32_t bundle_steps, int32_t layout,
                             int32_t precision, void* stream, lbm_server** out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    auto bad = [](const char* m) {
        g_server_create_error = m;
        return LBM_EINVAL;
    };
    if (hbm_budget_bytes < (1 << 20)) return bad("hbm_budget_bytes must be at least 1 MiB");
    if (max_slots < 1 || max_slots > 65536) return bad("max_slots must be in [1, 65536]");
    if (bundle_steps < 1 || bundle_steps > 4096) return bad("bundle_steps must be in [1, 4096]");
    if (layout < LBM_STREAM || layout > LBM_COLLISION) return bad("unknown layout");
    if (precision < LBM_FP32 || precision > LBM_FP16C_SR) return bad("unknown precision");

    lbm_server* s = new (std::nothrow) lbm_server();
    if (!s) return LBM_ENOMEM;
    s->layout = layout;
    s->precision = precision;
    s->elem = precision == LBM_FP32 ? 4 : 2;
    s->max_slots = max_slots;
    s->K = bundle_steps;
    s->budget = hbm_budget_bytes / ALIGN * ALIGN;
    s->slot_req.assign(max_slots, nullptr);
    // A full 64 x 4 tile needs >= 256 * (18 * elem + 1) bytes of pool; ragged
    // edge tiles are bounded per request.
    s->work_cap = 2 * (s->budget / (256 * (18 * s->elem + 1))) + 1024 * (int64_t)max_slots + 1024;

    auto cleanup = [&](lbm_status st, const char* m) {
        lbm_server_destroy(s);
        g_server_create_error = m;
        return st;
    };
    if (stream) {
        s->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
            return cleanup(LBM_EDEVICE, "hipStreamCreate failed");
        s->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) != hipSuccess)
        return cleanup(LBM_EDEVICE, "hipStreamCreate failed");
    for (int k = 0; k < MAX_IN_FLIGHT; ++k) {
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return cleanup(LBM_EDEVICE, "hipEventCreate failed");
        s->free_events.push_back(ev);
    }
    if (hipMalloc((void**)&s->pool, (size_t)s->budget) != hipSuccess) {
        s->pool = nullptr;
        (void)hipGetLastError();
        return cleanup(LBM_ENOMEM, "cannot allocate the HBM budget");
    }
    s->free_list[0] = s->budget;
    bool ok = hipMalloc((void**)&s->d_slots, sizeof(SlotDesc) * max_slots) == hipSuccess &&
              hipMalloc((void**)&s->d_work, sizeof(WorkItem) * s->work_cap) == hipSuccess &&
              hipMalloc((void**)&s->d_nwork, sizeof(int32_t)) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k)
        ok = hipHostMalloc((void**)&s->h_slots[k], sizeof(SlotDesc) * max_slots, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc((void**)&s->h_work[k], sizeof(WorkItem) * s->work_cap, hipHostMallocDefault) ==
                 hipSuccess &&
             hipHostMalloc((void**)&s->h_nwork[k], sizeof(int32_t), hipHostMallocDefault) == hipSuccess;
    // result arena: grows on demand (only while nothing is in flight)
    s->res_cap = std::min<int64_t>(s->budget, (int64_t)64 << 20);
    ok = ok && hipHostMalloc((void**)&s->h_res, (size_t)s->res_cap, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return cleanup(LBM_ENOMEM, "cannot allocate the descriptor tables");
    }
    for (int k = 0; k < 2; ++k) {
        std::memset(s->h_slots[k], 0, sizeof(SlotDesc) * max_slots);
        *s->h_nwork[k] = 0;
    }
    if (hipMemcpy(s->d_slots, s->h_slots[0], sizeof(SlotDesc) * max_slots, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_nwork, s->h_nwork[0], sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(LBM_EDEVICE, "descriptor upload failed");
    s->blocks = batched_blocks(layout, precision);

    // the bundle: K launches, launch k advancing every slot with k < steps_left
    for (int v = 0; v < lbm_server::NGRIDS; ++v) {
        s->grid_blocks[v] = std::max(1, s->blocks >> v);
        if (hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return cleanup(LBM_EDEVICE, "hipStreamBeginCapture failed");
        hipError_t e = hipSuccess;
        for (int k = 0; k < s->K && e == hipSuccess; ++k)
            e = launch_batched(layout, precision, s->d_slots, s->d_work, s->d_nwork, k, s->grid_blocks[v], s->cap);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(s->cap, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return cleanup(LBM_EDEVICE, "bundle capture failed");
        }
        s->graph[v] = g;
        if (hipGraphInstantiate(&s->gexec[v], g, nullptr, nullptr, 0) != hipSuccess)
            return cleanup(LBM_EDEVICE, "bundle instantiation failed");
    }
    *out = s;
    return LBM_OK;
}

lbm_status lbm_server_submit(lbm_server* s, const lbm_grid* grid, const uint8_t* flags, double tau,
                             const lbm_bc* bc, int64_t steps, uint64_t* id)
{
    if (!s || !grid || !flags || !bc || !id) return LBM_EINVAL;
    if (s->poisoned) return LBM_EDEVICE;
    if (steps < 0) return s->fail(LBM_EINVAL, "negative step count");
    if (bc->bounce != LBM_HALFWAY) return s->fail(LBM_EINVAL, "served requests use halfway bounce-back");
    lbm_grid rg = *grid;
    rg.scheme = LBM_NPTL;
    rg.layout = s->layout;
    rg.precision = s->precision;
    rg.tile_x = BATCH_TILE_X;
    rg.tile_y = BATCH_TILE_Y;
    Request* r = new (std::nothrow) Request();
    if (!r) return LBM_ENOMEM;
    std::string why;
    lbm_status st = setup_params(&rg, flags, tau, bc, r->kp, why);
    if (st != LBM_OK) {
        delete r;
        return s->fail(st, why);
    }
    const Geometry& g = r->kp.g;
    r->grid = rg;
    r->bc = *bc;
    r->tau = tau;
    r->steps = steps;
    r->lat_bytes = align_up(lattice_elems(g, s->layout) * s->elem);
    r->guard_bytes = align_up(lattice_guard(g) * s->elem);
    r->footprint = 2 * r->lat_bytes + 3 * r->guard_bytes + align_up(g.px * g.ny) + align_up(g.nx * g.ny) +
                   align_up(g.px * g.ny * (int64_t)sizeof(uint32_t));
    if (bc->x_axis == LBM_NEUMANN_OUTFLOW || bc->x_axis == LBM_NEUMANN_PRESSURE)
        r->footprint += align_up(2 * g.ny * (int64_t)sizeof(float));
    r->tiles = g.ntx * g.nty;
    if (r->footprint > s->budget || r->tiles > s->work_cap) {
        delete r;
        return s->fail(LBM_ENOMEM, "request footprint exceeds the server's HBM budget");
    }
    r->flags.assign(flags, flags + g.nx * g.ny);
    r->id = s->next_id++;
    s->reqs[r->id] = r;
    s->queue.push_back(r);
    *id = r->id;
    return LBM_OK;
}

lbm_status lbm_server_run_bundle(lbm_server* s)
{
    if (!s) return LBM_EINVAL;
    if (s->poisoned) return LBM_EDEVICE;
    lbm_status st = drain(s);
    if (st != LBM_OK) return st;
    // the staging set of this bundle was read by the bundle two launches ago
    while ((int)s->flight.size() >= MAX_IN_FLIGHT) {
        st = finish_oldest(s, true);
        if (st != LBM_OK) return st;
    }
    // admission in arrival order with backfill
    std::vector<Request*> admitted;
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request* r = *it;
        if (r->steps == 0) { // nothing to do: report at once
            r->state = Q_DONE;
            r->status = LBM_OK;
            const int64_t N = r->kp.g.nx * r->kp.g.ny;
            r->rho.assign(N, 0.0f);
            r->u.assign(2 * N, 0.0f);
            s->unreported.push_back(r->id);
            it = s->queue.erase(it);
            continue;
        }
        int slot = -1;
        for (int k = 0; k < s->max_slots; ++k)
            if (!s->slot_req[k]) {
                slot = k;
                break;
            }
        if (slot < 0) break;
        if (s->tiles_resident + r->tiles > s->work_cap) {
            ++it;
            continue;
        }
        const int64_t off = pool_alloc(s, r->footprint);
        if (off < 0) {
            ++it;
            continue;
        }
        r->off = off;
        claim(s, r, slot);
        admitted.push_back(r);
        it = s->queue.erase(it);
    }
    // descriptors and work list of the resident requests
    SlotDesc* hs = s->h_slots[s->stage];
    WorkItem* hw = s->h_work[s->stage];
    int32_t nw = 0;
    InFlight b;
    int64_t res_bytes = 0;
    for (int k = 0; k < s->max_slots; ++k) {
        Request* r = s->slot_req[k];
        SlotDesc& d = hs[k];
        if (!r) {
            d.steps_left = 0;
            continue;
        }
        const Geometry& g = r->kp.g;
        d.lat[0] = lat_ptr(s->pool, r, 0);
        d.lat[1] = lat_ptr(s->pool, r, 1);
        d.types = r->kp.types;
        d.links = r->kp.links;
        d.rin2 = r->rin2;
        d.g = g;
        d.ph = r->kp.ph;
        d.steps_done = r->steps_done;
        d.steps_left = r->steps - r->steps_done;
        for (int32_t ty = 0; ty < g.nty; ++ty)
            for (int32_t tx = 0; tx < g.ntx; ++tx) hw[nw++] = WorkItem{k, tx * g.tx, ty * g.ty};
        const int64_t adv = std::min<int64_t>(s->K, d.steps_left);
        b.updates += adv * g.nx * g.ny;
        if (adv == d.steps_left) {
            r->res_off = res_bytes; // relative to the bundle's region for now
            res_bytes += 3 * g.nx * g.ny * (int64_t)sizeof(float);
            b.finishing.push_back(r);
        }
    }
    if (nw == 0) { // nothing resident: nothing to overlap, wait for what is in flight
        if (!s->flight.empty()) return finish_oldest(s, true);
        return LBM_OK;
    }
    // the bundle's arena region: staged flags of the admitted requests, then
    // the results of the finishing ones
    int64_t up_bytes = 0;
    for (Request* r : admitted) up_bytes += (r->kp.g.nx * r->kp.g.ny + 15) / 16 * 16;
    int64_t roff = 0;
    while (!res_take(s, up_bytes + res_bytes, roff)) {
        if (!s->flight.empty()) {
            st = finish_oldest(s, true);
            if (st != LBM_OK) return st;
            continue;
        }
        // nothing in flight and the arena is too small: grow it
        (void)hipHostFree(s->h_res);
        s->h_res = nullptr;
        s->res_cap = std::max<int64_t>(2 * s->res_cap, up_bytes + res_bytes);
        if (hipHostMalloc((void**)&s->h_res, (size_t)s->res_cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            s->res_cap = 0;
            return s->fail(LBM_ENOMEM, "cannot allocate the pinned result arena");
        }
    }
    b.res_off = roff;
    b.res_bytes = up_bytes + res_bytes;
    {
        int64_t o = roff;
        for (Request* r : admitted) {
            st = upload(s, r, s->h_res + o);
            if (st != LBM_OK) return st;
            o += (r->kp.g.nx * r->kp.g.ny + 15) / 16 * 16;
        }
    }
    *s->h_nwork[s->stage] = nw;
    hipError_t e = hipMemcpyAsync(s->d_slots, hs, sizeof(SlotDesc) * s->max_slots, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_work, hw, sizeof(WorkItem) * nw, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_nwork, s->h_nwork[s->stage], sizeof(int32_t), hipMemcpyHostToDevice, s->stream);
    // the smallest captured grid with at least one block per work item
    int v = 0;
    while (v + 1 < lbm_server::NGRIDS && s->grid_blocks[v + 1] >= nw) ++v;
    if (e == hipSuccess) e = hipGraphLaunch(s->gexec[v], s->stream);
    st = s->check(e, "bundle launch");
    if (st != LBM_OK) return st;
    for (Request* r : s->slot_req)
        if (r) r->steps_done += std::min<int64_t>(s->K, r->steps - r->steps_done);
    for (Request* r : b.finishing) {
        r->res_off += roff + up_bytes;
        st = enqueue_readout(s, r);
        if (st != LBM_OK) return st;
    }
    b.ev = s->free_events.back();
    s->free_events.pop_back();
    st = s->check(hipEventRecord(b.ev, s->stream), "hipEventRecord");
    if (st != LBM_OK) return st;
    s->flight.push_back(std::move(b));
    s->stage ^= 1;
    ++s->bundles;
    return LBM_OK;
}

lbm_status lbm_server_poll(lbm_server* s, uint64_t* ids, int32_t* status, int32_t cap, int32_t* n)
{
    if (!s || !n || cap < 0 || (cap > 0 && (!ids || !status))) return LBM_EINVAL;
    if (s->poisoned) return LBM_EDEVICE;
    lbm_status st = drain(s);
    if (st != LBM_OK) return st;
    int32_t k = 0;
    while (k < cap && !s->unreported.empty()) {
        const uint64_t id = s->unreported.front();
        s->unreported.erase(s->unreported.begin());
        ids[k] = id;
        status[k] = s->reqs.count(id) ? s->reqs[id]->status : LBM_ENOTFOUND;
        ++k;
    }
    *n = k;
    return LBM_OK;
}

lbm_status lbm_server_fetch(lbm_server* s, uint64_t id, float* rho, float* u)
{
    if (!s) return LBM_EINVAL;
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return s->fail(LBM_ENOTFOUND, "unknown request id");
    Request* r = it->second;
    if (r->state != Q_DONE) return s->fail(LBM_EBUSY, "request not finished");
    if (rho) std::memcpy(rho, r->rho.data(), r->rho.size() * sizeof(float));
    if (u) std::memcpy(u, r->u.data(), r->u.size() * sizeof(float));
    const lbm_status st = (lbm_status)r->status;
    s->reqs.erase(it);
    delete r;
    return st;
}

lbm_status lbm_server_get_stats(const lbm_server* s, lbm_server_stats* out)
{
    if (!s || !out) return LBM_EINVAL;
    out->queued = (int32_t)s->queue.size();
    int32_t running = 0;
    for (Request* r : s->slot_req)
        if (r) ++running;
    out->running = running + s->finishing_pending; // resident, or read back behind a bundle in flight
    int32_t done = 0;
    for (auto& kv : s->reqs)
        if (kv.second->state == Q_DONE) ++done;
    out->finished_unfetched = done;
    out->pool_bytes = s->budget;
    out->pool_used = s->pool_used;
    out->bundles = s->bundles;
    out->node_updates = s->node_updates;
    return LBM_OK;
}

const char* lbm_server_last_error(const lbm_server* s)
{
    if (!s) return g_server_create_error.c_str();
    return s->err.c_str();
}

void lbm_server_destroy(lbm_server* s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->reqs) delete kv.second;
    s->reqs.clear();
    for (int v = 0; v < lbm_server::NGRIDS; ++v) {
        if (s->gexec[v]) (void)hipGraphExecDestroy(s->gexec[v]);
        if (s->graph[v]) (void)hipGraphDestroy(s->graph[v]);
    }
    for (InFlight& b : s->flight) s->free_events.push_back(b.ev);
    s->flight.clear();
    for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
    if (s->pool) (void)hipFree(s->pool);
    if (s->d_slots) (void)hipFree(s->d_slots);
    if (s->d_work) (void)hipFree(s->d_work);
    if (s->d_nwork) (void)hipFree(s->d_nwork);
    for (int k = 0; k < 2; ++k) {
        if (s->h_slots[k]) (void)hipHostFree(s->h_slots[k]);
        if (s->h_work[k]) (void)hipHostFree(s->h_work[k]);
        if (s->h_nwork[k]) (void)hipHostFree(s->h_nwork[k]);
    }
    if (s->h_res) (void)hipHostFree(s->h_res);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

} // extern "C"
