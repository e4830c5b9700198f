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
//   - retirement: a request that reached its step count has its macroscopic
//     fields read back, its slot and memory freed, and is reported by poll.
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
    int32_t tiles = 0;
    int state = Q_QUEUED;
    int slot = -1;
    int64_t off = -1;
    int64_t steps_done = 0;
    int32_t status = LBM_OK;
    std::vector<float> rho, u;
};

constexpr int64_t ALIGN = 256;
int64_t align_up(int64_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

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
    SlotDesc* h_slots = nullptr; // pinned staging
    WorkItem* h_work = nullptr;
    int32_t* h_nwork = nullptr;
    int64_t work_cap = 0;
    int64_t tiles_resident = 0;
    std::vector<Request*> slot_req;
    std::deque<Request*> queue;
    std::unordered_map<uint64_t, Request*> reqs;
    std::vector<uint64_t> unreported;
    uint64_t next_id = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipEvent_t ev = nullptr;
    bool in_flight = false;
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

// Read back rho and u of a request that reached its step count, then free its
// slot and memory.  Non-finite results mark the request LBM_EUNSTABLE.
lbm_status retire(lbm_server* s, Request* r)
{
    const Geometry& g = r->kp.g;
    const int64_t N = g.nx * g.ny;
    char* base = s->pool + r->off;
    void* cur = base + ((r->steps_done & 1) ? r->lat_bytes : 0);
    float* scratch = (float*)(base + ((r->steps_done & 1) ? 0 : r->lat_bytes)); // the other lattice
    r->rho.resize(N);
    r->u.resize(2 * N);
    KParams p = r->kp;
    if (r->rin2) p.rin = r->rin2 + (r->steps_done & 1) * g.ny;
    hipError_t e = launch_macros(ST_PULL, s->layout, s->precision, p, cur, scratch, scratch + N, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->rho.data(), scratch, N * sizeof(float), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->u.data(), scratch + N, 2 * N * sizeof(float), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->check(e, "request readout");
    r->status = LBM_OK;
    for (int64_t k = 0; k < 2 * N && r->status == LBM_OK; ++k)
        if (!std::isfinite(r->u[k])) r->status = LBM_EUNSTABLE;
    release(s, r);
    r->state = Q_DONE;
    s->unreported.push_back(r->id);
    return LBM_OK;
}

// Account for a finished bundle (blocking: wait for it).
lbm_status complete_bundle(lbm_server* s, bool blocking)
{
    if (!s->in_flight) return LBM_OK;
    if (blocking) {
        lbm_status st = s->check(hipEventSynchronize(s->ev), "hipEventSynchronize");
        if (st != LBM_OK) return st;
    } else {
        hipError_t q = hipEventQuery(s->ev);
        if (q == hipErrorNotReady) return LBM_OK;
        if (q != hipSuccess) return s->check(q, "hipEventQuery");
    }
    s->in_flight = false;
    for (int k = 0; k < s->max_slots; ++k) {
        Request* r = s->slot_req[k];
        if (!r) continue;
        const int64_t adv = std::min<int64_t>(s->K, r->steps - r->steps_done);
        r->steps_done += adv;
        s->node_updates += adv * r->kp.g.nx * r->kp.g.ny;
        if (r->steps_done >= r->steps) {
            lbm_status st = retire(s, r);
            if (st != LBM_OK) return st;
        }
    }
    return LBM_OK;
}

lbm_status admit(lbm_server* s, Request* r, int slot)
{
    char* base = s->pool + r->off;
    const Geometry& g = r->kp.g;
    uint8_t* types = (uint8_t*)(base + 2 * r->lat_bytes);
    uint8_t* dflags = types + align_up(g.px * g.ny);
    r->kp.types = types;
    const bool neumann = r->bc.x_axis == LBM_NEUMANN_OUTFLOW || r->bc.x_axis == LBM_NEUMANN_PRESSURE;
    r->rin2 = neumann ? (float*)(dflags + align_up(g.nx * g.ny)) : nullptr;
    hipError_t e =
        hipMemcpyAsync(dflags, r->flags.data(), (size_t)(g.nx * g.ny), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && r->rin2) e = hipMemsetAsync(r->rin2, 0, (size_t)(2 * g.ny) * sizeof(float), s->stream);
    if (e == hipSuccess) e = launch_types(g, dflags, types, s->stream);
    if (e == hipSuccess) e = launch_init(ST_PULL, s->layout, s->precision, r->kp, base, s->stream);
    if (e != hipSuccess) return s->check(e, "request initialisation");
    r->slot = slot;
    r->state = Q_RUNNING;
    s->slot_req[slot] = r;
    s->tiles_resident += r->tiles;
    return LBM_OK;
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
    if (hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess)
        return cleanup(LBM_EDEVICE, "hipEventCreate failed");
    if (hipMalloc((void**)&s->pool, (size_t)s->budget) != hipSuccess) {
        s->pool = nullptr;
        (void)hipGetLastError();
        return cleanup(LBM_ENOMEM, "cannot allocate the HBM budget");
    }
    s->free_list[0] = s->budget;
    if (hipMalloc((void**)&s->d_slots, sizeof(SlotDesc) * max_slots) != hipSuccess ||
        hipMalloc((void**)&s->d_work, sizeof(WorkItem) * s->work_cap) != hipSuccess ||
        hipMalloc((void**)&s->d_nwork, sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc((void**)&s->h_slots, sizeof(SlotDesc) * max_slots, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s->h_work, sizeof(WorkItem) * s->work_cap, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s->h_nwork, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(LBM_ENOMEM, "cannot allocate the descriptor tables");
    }
    std::memset(s->h_slots, 0, sizeof(SlotDesc) * max_slots);
    *s->h_nwork = 0;
    if (hipMemcpy(s->d_slots, s->h_slots, sizeof(SlotDesc) * max_slots, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_nwork, s->h_nwork, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(LBM_EDEVICE, "descriptor upload failed");
    s->blocks = batched_blocks(layout, precision);

    // the bundle: K launches, launch k advancing every slot with k < steps_left
    if (hipStreamBeginCapture(s->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return cleanup(LBM_EDEVICE, "hipStreamBeginCapture failed");
    hipError_t e = hipSuccess;
    for (int k = 0; k < s->K && e == hipSuccess; ++k)
        e = launch_batched(layout, precision, s->d_slots, s->d_work, s->d_nwork, k, s->blocks, s->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return cleanup(LBM_EDEVICE, "bundle capture failed");
    }
    s->graph = g;
    if (hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0) != hipSuccess)
        return cleanup(LBM_EDEVICE, "bundle instantiation failed");
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
    r->footprint = 2 * r->lat_bytes + align_up(g.px * g.ny) + align_up(g.nx * g.ny);
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
    lbm_status st = complete_bundle(s, true);
    if (st != LBM_OK) return st;
    // admission in arrival order with backfill
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
        st = admit(s, r, slot);
        if (st != LBM_OK) return st;
        it = s->queue.erase(it);
    }
    // descriptors and work list of the resident requests
    int32_t nw = 0;
    for (int k = 0; k < s->max_slots; ++k) {
        Request* r = s->slot_req[k];
        SlotDesc& d = s->h_slots[k];
        if (!r) {
            d.steps_left = 0;
            continue;
        }
        char* base = s->pool + r->off;
        d.lat[0] = base;
        d.lat[1] = base + r->lat_bytes;
        d.types = r->kp.types;
        d.rin2 = r->rin2;
        d.g = r->kp.g;
        d.ph = r->kp.ph;
        d.steps_done = r->steps_done;
        d.steps_left = r->steps - r->steps_done;
        for (int32_t t = 0; t < r->tiles; ++t) s->h_work[nw++] = WorkItem{k, t};
    }
    *s->h_nwork = nw;
    hipError_t e = hipMemcpyAsync(s->d_slots, s->h_slots, sizeof(SlotDesc) * s->max_slots, hipMemcpyHostToDevice,
                                  s->stream);
    if (e == hipSuccess && nw > 0)
        e = hipMemcpyAsync(s->d_work, s->h_work, sizeof(WorkItem) * nw, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d_nwork, s->h_nwork, sizeof(int32_t), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess && nw > 0) e = hipGraphLaunch(s->gexec, s->stream);
    if (e == hipSuccess) e = hipEventRecord(s->ev, s->stream);
    st = s->check(e, "bundle launch");
    if (st != LBM_OK) return st;
    s->in_flight = true;
    if (nw > 0) ++s->bundles;
    return LBM_OK;
}

lbm_status lbm_server_poll(lbm_server* s, uint64_t* ids, int32_t* status, int32_t cap, int32_t* n)
{
    if (!s || !n || cap < 0 || (cap > 0 && (!ids || !status))) return LBM_EINVAL;
    if (s->poisoned) return LBM_EDEVICE;
    lbm_status st = complete_bundle(s, false);
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
    out->running = running;
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
    if (s->gexec) (void)hipGraphExecDestroy(s->gexec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    if (s->ev) (void)hipEventDestroy(s->ev);
    if (s->pool) (void)hipFree(s->pool);
    if (s->d_slots) (void)hipFree(s->d_slots);
    if (s->d_work) (void)hipFree(s->d_work);
    if (s->d_nwork) (void)hipFree(s->d_nwork);
    if (s->h_slots) (void)hipHostFree(s->h_slots);
    if (s->h_work) (void)hipHostFree(s->h_work);
    if (s->h_nwork) (void)hipHostFree(s->h_nwork);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

} // extern "C"
