// Serving pool (zm_pool_* in include/zm.h): continuous batching of
// simulation requests with admission by device-memory footprint.
//
// Workspace = [request budget | tables].  Requests get 256-byte aligned
// regions of the budget from a first-fit allocator with coalescing; each
// region has exactly the layout of a single-instance context.  The tables
// region holds the device descriptors, the pair work list, the work counters
// and one non-finite flag per live request; it is rewritten between
// iterations when membership changes.  An iteration is synchronous: it
// waits for its own kernels (the pool stream) to time them and to retire
// finished or failed requests before the next admission.
#include "zm.h"
#include "zm_batch_internal.h"
#include "zm_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

namespace {

constexpr int kMaxLive = 4096;
constexpr size_t kMaxItems = size_t(1) << 22;

struct TablesLayout {
    size_t desc, items, counters, flags, total;
};

TablesLayout tables_layout()
{
    TablesLayout t;
    size_t o = 0;
    t.desc = o;
    o = zm::align_up(o + sizeof(zm::InstDesc) * kMaxLive);
    t.items = o;
    o = zm::align_up(o + sizeof(zm::WorkItem) * kMaxItems);
    t.counters = o;
    o = zm::align_up(o + sizeof(int) * zm::kMaxPairGroups);
    t.flags = o;
    o = zm::align_up(o + sizeof(int) * kMaxLive);
    t.total = o;
    return t;
}

struct Request {
    zm_params prm;
    zm::PairShape shape;
    zm::Layout layout;
    size_t bytes = 0;
    size_t offset = 0;          // in the budget region, valid unless queued
    size_t items = 0;
    int32_t state = ZM_REQ_QUEUED;
    int32_t steps = 0, done = 0;
    const double* src_z = nullptr;
    const double* src_w = nullptr;
};

// First-fit allocator over [0, budget) with coalescing of freed ranges.
class Arena {
public:
    explicit Arena(size_t budget) : budget_(budget) { free_[0] = budget; }
    bool alloc(size_t bytes, size_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t budget() const { return budget_; }

private:
    size_t budget_;
    size_t used_ = 0;
    std::map<size_t, size_t> free_;
};

thread_local std::string g_pool_create_error;

size_t request_bytes(const zm_params& p, zm::PairShape* sh_out, zm::Layout* L_out)
{
    const zm::PairShape sh = zm::choose_pair_shape(p.n1, p.n2, p.precision);
    const zm::Layout L = zm::make_layout(p, sh);
    if (sh_out) *sh_out = sh;
    if (L_out) *L_out = L;
    return zm::align_up(L.total);
}

}  // namespace

struct zm_pool {
    Arena arena;
    TablesLayout tl;
    char* ws = nullptr;
    size_t budget = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    uint32_t flags = 0;
    int persistent_groups = 1024;
    int64_t next_id = 1;
    std::map<int64_t, Request> reqs;
    std::deque<int64_t> queue;
    std::vector<int64_t> live;     // admission order = table order
    size_t live_items = 0;
    bool dirty = true;             // tables must be rebuilt
    zm::BatchLaunch launch{};
    zm::TableBuild tables;         // host copy, kept alive while its upload may be pending
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int32_t iterations = 0;
    int64_t pairs_done = 0;
    std::string err;

    explicit zm_pool(size_t b) : arena(b), budget(b) {}
};

namespace {

zm_status pfail(zm_pool* p, zm_status st, const std::string& msg)
{
    if (p) p->err = msg;
    return st;
}

zm_status phip(zm_pool* p, hipError_t e, const char* where)
{
    return pfail(p, ZM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

void drop_live(zm_pool* P, int64_t id)
{
    auto it = std::find(P->live.begin(), P->live.end(), id);
    if (it != P->live.end()) {
        P->live.erase(it);
        P->live_items -= P->reqs[id].items;
        P->dirty = true;
    }
}

// Admit queued requests first-in first-out while budget, live slots and
// work-list capacity allow.
zm_status admit(zm_pool* P)
{
    while (!P->queue.empty()) {
        Request& r = P->reqs[P->queue.front()];
        if ((int)P->live.size() >= kMaxLive || P->live_items + r.items > kMaxItems) break;
        size_t off;
        if (!P->arena.alloc(r.bytes, &off)) break;
        r.offset = off;
        double* y0 = reinterpret_cast<double*>(P->ws + off + r.layout.y0);
        const size_t N = (size_t)r.prm.n1 * r.prm.n2;
        hipError_t e = hipMemcpyAsync(y0, r.src_z, 3 * N * sizeof(double), hipMemcpyDeviceToDevice,
                                      P->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(y0 + 3 * N, r.src_w, 2 * N * sizeof(double),
                               hipMemcpyDeviceToDevice, P->stream);
        // its fold statistics start cleared (the arena slot held another request)
        if (e == hipSuccess)
            e = hipMemsetAsync(P->ws + off + r.layout.fold, 0, zm::kFoldWords * sizeof(int),
                               P->stream);
        if (e != hipSuccess) {
            P->arena.release(off, r.bytes);
            return phip(P, e, "admission copy");
        }
        r.state = ZM_REQ_LIVE;
        r.src_z = r.src_w = nullptr;
        P->live.push_back(P->queue.front());
        P->live_items += r.items;
        P->queue.pop_front();
        P->dirty = true;
    }
    return ZM_OK;
}

zm_status rebuild(zm_pool* P)
{
    const int n = (int)P->live.size();
    std::vector<zm_params> prm(n);
    std::vector<zm::PairShape> shapes(n);
    std::vector<zm::Layout> layouts(n);
    std::vector<char*> bases(n);
    std::vector<int*> flags(n);
    int* dflags = reinterpret_cast<int*>(P->ws + P->budget + P->tl.flags);
    for (int i = 0; i < n; ++i) {
        const Request& r = P->reqs[P->live[i]];
        prm[i] = r.prm;
        shapes[i] = r.shape;
        layouts[i] = r.layout;
        bases[i] = P->ws + r.offset;
        flags[i] = (P->flags & ZM_FLAG_CHECK_FINITE) ? dflags + i : nullptr;
    }
    zm::TableBuild& tb = P->tables;
    zm::build_tables(prm.data(), shapes.data(), layouts.data(), bases.data(), flags.data(), n, tb);
    char* tbase = P->ws + P->budget;
    hipError_t e = hipSuccess;
    if (n > 0)
        e = hipMemcpyAsync(tbase + P->tl.desc, tb.table.data(), sizeof(zm::InstDesc) * n,
                           hipMemcpyHostToDevice, P->stream);
    if (e == hipSuccess && !tb.items.empty())
        e = hipMemcpyAsync(tbase + P->tl.items, tb.items.data(),
                           sizeof(zm::WorkItem) * tb.items.size(), hipMemcpyHostToDevice, P->stream);
    if (e != hipSuccess) return phip(P, e, "table upload");
    zm::BatchLaunch& L = P->launch;
    L.table = reinterpret_cast<const zm::InstDesc*>(tbase + P->tl.desc);
    L.count = n;
    L.total_blocks = tb.total_blocks;
    L.total_tie_blocks = tb.total_tie_blocks;
    L.total_reduce_blocks = tb.total_reduce_blocks;
    L.items = reinterpret_cast<const zm::WorkItem*>(tbase + P->tl.items);
    L.ngroups = (int)tb.groups.size();
    for (int g = 0; g < L.ngroups; ++g) L.groups[g] = tb.groups[g];
    L.counters = reinterpret_cast<int*>(tbase + P->tl.counters);
    L.persistent_groups = P->persistent_groups;
    L.any_even = tb.any_even;
    P->dirty = false;
    return ZM_OK;
}

}  // namespace

extern "C" {

size_t zm_pool_workspace_bytes(size_t budget_bytes)
{
    return zm::align_up(budget_bytes) + tables_layout().total;
}

size_t zm_pool_request_bytes(const zm_params* params)
{
    if (zm::validate(params) || params->flags != 0 || params->cutoff != 0.0 ||
        params->model != ZM_MODEL_HIGH || params->boundary != ZM_BOUNDARY_PERIODIC)
        return 0;
    if (zm::fp32_shape_problem(*params,
                               zm::choose_pair_shape(params->n1, params->n2, params->precision)))
        return 0;
    return request_bytes(*params, nullptr, nullptr);
}

zm_status zm_pool_create(zm_pool** out, size_t budget_bytes, uint32_t flags, void* d_workspace,
                         size_t workspace_bytes, void* hip_stream)
{
    g_pool_create_error.clear();
    if (!out) { g_pool_create_error = "out is NULL"; return ZM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (flags & ~ZM_FLAG_CHECK_FINITE) { g_pool_create_error = "unknown flag bits"; return ZM_ERR_INVALID_ARG; }
    if (budget_bytes == 0) { g_pool_create_error = "budget must be > 0"; return ZM_ERR_INVALID_ARG; }
    const size_t budget = zm::align_up(budget_bytes);
    if (!zm::aligned(d_workspace) || workspace_bytes < zm_pool_workspace_bytes(budget_bytes)) {
        g_pool_create_error = "workspace NULL, misaligned or smaller than zm_pool_workspace_bytes()";
        return ZM_ERR_WORKSPACE;
    }
    zm_pool* P = new (std::nothrow) zm_pool(budget);
    if (!P) { g_pool_create_error = "host allocation failed"; return ZM_ERR_CAPACITY; }
    P->tl = tables_layout();
    P->ws = reinterpret_cast<char*>(d_workspace);
    P->stream = reinterpret_cast<hipStream_t>(hip_stream);
    P->flags = flags;
    int cus = 0;
    hipError_t e = hipGetDevice(&P->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P->device);
    if (e == hipSuccess) e = hipEventCreate(&P->ev0);
    if (e == hipSuccess) e = hipEventCreate(&P->ev1);
    if (e != hipSuccess) {
        g_pool_create_error = std::string("device setup: ") + hipGetErrorString(e);
        if (P->ev0) (void)hipEventDestroy(P->ev0);
        delete P;
        return ZM_ERR_HIP;
    }
    P->persistent_groups = 4 * (cus > 0 ? cus : 256);
    *out = P;
    return ZM_OK;
}

zm_status zm_pool_submit(zm_pool* P, const zm_params* params, const double* d_z, const double* d_w,
                         int32_t steps, int64_t* id)
{
    if (!P) return ZM_ERR_INVALID_ARG;
    if (!id) return pfail(P, ZM_ERR_INVALID_ARG, "id is NULL");
    if (const char* why = zm::validate(params)) return pfail(P, ZM_ERR_INVALID_ARG, why);
    if (params->flags != 0) return pfail(P, ZM_ERR_INVALID_ARG, "request flags must be 0");
    if (params->cutoff != 0.0)
        return pfail(P, ZM_ERR_UNSUPPORTED, "the cutoff solver is not available in a pool");
    if (params->model != ZM_MODEL_HIGH)
        return pfail(P, ZM_ERR_UNSUPPORTED, "the low-order model is not available in a pool");
    if (params->boundary != ZM_BOUNDARY_PERIODIC)
        return pfail(P, ZM_ERR_UNSUPPORTED, "free sheets are not available in a pool");
    if (const char* why = zm::fp32_shape_problem(
            *params, zm::choose_pair_shape(params->n1, params->n2, params->precision)))
        return pfail(P, ZM_ERR_UNSUPPORTED, why);
    if (steps < 1) return pfail(P, ZM_ERR_INVALID_ARG, "steps must be >= 1");
    if (!zm::aligned(d_z) || !zm::aligned(d_w))
        return pfail(P, ZM_ERR_INVALID_ARG, "state pointers must be non-NULL and 256-byte aligned");
    Request r;
    r.prm = *params;
    r.bytes = request_bytes(*params, &r.shape, &r.layout);
    r.items = 0;
    for (int sp = 0; sp < r.shape.splits; ++sp)
        if (params->n2 - sp * r.shape.rows_per_split > 0) r.items += (size_t)(r.shape.px * r.shape.py);
    if (r.bytes > P->budget || r.items > kMaxItems)
        return pfail(P, ZM_ERR_CAPACITY, "request larger than the pool budget");
    r.steps = steps;
    r.src_z = d_z;
    r.src_w = d_w;
    *id = P->next_id++;
    P->reqs[*id] = r;
    P->queue.push_back(*id);
    return ZM_OK;
}

zm_status zm_pool_iterate(zm_pool* P, zm_step_record* records, int32_t capacity, int32_t* count)
{
    if (!P) return ZM_ERR_INVALID_ARG;
    if (!count || capacity < 0 || (capacity > 0 && !records))
        return pfail(P, ZM_ERR_INVALID_ARG, "bad record buffer");
    *count = 0;
    zm::DeviceGuard g(P->device);
    if (!g.ok) return pfail(P, ZM_ERR_HIP, "cannot select the pool device");
    zm_status st = admit(P);
    if (st != ZM_OK) return st;
    if (P->live.empty()) return ZM_OK;
    if (P->dirty) {
        st = rebuild(P);
        if (st != ZM_OK) return st;
    }
    const int n = (int)P->live.size();
    int* dflags = reinterpret_cast<int*>(P->ws + P->budget + P->tl.flags);
    const bool check = (P->flags & ZM_FLAG_CHECK_FINITE) != 0;
    hipError_t e = hipSuccess;
    if (check) e = hipMemsetAsync(dflags, 0, sizeof(int) * n, P->stream);
    if (e == hipSuccess) e = hipEventRecord(P->ev0, P->stream);
    for (int stage = 0; stage < 3 && e == hipSuccess; ++stage)
        e = zm::launch_batch_stage(P->launch, stage, P->stream);
    if (e == hipSuccess) e = hipEventRecord(P->ev1, P->stream);
    if (e == hipSuccess) e = hipEventSynchronize(P->ev1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, P->ev0, P->ev1);
    if (e != hipSuccess) return phip(P, e, "iteration");
    std::vector<int> hflags;
    if (check) {
        hflags.resize(n);
        e = hipMemcpy(hflags.data(), dflags, sizeof(int) * n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return phip(P, e, "flag read");
    }
    ++P->iterations;
    const std::vector<int64_t> advanced = P->live;
    int w = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t id = advanced[i];
        Request& r = P->reqs[id];
        r.done += 1;
        const int64_t N = (int64_t)r.prm.n1 * r.prm.n2;
        const int64_t side = 2 * (int64_t)r.prm.image_layers + 1;
        P->pairs_done += 3 * N * N * side * side;
        if (check && hflags[i]) {
            r.state = ZM_REQ_FAILED;
            drop_live(P, id);
            P->arena.release(r.offset, r.bytes);
        } else if (r.done >= r.steps) {
            r.state = ZM_REQ_FINISHED;
            drop_live(P, id);
        }
        if (w < capacity) records[w++] = zm_step_record{id, r.done, r.state, (double)ms};
    }
    *count = w;
    return ZM_OK;
}

zm_status zm_pool_query(const zm_pool* P, int64_t id, int32_t* state, int32_t* steps_done)
{
    if (!P || !state) return ZM_ERR_INVALID_ARG;
    auto it = P->reqs.find(id);
    if (it == P->reqs.end()) {
        *state = ZM_REQ_UNKNOWN;
        if (steps_done) *steps_done = 0;
        return ZM_OK;
    }
    *state = it->second.state;
    if (steps_done) *steps_done = it->second.done;
    return ZM_OK;
}

zm_status zm_pool_fetch(zm_pool* P, int64_t id, double* d_z, double* d_w)
{
    if (!P) return ZM_ERR_INVALID_ARG;
    auto it = P->reqs.find(id);
    if (it == P->reqs.end()) return pfail(P, ZM_ERR_INVALID_ARG, "unknown request");
    const Request& r = it->second;
    if (r.state != ZM_REQ_LIVE && r.state != ZM_REQ_FINISHED)
        return pfail(P, ZM_ERR_INVALID_ARG, "request has no resident state");
    if (!zm::aligned(d_z) || !zm::aligned(d_w))
        return pfail(P, ZM_ERR_INVALID_ARG, "state pointers must be non-NULL and 256-byte aligned");
    zm::DeviceGuard g(P->device);
    if (!g.ok) return pfail(P, ZM_ERR_HIP, "cannot select the pool device");
    const size_t N = (size_t)r.prm.n1 * r.prm.n2;
    const double* y0 = reinterpret_cast<const double*>(P->ws + r.offset + r.layout.y0);
    hipError_t e = hipMemcpyAsync(d_z, y0, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, P->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_w, y0 + 3 * N, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, P->stream);
    if (e != hipSuccess) return phip(P, e, "state copy");
    return ZM_OK;
}

zm_status zm_pool_release(zm_pool* P, int64_t id)
{
    if (!P) return ZM_ERR_INVALID_ARG;
    auto it = P->reqs.find(id);
    if (it == P->reqs.end()) return pfail(P, ZM_ERR_INVALID_ARG, "unknown request");
    Request& r = it->second;
    if (r.state != ZM_REQ_FINISHED && r.state != ZM_REQ_FAILED)
        return pfail(P, ZM_ERR_INVALID_ARG, "only finished or failed requests can be released");
    if (r.state == ZM_REQ_FINISHED) {
        // copies of its state out (zm_pool_fetch) are ordered before reuse
        // of the region by the stream
        P->arena.release(r.offset, r.bytes);
    }
    P->reqs.erase(it);
    return ZM_OK;
}

zm_status zm_pool_cancel(zm_pool* P, int64_t id)
{
    if (!P) return ZM_ERR_INVALID_ARG;
    auto it = P->reqs.find(id);
    if (it == P->reqs.end()) return pfail(P, ZM_ERR_INVALID_ARG, "unknown request");
    Request& r = it->second;
    if (r.state == ZM_REQ_QUEUED) {
        P->queue.erase(std::find(P->queue.begin(), P->queue.end(), id));
    } else if (r.state == ZM_REQ_LIVE) {
        drop_live(P, id);
        P->arena.release(r.offset, r.bytes);
    } else {
        return pfail(P, ZM_ERR_INVALID_ARG, "request already finished; release it instead");
    }
    P->reqs.erase(it);
    return ZM_OK;
}

zm_status zm_pool_get_stats(const zm_pool* P, zm_pool_stats* out)
{
    if (!P || !out) return ZM_ERR_INVALID_ARG;
    int fin = 0;
    for (const auto& kv : P->reqs) fin += (kv.second.state == ZM_REQ_FINISHED);
    out->queued = (int32_t)P->queue.size();
    out->live = (int32_t)P->live.size();
    out->finished = fin;
    out->iterations = P->iterations;
    out->used_bytes = (int64_t)P->arena.used();
    out->budget_bytes = (int64_t)P->budget;
    out->pairs_done = P->pairs_done;
    return ZM_OK;
}

zm_status zm_pool_destroy(zm_pool* P)
{
    if (!P) return ZM_OK;
    zm_status st = ZM_OK;
    {
        zm::DeviceGuard g(P->device);
        if (g.ok && hipStreamSynchronize(P->stream) != hipSuccess) st = ZM_ERR_HIP;
        if (P->ev0) (void)hipEventDestroy(P->ev0);
        if (P->ev1) (void)hipEventDestroy(P->ev1);
    }
    delete P;
    return st;
}

const char* zm_pool_last_error(const zm_pool* P)
{
    if (!P) return g_pool_create_error.c_str();
    return P->err.c_str();
}

}  // extern "C"
