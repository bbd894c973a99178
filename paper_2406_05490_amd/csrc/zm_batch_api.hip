// Host side of the batched ensemble (zm_batch_* in include/zm.h).
//
// The workspace holds, per instance, the same regions as a single-instance
// context, followed by the device descriptor table, the pair work list and
// the work counters.  Work items are ordered longest first (targets in the
// patch x sources in the split) so the persistent pair launch finishes with
// its smallest items.
#include "zm.h"
#include "zm_batch_internal.h"
#include "zm_host.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_batch_create_error;

struct BatchPlan {
    std::vector<zm::PairShape> shapes;
    std::vector<zm::Layout> layouts;
    std::vector<size_t> inst_off;
    size_t n_items = 0;
    size_t table_off = 0, items_off = 0, counters_off = 0, flag_off = 0, total = 0;
};

// Number of pair work items of one member.
size_t count_items(const zm_params& p, const zm::PairShape& sh)
{
    size_t n = 0;
    for (int sp = 0; sp < sh.splits; ++sp)
        if (p.n2 - sp * sh.rows_per_split > 0) ++n;
    return n * (size_t)(sh.px * sh.py);
}

const char* plan_batch(const zm_params* params, int32_t count, BatchPlan& P)
{
    if (!params) return "params is NULL";
    if (count < 1) return "count must be >= 1";
    if (count > (1 << 20)) return "count too large";
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        if (const char* why = zm::validate(&params[i])) return why;
        if (params[i].flags != 0) return "per-instance flags must be 0 in a batch";
        if (params[i].cutoff != 0.0) return "the cutoff solver is not available in a batch";
        if (params[i].model != ZM_MODEL_HIGH) return "the low-order model is not available in a batch";
        if (params[i].boundary != ZM_BOUNDARY_PERIODIC) return "free sheets are not available in a batch";
        const zm::PairShape sh =
            zm::choose_pair_shape(params[i].n1, params[i].n2, params[i].precision);
        if (const char* why = zm::fp32_shape_problem(params[i], sh)) return why;
        const zm::Layout L = zm::make_layout(params[i], sh);
        P.shapes.push_back(sh);
        P.layouts.push_back(L);
        P.inst_off.push_back(off);
        off = zm::align_up(off + L.total);
        P.n_items += count_items(params[i], sh);
    }
    P.table_off = off;
    off = zm::align_up(off + sizeof(zm::InstDesc) * count);
    P.items_off = off;
    off = zm::align_up(off + sizeof(zm::WorkItem) * std::max<size_t>(1, P.n_items));
    P.counters_off = off;
    off = zm::align_up(off + zm::kMaxPairGroups * sizeof(int));
    P.flag_off = off;
    off = zm::align_up(off + sizeof(int));
    P.total = off;
    return nullptr;
}

}  // namespace

struct zm_batch {
    std::vector<zm_params> prm;
    BatchPlan plan;
    std::vector<zm::PairGroup> groups;
    zm::BatchLaunch launch;
    hipStream_t stream = nullptr;
    int device = 0;
    char* ws = nullptr;
    uint32_t flags = 0;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    std::string err;
};

namespace {

zm_status bfail(zm_batch* b, zm_status st, const std::string& msg)
{
    if (b) b->err = msg;
    return st;
}

zm_status bhip(zm_batch* b, hipError_t e, const char* where)
{
    return bfail(b, ZM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

hipError_t enqueue_step(zm_batch* b, hipStream_t s)
{
    for (int stage = 0; stage < 3; ++stage) {
        hipError_t e = zm::launch_batch_stage(b->launch, stage, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

zm_status ensure_graph(zm_batch* b)
{
    if (b->graph) return ZM_OK;
    hipError_t e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bhip(b, e, "capture stream");
    e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bhip(b, e, "begin capture");
    hipError_t le = enqueue_step(b, b->capture_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->capture_stream, &g);
    if (le != hipSuccess) { if (g) (void)hipGraphDestroy(g); return bhip(b, le, "captured launch"); }
    if (e != hipSuccess) return bhip(b, e, "end capture");
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { b->graph = nullptr; return bhip(b, e, "graph instantiate"); }
    return ZM_OK;
}

}  // namespace

namespace zm {

void build_tables(const zm_params* params, const PairShape* shapes, const Layout* layouts,
                  char* const* bases, int* const* flags, int count, TableBuild& out)
{
    out = TableBuild();
    out.table.resize(count);
    std::vector<std::pair<double, WorkItem>> keyed[kMaxPairGroups];
    int block = 0, tie_block = 0, reduce_block = 0;
    for (int i = 0; i < count; ++i) {
        InstDesc& d = out.table[i];
        std::memset(&d, 0, sizeof(d));
        d.m = make_mesh(params[i]);
        d.sh = shapes[i];
        d.precision = params[i].precision;
        d.block_begin = block;
        d.blocks = (d.m.N + 255) / 256;
        block += d.blocks;
        d.tie_block_begin = tie_block;
        tie_block += dev_tie_blocks(d.m.n1, d.m.n2);
        d.reduce_block_begin = reduce_block;
        reduce_block += (d.m.N * dev_reduce_lanes(d.m.N, shapes[i].splits) + 255) / 256;
        char* base = bases[i];
        const Layout& L = layouts[i];
        d.Y[0] = reinterpret_cast<double*>(base + L.y0);
        d.Y[1] = reinterpret_cast<double*>(base + L.y1);
        d.Y[2] = reinterpret_cast<double*>(base + L.y2);
        d.gam = reinterpret_cast<double*>(base + L.gam);
        d.q = reinterpret_cast<double*>(base + L.q);
        d.part = reinterpret_cast<double*>(base + L.part);
        d.tie = reinterpret_cast<double*>(base + L.tie);
        d.u = reinterpret_cast<double*>(base + L.u);
        d.V = reinterpret_cast<double*>(base + L.V);
        d.fold = reinterpret_cast<int*>(base + L.fold);
        d.flag = flags ? flags[i] : nullptr;
        if (params[i].n1 % 2 == 0 || params[i].n2 % 2 == 0) out.any_even = true;
        const PairShape& sh = shapes[i];
        const int g = (params[i].precision == ZM_FP32_PAIRS ? 9 : 0) +
                      3 * (sh.R == 1 ? 0 : (sh.R == 2 ? 1 : 2)) +
                      (sh.cx == 32 ? 0 : (sh.cx == 16 ? 1 : 2));
        const int side = 2 * params[i].image_layers + 1;
        for (int pt = 0; pt < sh.px * sh.py; ++pt) {
            for (int sp = 0; sp < sh.splits; ++sp) {
                const int rows = std::min(sh.rows_per_split, params[i].n2 - sp * sh.rows_per_split);
                if (rows <= 0) continue;
                const double cost = (double)rows * params[i].n1 * side * side;
                keyed[g].push_back({cost, WorkItem{i, pt, sp, 0}});
            }
        }
    }
    out.total_blocks = block;
    out.total_tie_blocks = tie_block;
    out.total_reduce_blocks = reduce_block;
    static const int kR[3] = {1, 2, 4};
    static const int kPX[3] = {32, 16, 8};
    for (int g = 0; g < kMaxPairGroups; ++g) {
        if (keyed[g].empty()) continue;
        std::stable_sort(keyed[g].begin(), keyed[g].end(),
                         [](const auto& a, const auto& b) { return a.first > b.first; });
        out.groups.push_back(PairGroup{g / 9, kR[(g / 3) % 3], kPX[g % 3], (int)out.items.size(),
                                       (int)keyed[g].size()});
        for (auto& k : keyed[g]) out.items.push_back(k.second);
    }
}

}  // namespace zm

extern "C" {

size_t zm_batch_workspace_bytes(const zm_params* params, int32_t count)
{
    BatchPlan P;
    if (plan_batch(params, count, P)) return 0;
    return P.total;
}

zm_status zm_batch_create(zm_batch** out, const zm_params* params, int32_t count,
                          uint32_t batch_flags, void* d_workspace, size_t workspace_bytes,
                          void* hip_stream)
{
    g_batch_create_error.clear();
    if (!out) { g_batch_create_error = "out is NULL"; return ZM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (batch_flags & ~(ZM_FLAG_GRAPH | ZM_FLAG_CHECK_FINITE)) {
        g_batch_create_error = "unknown batch flag bits";
        return ZM_ERR_INVALID_ARG;
    }
    zm_batch* b = new (std::nothrow) zm_batch();
    if (!b) { g_batch_create_error = "host allocation failed"; return ZM_ERR_CAPACITY; }
    if (const char* why = plan_batch(params, count, b->plan)) {
        g_batch_create_error = why;
        delete b;
        bool cut = false;
        for (int i = 0; params && i < count; ++i)
            cut = cut || params[i].cutoff != 0.0 || params[i].model != ZM_MODEL_HIGH ||
                  params[i].boundary != ZM_BOUNDARY_PERIODIC ||
                  (!zm::validate(&params[i]) &&
                   zm::fp32_shape_problem(params[i], zm::choose_pair_shape(params[i].n1, params[i].n2,
                                                                           params[i].precision)));
        return cut ? ZM_ERR_UNSUPPORTED : ZM_ERR_INVALID_ARG;
    }
    if (!zm::aligned(d_workspace) || workspace_bytes < b->plan.total) {
        g_batch_create_error = "workspace NULL, misaligned or smaller than zm_batch_workspace_bytes()";
        delete b;
        return ZM_ERR_WORKSPACE;
    }
    hipError_t e = hipGetDevice(&b->device);
    int cus = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e != hipSuccess) {
        g_batch_create_error = std::string("device query: ") + hipGetErrorString(e);
        delete b;
        return ZM_ERR_HIP;
    }
    b->prm.assign(params, params + count);
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->ws = reinterpret_cast<char*>(d_workspace);
    b->flags = batch_flags;
    const BatchPlan& P = b->plan;

    std::vector<char*> bases(count);
    std::vector<int*> flags(count);
    for (int i = 0; i < count; ++i) {
        bases[i] = b->ws + P.inst_off[i];
        flags[i] = (batch_flags & ZM_FLAG_CHECK_FINITE) ? reinterpret_cast<int*>(b->ws + P.flag_off)
                                                        : nullptr;
    }
    zm::TableBuild tb;
    zm::build_tables(params, P.shapes.data(), P.layouts.data(), bases.data(), flags.data(), count,
                     tb);
    b->groups = tb.groups;
    zm::InstDesc* dtable = reinterpret_cast<zm::InstDesc*>(b->ws + P.table_off);
    zm::WorkItem* ditems = reinterpret_cast<zm::WorkItem*>(b->ws + P.items_off);
    e = hipMemcpyAsync(dtable, tb.table.data(), sizeof(zm::InstDesc) * count, hipMemcpyHostToDevice,
                       b->stream);
    if (e == hipSuccess && !tb.items.empty())
        e = hipMemcpyAsync(ditems, tb.items.data(), sizeof(zm::WorkItem) * tb.items.size(),
                           hipMemcpyHostToDevice, b->stream);
    // every instance's fold statistics start cleared
    for (int i = 0; e == hipSuccess && i < count; ++i)
        e = hipMemsetAsync(bases[i] + P.layouts[i].fold, 0, zm::kFoldWords * sizeof(int),
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        g_batch_create_error = std::string("table upload: ") + hipGetErrorString(e);
        delete b;
        return ZM_ERR_HIP;
    }
    zm::BatchLaunch& L = b->launch;
    L.table = dtable;
    L.count = count;
    L.total_blocks = tb.total_blocks;
    L.total_tie_blocks = tb.total_tie_blocks;
    L.total_reduce_blocks = tb.total_reduce_blocks;
    L.items = ditems;
    L.ngroups = (int)tb.groups.size();
    for (int g = 0; g < L.ngroups; ++g) L.groups[g] = tb.groups[g];
    L.counters = reinterpret_cast<int*>(b->ws + P.counters_off);
    L.persistent_groups = 4 * (cus > 0 ? cus : 256);
    L.any_even = tb.any_even;
    *out = b;
    return ZM_OK;
}

zm_status zm_batch_init_state(zm_batch* b, int32_t index, const double* d_z, const double* d_w)
{
    if (!b) return ZM_ERR_INVALID_ARG;
    if (index < 0 || index >= (int32_t)b->prm.size())
        return bfail(b, ZM_ERR_INVALID_ARG, "index out of range");
    if (!zm::aligned(d_z) || !zm::aligned(d_w))
        return bfail(b, ZM_ERR_INVALID_ARG, "state pointers must be non-NULL and 256-byte aligned");
    zm::DeviceGuard g(b->device);
    if (!g.ok) return bfail(b, ZM_ERR_HIP, "cannot select the batch device");
    const size_t N = (size_t)b->prm[index].n1 * b->prm[index].n2;
    double* y0 = reinterpret_cast<double*>(b->ws + b->plan.inst_off[index] + b->plan.layouts[index].y0);
    hipError_t e = hipMemcpyAsync(y0, d_z, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(y0 + 3 * N, d_w, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return bhip(b, e, "state copy");
    return ZM_OK;
}

zm_status zm_batch_get_state(zm_batch* b, int32_t index, double* d_z, double* d_w)
{
    if (!b) return ZM_ERR_INVALID_ARG;
    if (index < 0 || index >= (int32_t)b->prm.size())
        return bfail(b, ZM_ERR_INVALID_ARG, "index out of range");
    if (!zm::aligned(d_z) || !zm::aligned(d_w))
        return bfail(b, ZM_ERR_INVALID_ARG, "state pointers must be non-NULL and 256-byte aligned");
    zm::DeviceGuard g(b->device);
    if (!g.ok) return bfail(b, ZM_ERR_HIP, "cannot select the batch device");
    const size_t N = (size_t)b->prm[index].n1 * b->prm[index].n2;
    const double* y0 =
        reinterpret_cast<const double*>(b->ws + b->plan.inst_off[index] + b->plan.layouts[index].y0);
    hipError_t e = hipMemcpyAsync(d_z, y0, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_w, y0 + 3 * N, 2 * N * sizeof(double), hipMemcpyDeviceToDevice, b->stream);
    if (e != hipSuccess) return bhip(b, e, "state copy");
    return ZM_OK;
}

zm_status zm_batch_step(zm_batch* b, int32_t nsteps)
{
    if (!b) return ZM_ERR_INVALID_ARG;
    if (nsteps < 0) return bfail(b, ZM_ERR_INVALID_ARG, "nsteps must be >= 0");
    zm::DeviceGuard g(b->device);
    if (!g.ok) return bfail(b, ZM_ERR_HIP, "cannot select the batch device");
    int* flag = reinterpret_cast<int*>(b->ws + b->plan.flag_off);
    const bool check = (b->flags & ZM_FLAG_CHECK_FINITE) != 0;
    hipError_t e;
    if (check) {
        e = hipMemsetAsync(flag, 0, sizeof(int), b->stream);
        if (e != hipSuccess) return bhip(b, e, "flag clear");
    }
    if (b->flags & ZM_FLAG_GRAPH) {
        if (nsteps > 0) {
            zm_status st = ensure_graph(b);
            if (st != ZM_OK) return st;
        }
        for (int i = 0; i < nsteps; ++i) {
            e = hipGraphLaunch(b->graph, b->stream);
            if (e != hipSuccess) return bhip(b, e, "graph launch");
        }
    } else {
        for (int i = 0; i < nsteps; ++i) {
            e = enqueue_step(b, b->stream);
            if (e != hipSuccess) return bhip(b, e, "batch launch");
        }
    }
    if (check) {
        int host_flag = 0;
        e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return bhip(b, e, "flag read");
        if (host_flag) return bfail(b, ZM_ERR_NONFINITE, "some instance became non-finite");
    }
    return ZM_OK;
}

zm_status zm_batch_get_info(const zm_batch* b, zm_batch_info* out)
{
    if (!b || !out) return ZM_ERR_INVALID_ARG;
    out->count = (int32_t)b->prm.size();
    out->work_items[0] = out->work_items[1] = 0;
    for (const auto& G : b->groups) out->work_items[G.precision] += G.nitems;
    out->persistent_groups = b->launch.persistent_groups;
    int64_t pairs = 0;
    for (const auto& p : b->prm) {
        const int64_t N = (int64_t)p.n1 * p.n2;
        const int64_t side = 2 * (int64_t)p.image_layers + 1;
        pairs += 3 * N * N * side * side;
    }
    out->pairs_per_step = pairs;
    return ZM_OK;
}

zm_status zm_batch_destroy(zm_batch* b)
{
    if (!b) return ZM_OK;
    zm_status st = ZM_OK;
    {
        zm::DeviceGuard g(b->device);
        if (g.ok && hipStreamSynchronize(b->stream) != hipSuccess) st = ZM_ERR_HIP;
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    }
    delete b;
    return st;
}

const char* zm_batch_last_error(const zm_batch* b)
{
    if (!b) return g_batch_create_error.c_str();
    return b->err.c_str();
}

}  // extern "C"
