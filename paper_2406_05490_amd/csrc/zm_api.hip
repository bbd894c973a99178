// Host runtime behind the C ABI declared in include/zm.h.
//
// A context owns no device memory: it carves the caller's workspace into
// the RK3 state buffers and the per-evaluation scratch, and enqueues the
// kernel sequence on the caller's stream.  Per derivative evaluation:
//   k_surface -> k_pairs -> [k_ties] -> k_reduce -> k_update
// or, for a cutoff context,
//   k_surface -> cell binning and sort -> k_cut_pairs -> k_reduce -> k_update
// or, for the low-order model,
//   k_surface -> FFT velocity (pack, FFTs, transposes, symbol) -> k_update
#include "zm.h"
#include "zm_host.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using zm::Layout;
using zm::aligned;
using zm::DeviceGuard;
using zm::make_layout;
using zm::overlaps;
using zm::validate;

namespace {

thread_local std::string g_create_error;

struct Timed {
    int kernel;
    hipEvent_t start, stop;
};

}  // namespace

void zm::set_create_error(const std::string& msg) { g_create_error = msg; }

struct zm_ctx {
    zm_params prm;
    zm::Mesh mesh;
    zm::PairShape shape;
    Layout layout;
    hipStream_t stream = nullptr;
    int device = 0;
    char* ws = nullptr;
    std::string err;
    bool profiling = false;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> spare;
    zm_kernel_stats stats[ZM_KERNEL_COUNT];
    hipStream_t capture_stream = nullptr;   // graph capture (non-blocking, default priority)
    hipGraphExec_t graph = nullptr;         // one captured RK3 step
    bool cutoff = false;                    // cutoff BR solver
    zm::CutGrid cut{};
    zm::CutBuffers cb{};
    bool low = false;                       // low-order model (FFT velocity)
    bool medium = false;                    // medium order: BR moves the sheet, FFT velocity in V
    zm::LowBuffers lb{};

    double* at(size_t off) { return reinterpret_cast<double*>(ws + off); }
    size_t N() const { return (size_t)mesh.N; }
};

namespace {

zm_status fail(zm_ctx* c, zm_status st, const std::string& msg)
{
    if (c) c->err = msg;
    return st;
}

zm_status hip_fail(zm_ctx* c, hipError_t e, const char* where)
{
    return fail(c, ZM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

hipEvent_t get_event(zm_ctx* c)
{
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Enqueue one launch, bracketed by timing events when profiling is on.
template <class F>
hipError_t timed(zm_ctx* c, int kernel, F&& launch)
{
    if (!c->profiling) return launch();
    hipEvent_t a = get_event(c), b = get_event(c);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, c->stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, c->stream);
    if (e != hipSuccess) return e;
    c->pending.push_back({kernel, a, b});
    return hipSuccess;
}

// Medium order: the Bernoulli potential V from the FFT (flat-sheet)
// velocity, after the BR sum has produced the sheet velocity.  Nothing to
// do for the other models or without V.
zm_status medium_potential(zm_ctx* c, const double* z, const double* w, double* V,
                           hipStream_t stream)
{
    if (!c->medium || !V) return ZM_OK;
    hipError_t e = timed(c, ZM_KERNEL_FFT, [&] {
        return zm::launch_low_velocity(c->mesh, z, w, c->lb, nullptr, V, stream);
    });
    if (e != hipSuccess) return hip_fail(c, e, "FFT velocity launch");
    return ZM_OK;
}

// u (3 planes) = the velocity that moves the sheet (BR sum, or the FFT
// velocity for the low-order model); optionally V as well.
zm_status eval_velocity(zm_ctx* c, const double* z, const double* w, double* u, double* V,
                        hipStream_t stream)
{
    const zm::Mesh& m = c->mesh;
    double* gam = c->at(c->layout.gam);
    double* q = c->at(c->layout.q);
    double* part = c->at(c->layout.part);
    double* tie = c->at(c->layout.tie);
    int* fold = reinterpret_cast<int*>(c->ws + c->layout.fold);
    hipError_t e;
    if (c->low) {   // the FFT velocity needs no source strengths
        e = timed(c, ZM_KERNEL_FFT,
                  [&] { return zm::launch_low_velocity(m, z, w, c->lb, u, V, stream); });
        if (e != hipSuccess) return hip_fail(c, e, "FFT velocity launch");
        return ZM_OK;
    }
    e = timed(c, ZM_KERNEL_SURFACE,
              [&] { return zm::launch_surface(m, z, w, gam, q, fold, stream); });
    if (e != hipSuccess) return hip_fail(c, e, "surface kernel launch");
    if (c->cutoff) {
        int half = 0;
        e = timed(c, ZM_KERNEL_CELLS,
                  [&] { return zm::launch_cut_cells(m, c->cut, z, gam, c->cb, fold, &half, stream); });
        if (e != hipSuccess) return hip_fail(c, e, "cell binning launch");
        e = timed(c, ZM_KERNEL_PAIRS, [&] {
            return zm::launch_cut_pairs(m, c->cut, z, gam, c->cb, half, part, c->profiling, fold,
                                        stream);
        });
        if (e != hipSuccess) return hip_fail(c, e, "cutoff pair kernel launch");
        e = timed(c, ZM_KERNEL_REDUCE, [&] {
            return zm::launch_reduce(m, c->cut.planes, part, tie, q, z, u, c->medium ? nullptr : V,
                                     stream, false);
        });
        if (e != hipSuccess) return hip_fail(c, e, "reduce kernel launch");
        return medium_potential(c, z, w, V, stream);
    }
    e = timed(c, ZM_KERNEL_PAIRS, [&] {
        return c->prm.precision == ZM_FP32_PAIRS
                   ? zm::launch_pairs_f32(m, c->shape, z, gam, part, fold, stream)
                   : zm::launch_pairs_f64(m, c->shape, z, gam, part, fold, stream);
    });
    if (e != hipSuccess) return hip_fail(c, e, "pair kernel launch");
    const bool ties = m.periodic && ((m.n1 % 2) == 0 || (m.n2 % 2) == 0);
    if (ties) {
        e = timed(c, ZM_KERNEL_TIES, [&] { return zm::launch_ties(m, z, gam, tie, stream); });
        if (e != hipSuccess) return hip_fail(c, e, "tie kernel launch");
    }
    e = timed(c, ZM_KERNEL_REDUCE, [&] {
        return zm::launch_reduce(m, c->shape.splits, part, tie, q, z, u, c->medium ? nullptr : V,
                                 stream, m.periodic != 0);
    });
    if (e != hipSuccess) return hip_fail(c, e, "reduce kernel launch");
    return medium_potential(c, z, w, V, stream);
}

}  // namespace

extern "C" {

size_t zm_workspace_bytes(const zm_params* params)
{
    if (validate(params)) return 0;
    if (params->cutoff > 0.0 && params->precision != ZM_FP64) return 0;
    if (params->model == ZM_MODEL_LOW &&
        (params->precision != ZM_FP64 || !zm::low_order_supported_side(params->n1) ||
         !zm::low_order_supported_side(params->n2)))
        return 0;
    if (params->model == ZM_MODEL_MEDIUM && (!zm::low_order_supported_side(params->n1) ||
                                             !zm::low_order_supported_side(params->n2)))
        return 0;
    const zm::PairShape sh = zm::choose_pair_shape(params->n1, params->n2, params->precision);
    if (params->model != ZM_MODEL_LOW && zm::fp32_shape_problem(*params, sh)) return 0;
    return make_layout(*params, sh).total;
}

zm_status zm_create(zm_ctx** out, const zm_params* params, void* d_workspace,
                    size_t workspace_bytes, void* hip_stream)
{
    g_create_error.clear();
    if (!out) { g_create_error = "out is NULL"; return ZM_ERR_INVALID_ARG; }
    *out = nullptr;
    if (const char* why = validate(params)) { g_create_error = why; return ZM_ERR_INVALID_ARG; }
    if (params->cutoff > 0.0 && params->precision != ZM_FP64) {
        g_create_error = "the cutoff solver is FP64 only";
        return ZM_ERR_UNSUPPORTED;
    }
    if (params->model == ZM_MODEL_LOW &&
        (params->precision != ZM_FP64 || !zm::low_order_supported_side(params->n1) ||
         !zm::low_order_supported_side(params->n2))) {
        g_create_error = "the low-order model needs FP64 and sides that are powers of two <= 4096";
        return ZM_ERR_UNSUPPORTED;
    }
    if (params->model == ZM_MODEL_MEDIUM && (!zm::low_order_supported_side(params->n1) ||
                                             !zm::low_order_supported_side(params->n2))) {
        g_create_error = "the medium-order model needs sides that are powers of two <= 4096";
        return ZM_ERR_UNSUPPORTED;
    }
    const zm::PairShape sh = zm::choose_pair_shape(params->n1, params->n2, params->precision);
    if (params->model != ZM_MODEL_LOW) {
        if (const char* why = zm::fp32_shape_problem(*params, sh)) {
            g_create_error = why;
            return ZM_ERR_UNSUPPORTED;
        }
    }
    const Layout L = make_layout(*params, sh);
    if (!d_workspace || !aligned(d_workspace)) {
        g_create_error = "workspace is NULL or not 256-byte aligned";
        return ZM_ERR_WORKSPACE;
    }
    if (workspace_bytes < L.total) {
        g_create_error = "workspace smaller than zm_workspace_bytes()";
        return ZM_ERR_WORKSPACE;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return ZM_ERR_HIP;
    }
    zm_ctx* c = new (std::nothrow) zm_ctx();
    if (!c) { g_create_error = "host allocation failed"; return ZM_ERR_CAPACITY; }
    c->prm = *params;
    c->shape = sh;
    c->layout = L;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->device = dev;
    c->ws = reinterpret_cast<char*>(d_workspace);
    std::memset(c->stats, 0, sizeof(c->stats));
    c->mesh = zm::make_mesh(*params);
    if (params->model == ZM_MODEL_LOW || params->model == ZM_MODEL_MEDIUM) {
        c->low = params->model == ZM_MODEL_LOW;
        c->medium = params->model == ZM_MODEL_MEDIUM;
        char* ws = c->ws;
        c->lb.a = reinterpret_cast<double2*>(ws + L.lo_a);
        c->lb.b = reinterpret_cast<double2*>(ws + L.lo_b);
        c->lb.tw1 = reinterpret_cast<double2*>(ws + L.lo_tw1);
        c->lb.tw2 = reinterpret_cast<double2*>(ws + L.lo_tw2);
    }
    if (zm::has_cutoff(*params)) {
        c->cutoff = true;
        c->cut = zm::cut_grid_of(*params);
        char* ws = c->ws;
        for (int h = 0; h < 2; ++h) {
            c->cb.keys[h] = reinterpret_cast<unsigned*>(ws + L.cut_keys[h]);
            c->cb.vals[h] = reinterpret_cast<unsigned*>(ws + L.cut_vals[h]);
        }
        c->cb.hist = reinterpret_cast<unsigned*>(ws + L.cut_hist);
        c->cb.start = reinterpret_cast<int*>(ws + L.cut_start);
        c->cb.end = reinterpret_cast<int*>(ws + L.cut_end);
        c->cb.bstart = reinterpret_cast<int*>(ws + L.cut_bstart);
        c->cb.bend = reinterpret_cast<int*>(ws + L.cut_bend);
        c->cb.src = reinterpret_cast<double*>(ws + L.cut_src);
        c->cb.counts = reinterpret_cast<unsigned long long*>(ws + L.cut_counts);
        c->cb.kflag = reinterpret_cast<int*>(ws + L.cut_kflag);
    }
    // the surface kernel's fold statistics start cleared (each evaluation's
    // last surface workgroup clears them again for the next one)
    e = hipMemsetAsync(c->ws + L.fold, 0, zm::kFoldWords * sizeof(int), c->stream);
    if (e != hipSuccess) {
        g_create_error = std::string("workspace clear: ") + hipGetErrorString(e);
        delete c;
        return ZM_ERR_HIP;
    }
    *out = c;
    return ZM_OK;
}

zm_status zm_init_state(zm_ctx* c, const double* d_z, const double* d_w)
{
    if (!c) return ZM_ERR_INVALID_ARG;
    if (!aligned(d_z) || !aligned(d_w))
        return fail(c, ZM_ERR_INVALID_ARG, "state pointers must be non-NULL and 256-byte aligned");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, ZM_ERR_HIP, "cannot select the context device");
    const size_t N = c->N();
    double* y0 = c->at(c->layout.y0);
    hipError_t e = hipMemcpyAsync(y0, d_z, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(y0 + 3 * N, d_w, 2 * N * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "state copy");
    return ZM_OK;
}

zm_status zm_get_state(zm_ctx* c, double* d_z, double* d_w)
{
    if (!c) return ZM_ERR_INVALID_ARG;
    if (!aligned(d_z) || !aligned(d_w))
        return fail(c, ZM_ERR_INVALID_ARG, "state pointers must be non-NULL and 256-byte aligned");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, ZM_ERR_HIP, "cannot select the context device");
    const size_t N = c->N();
    const double* y0 = c->at(c->layout.y0);
    hipError_t e = hipMemcpyAsync(d_z, y0, 3 * N * sizeof(double), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_w, y0 + 3 * N, 2 * N * sizeof(double), hipMemcpyDeviceToDevice,
                           c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "state copy");
    return ZM_OK;
}

zm_status zm_br_velocity(zm_ctx* c, const double* d_z, const double* d_w, double* d_u)
{
    if (!c) return ZM_ERR_INVALID_ARG;
    if (!aligned(d_z) || !aligned(d_w) || !aligned(d_u))
        return fail(c, ZM_ERR_INVALID_ARG, "pointers must be non-NULL and 256-byte aligned");
    const size_t N = c->N(), d = sizeof(double);
    if (overlaps(d_u, 3 * N * d, d_z, 3 * N * d) || overlaps(d_u, 3 * N * d, d_w, 2 * N * d))
        return fail(c, ZM_ERR_INVALID_ARG, "d_u overlaps an input");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, ZM_ERR_HIP, "cannot select the context device");
    return eval_velocity(c, d_z, d_w, d_u, nullptr, c->stream);
}

zm_status zm_rhs(zm_ctx* c, const double* d_z, const double* d_w, double* d_zt, double* d_wt)
{
    if (!c) return ZM_ERR_INVALID_ARG;
    if (!aligned(d_z) || !aligned(d_w) || !aligned(d_zt) || !aligned(d_wt))
        return fail(c, ZM_ERR_INVALID_ARG, "pointers must be non-NULL and 256-byte aligned");
    const size_t N = c->N(), d = sizeof(double);
    const void* in[2] = {d_z, d_w};
    const size_t nin[2] = {3 * N * d, 2 * N * d};
    for (int i = 0; i < 2; ++i)
        if (overlaps(d_zt, 3 * N * d, in[i], nin[i]) || overlaps(d_wt, 2 * N * d, in[i], nin[i]))
            return fail(c, ZM_ERR_INVALID_ARG, "an output overlaps an input");
    if (overlaps(d_zt, 3 * N * d, d_wt, 2 * N * d))
        return fail(c, ZM_ERR_INVALID_ARG, "d_zt overlaps d_wt");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, ZM_ERR_HIP, "cannot select the context device");
    double* u = c->at(c->layout.u);
    double* V = c->at(c->layout.V);
    zm_status st = eval_velocity(c, d_z, d_w, u, V, c->stream);
    if (st != ZM_OK) return st;
    hipError_t e = timed(c, ZM_KERNEL_UPDATE, [&] {
        return zm::launch_update(c->mesh, 3, nullptr, nullptr, d_z, d_w, u, V, d_zt, d_wt, nullptr,
                                 c->stream);
    });
    if (e != hipSuccess) return hip_fail(c, e, "update kernel launch");
    return ZM_OK;
}

}  // extern "C"

namespace {

// Enqueue one RK3 step (three derivative evaluations and stage updates).
zm_status enqueue_step(zm_ctx* c, hipStream_t stream)
{
    const size_t N = c->N();
    double* Y[3] = {c->at(c->layout.y0), c->at(c->layout.y1), c->at(c->layout.y2)};
    double* u = c->at(c->layout.u);
    double* V = c->at(c->layout.V);
    int* flag = (c->prm.flags & ZM_FLAG_CHECK_FINITE)
                    ? reinterpret_cast<int*>(c->ws + c->layout.flag) : nullptr;
    for (int stage = 0; stage < 3; ++stage) {
        double* ys = Y[stage];                       // state F is evaluated at
        double* out = Y[(stage + 1) % 3];            // Y1, Y2, then Y0 in place
        zm_status st = eval_velocity(c, ys, ys + 3 * N, u, V, stream);
        if (st != ZM_OK) return st;
        hipError_t e = timed(c, ZM_KERNEL_UPDATE, [&] {
            return zm::launch_update(c->mesh, stage, Y[0], Y[0] + 3 * N, ys, ys + 3 * N, u, V, out,
                                     out + 3 * N, flag, stream);
        });
        if (e != hipSuccess) return hip_fail(c, e, "update kernel launch");
    }
    return ZM_OK;
}

// Capture one step into a graph on a private non-blocking stream (the
// caller's stream may be the null stream, which cannot be captured).  The
// graph holds kernel nodes only.
zm_status ensure_graph(zm_ctx* c)
{
    if (c->graph) return ZM_OK;
    hipError_t e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(c, e, "capture stream");
    e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(c, e, "begin capture");
    const bool prof = c->profiling;
    c->profiling = false;
    zm_status st = enqueue_step(c, c->capture_stream);
    c->profiling = prof;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->capture_stream, &g);
    if (st != ZM_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return hip_fail(c, e, "end capture");
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) { c->graph = nullptr; return hip_fail(c, e, "graph instantiate"); }
    return ZM_OK;
}

}  // namespace

extern "C" {

zm_status zm_step(zm_ctx* c, int32_t nsteps)
{
    if (!c) return ZM_ERR_INVALID_ARG;
    if (nsteps < 0) return fail(c, ZM_ERR_INVALID_ARG, "nsteps must be >= 0");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, ZM_ERR_HIP, "cannot select the context device");
    int* flag = reinterpret_cast<int*>(c->ws + c->layout.flag);
    const bool check = (c->prm.flags & ZM_FLAG_CHECK_FINITE) != 0;
    hipError_t e;
    if (check) {
        e = hipMemsetAsync(flag, 0, sizeof(int), c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "flag clear");
    }
    const bool graph = (c->prm.flags & ZM_FLAG_GRAPH) && !c->profiling;
    if (graph && nsteps > 0) {
        zm_status st = ensure_graph(c);
        if (st != ZM_OK) return st;
    }
    for (int step = 0; step < nsteps; ++step) {
        if (graph) {
            e = hipGraphLaunch(c->graph, c->stream);
            if (e != hipSuccess) return hip_fail(c, e, "graph launch");
        } else {
            zm_status st = enqueue_step(c, c->stream);
            if (st != ZM_OK) return st;
        }
    }
    if (check) {
        int host_flag = 0;
        e = hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "flag read");
        if (host_flag) return fail(c, ZM_ERR_NONFINITE, "state became non-finite");
    }
    return ZM_OK;
}

zm_status zm_destroy(zm_ctx* c)
{
    if (!c) return ZM_OK;
    zm_status st = ZM_OK;
    {
        DeviceGuard g(c->device);
        if (g.ok && hipStreamSynchronize(c->stream) != hipSuccess) st = ZM_ERR_HIP;
        for (auto& t : c->pending) {
            (void)hipEventDestroy(t.start);
            (void)hipEventDestroy(t.stop);
        }
        for (auto e : c->spare) (void)hipEventDestroy(e);
        if (c->graph) (void)hipGraphExecDestroy(c->graph);
        if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    }
    delete c;
    return st;
}

const char* zm_status_string(zm_status s)
{
    switch (s) {
    case ZM_OK: return "ok";
    case ZM_ERR_INVALID_ARG: return "invalid argument";
    case ZM_ERR_UNSUPPORTED: return "unsupported";
    case ZM_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case ZM_ERR_HIP: return "HIP runtime error";
    case ZM_ERR_NONFINITE: return "non-finite state";
    case ZM_ERR_CAPACITY: return "capacity exceeded";
    default: return "unknown status";
    }
}

const char* zm_last_error(const zm_ctx* c)
{
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

zm_status zm_get_launch_info(const zm_ctx* c, zm_launch_info* out)
{
    if (!c || !out) return ZM_ERR_INVALID_ARG;
    if (c->cutoff) {
        const zm::CutGrid& g = c->cut;
        out->targets_per_lane = 1;
        out->patch_cols = g.B;   // in cells
        out->patch_rows = g.B;
        out->source_splits = g.planes;
        out->workgroups = g.nb1 * g.nb2 * g.slots;
        out->threads_per_group = 256;
        out->pairs_per_eval = (int64_t)c->mesh.N * (int64_t)c->mesh.N;
        return ZM_OK;
    }
    const zm::PairShape& sh = c->shape;
    out->targets_per_lane = sh.R;
    out->patch_cols = sh.cx;
    out->patch_rows = sh.prow;
    out->source_splits = sh.splits;
    out->workgroups = sh.px * sh.py * sh.splits;
    out->threads_per_group = 256;
    const int64_t side = 2 * (int64_t)c->mesh.K + 1;
    out->pairs_per_eval = (int64_t)c->mesh.N * (int64_t)c->mesh.N * side * side;
    return ZM_OK;
}

zm_status zm_profile_enable(zm_ctx* c, int32_t on)
{
    if (!c) return ZM_ERR_INVALID_ARG;
    if (on && !c->profiling && c->cutoff) {
        DeviceGuard g(c->device);
        if (!g.ok) return fail(c, ZM_ERR_HIP, "cannot select the context device");
        hipError_t e = zm::launch_cut_count_reset(c->cb.counts, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "pair counter reset");
    }
    c->profiling = (on != 0);
    return ZM_OK;
}

zm_status zm_cutoff_info_get(zm_ctx* c, zm_cutoff_info* out)
{
    if (!c || !out) return ZM_ERR_INVALID_ARG;
    if (!c->cutoff) return fail(c, ZM_ERR_UNSUPPORTED, "not a cutoff context");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, ZM_ERR_HIP, "cannot select the context device");
    static_assert(zm::kCutPathCells == ZM_CUT_PATH_CELLS && zm::kCutPathWindow == ZM_CUT_PATH_WINDOW &&
                      zm::kCutPathStencil == ZM_CUT_PATH_STENCIL,
                  "path bits");
    unsigned long long h[zm::kCutCountWords] = {0, 0, 0};
    hipError_t e = hipMemcpyAsync(h, c->cb.counts, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = zm::launch_cut_count_reset(c->cb.counts, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "pair counter read");
    out->cells1 = c->cut.nc1;
    out->cells2 = c->cut.nc2;
    out->cells_per_cutoff = c->cut.m;
    out->block_cells = c->cut.B;
    out->slots = c->cut.planes;
    out->paths = (int32_t)h[2];
    out->pairs_tested = (int64_t)h[0];
    out->pairs_accepted = (int64_t)h[1];
    return ZM_OK;
}

zm_status zm_profile_read(zm_ctx* c, zm_kernel_stats* out)
{
    if (!c || !out) return ZM_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    if (!g.ok) return fail(c, ZM_ERR_HIP, "cannot select the context device");
    zm_status st = ZM_OK;
    for (auto& t : c->pending) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.start, t.stop);
        if (e != hipSuccess) {
            st = hip_fail(c, e, "event timing");
        } else {
            c->stats[t.kernel].launches += 1;
            c->stats[t.kernel].total_ms += (double)ms;
        }
        c->spare.push_back(t.start);
        c->spare.push_back(t.stop);
    }
    c->pending.clear();
    std::memcpy(out, c->stats, sizeof(c->stats));
    std::memset(c->stats, 0, sizeof(c->stats));
    return st;
}

int32_t zm_abi_version(void) { return 5; }

}  // extern "C"
