// Process-wide launch-shape table and the autotuner (zm_tuning_*,
// zm_autotune* in include/zm.h).
#include "zm.h"
#include "zm_batch_internal.h"
#include "zm_host.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

namespace {

std::mutex g_mu;
std::map<std::tuple<int, int, int>, zm_pair_tuning> g_table;

bool valid_tuning(const zm_pair_tuning& t)
{
    return (t.targets_per_lane == 1 || t.targets_per_lane == 2 || t.targets_per_lane == 4) &&
           t.source_splits >= 1;
}

// Candidate shapes: R in {1, 2, 4} x splits in {s0/4, s0/2, s0, 2 s0, 4 s0,
// 8 s0} where s0 is the split count giving >= 2048 workgroups for that R,
// clamped to [1, n2], plus the untuned default shape, deduplicated; for the
// FP32 form only the R whose patches keep its error bound.  (Finer splits
// pay in FP32: 8 s0 at 256 x 256.)
std::vector<zm::PairShape> candidates(const zm_params& p)
{
    std::vector<zm::PairShape> out;
    auto add = [&](const zm::PairShape& sh) {
        bool dup = false;
        for (const auto& o : out) dup |= (o.R == sh.R && o.splits == sh.splits);
        if (!dup) out.push_back(sh);
    };
    for (int R : {1, 2, 4}) {
        const zm::PairShape d = zm::make_pair_shape(p.n1, p.n2, p.precision, R, 0);
        if (zm::fp32_shape_problem(p, d)) continue;
        for (int f : {-2, -1, 0, 1, 2, 3}) {
            int s = f < 0 ? d.splits >> (-f) : d.splits << f;
            add(zm::make_pair_shape(p.n1, p.n2, p.precision, R, std::max(1, s)));
        }
    }
    const zm::PairShape d = zm::default_pair_shape(p.n1, p.n2, p.precision);
    if (!zm::fp32_shape_problem(p, d)) add(d);
    return out;
}

struct TuneLayout {
    size_t z, gam, part, total;
};

TuneLayout tune_layout(const zm_params& p)
{
    const size_t N = (size_t)p.n1 * p.n2, d = sizeof(double);
    int max_splits = 1;
    for (const auto& sh : candidates(p)) max_splits = std::max(max_splits, sh.splits);
    TuneLayout L;
    L.z = 0;
    L.gam = zm::align_up(3 * N * d);
    L.part = L.gam + zm::align_up(3 * N * d);
    L.total = L.part + zm::align_up((size_t)max_splits * 3 * N * d);
    return L;
}

// ---- batch tuning ---------------------------------------------------------
//
// A batch runs every member's pair sweep in one persistent launch per (pair
// form, targets per lane), so the best shape of a mesh size depends on the
// rest of the batch: small members need few source splits there (the other
// members keep the device busy, and every item pays its staging and
// work-counter cost), unlike a solo launch that must fill the device alone.
// The batch tuner therefore times the batched sweep itself.  Candidates of a
// size: targets per lane 1, 2, 4 (for FP32 only shapes the form accepts) x
// source splits 1, 2, 4, ... up to n2 and the solo candidates' counts.

using Key = std::tuple<int, int, int>;

Key key_of(const zm_params& p) { return Key{p.n1, p.n2, p.precision}; }

std::vector<zm::PairShape> batch_candidates(const zm_params& p)
{
    std::vector<zm::PairShape> out;
    auto add = [&](const zm::PairShape& sh) {
        if (zm::fp32_shape_problem(p, sh)) return;
        for (const auto& o : out)
            if (o.R == sh.R && o.splits == sh.splits) return;
        out.push_back(sh);
    };
    for (int R : {1, 2, 4}) {
        for (int s = 1; s <= p.n2; s *= 2) add(zm::make_pair_shape(p.n1, p.n2, p.precision, R, s));
        add(zm::make_pair_shape(p.n1, p.n2, p.precision, R, p.n2));
    }
    for (const auto& sh : candidates(p)) add(sh);
    return out;
}

// Workspace of the batch tuner: per member its positions and source
// strengths (synthetic), and partial sums for the largest candidate split
// count of its size; then the descriptor table, the longest work list any
// candidate set can produce, and the work counters.
struct BatchTuneLayout {
    std::vector<size_t> z, gam, part, fold;
    size_t table = 0, items = 0, counters = 0, total = 0;
    size_t max_items = 0;
};

BatchTuneLayout batch_tune_layout(const zm_params* params, int count)
{
    BatchTuneLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = zm::align_up(o + bytes); return at; };
    for (int i = 0; i < count; ++i) {
        const zm_params& p = params[i];
        const size_t N = (size_t)p.n1 * p.n2, d = sizeof(double);
        int max_splits = 1;
        size_t max_items = 0;
        for (const auto& sh : batch_candidates(p)) {
            max_splits = std::max(max_splits, sh.splits);
            max_items = std::max(max_items, (size_t)sh.px * sh.py * sh.splits);
        }
        L.z.push_back(take(3 * N * d));
        L.gam.push_back(take(3 * N * d));
        L.part.push_back(take((size_t)max_splits * 3 * N * d));
        L.fold.push_back(take(zm::kFoldWords * sizeof(int)));
        L.max_items += max_items;
    }
    L.table = take(sizeof(zm::InstDesc) * count);
    L.items = take(sizeof(zm::WorkItem) * std::max<size_t>(1, L.max_items));
    L.counters = take(zm::kMaxPairGroups * sizeof(int));
    L.total = o;
    return L;
}

const char* batch_tune_check(const zm_params* params, int32_t count)
{
    if (!params) return "params is NULL";
    if (count < 1 || count > (1 << 20)) return "count must be in [1, 2^20]";
    for (int i = 0; i < count; ++i) {
        if (const char* why = zm::validate(&params[i])) return why;
        if (params[i].cutoff != 0.0 || params[i].model != ZM_MODEL_HIGH ||
            params[i].boundary != ZM_BOUNDARY_PERIODIC)
            return "batches take the exact high-order model on periodic sheets only";
        if (batch_candidates(params[i]).empty())
            return "the FP32 pair form is refused on a member's mesh";
    }
    return nullptr;
}

}  // namespace

namespace zm {

bool lookup_tuning(int n1, int n2, int precision, int* R, int* splits)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find({n1, n2, precision});
    if (it == g_table.end()) return false;
    *R = it->second.targets_per_lane;
    *splits = it->second.source_splits;
    return true;
}

}  // namespace zm

extern "C" {

zm_status zm_tuning_set(int32_t n1, int32_t n2, int32_t precision, const zm_pair_tuning* t)
{
    if (n1 < 8 || n2 < 8 || (precision != ZM_FP64 && precision != ZM_FP32_PAIRS))
        return ZM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!t) {
        g_table.erase({n1, n2, precision});
        return ZM_OK;
    }
    if (!valid_tuning(*t)) return ZM_ERR_INVALID_ARG;
    g_table[{n1, n2, precision}] = *t;
    return ZM_OK;
}

zm_status zm_tuning_get(int32_t n1, int32_t n2, int32_t precision, zm_pair_tuning* out)
{
    if (!out || n1 < 8 || n2 < 8 || (precision != ZM_FP64 && precision != ZM_FP32_PAIRS))
        return ZM_ERR_INVALID_ARG;
    const zm::PairShape sh = zm::choose_pair_shape(n1, n2, precision);
    out->targets_per_lane = sh.R;
    out->source_splits = sh.splits;
    return ZM_OK;
}

size_t zm_autotune_workspace_bytes(const zm_params* params)
{
    if (zm::validate(params) || candidates(*params).empty()) return 0;
    return tune_layout(*params).total;
}

zm_status zm_autotune(const zm_params* params, void* d_workspace, size_t workspace_bytes,
                      void* hip_stream, zm_pair_tuning* best, double* best_ms)
{
    if (zm::validate(params)) return ZM_ERR_INVALID_ARG;
    if (candidates(*params).empty()) return ZM_ERR_UNSUPPORTED;   // FP32 form refused on this mesh
    const TuneLayout L = tune_layout(*params);
    if (!zm::aligned(d_workspace) || workspace_bytes < L.total) return ZM_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    char* ws = reinterpret_cast<char*>(d_workspace);
    double* z = reinterpret_cast<double*>(ws + L.z);
    double* gam = reinterpret_cast<double*>(ws + L.gam);
    double* part = reinterpret_cast<double*>(ws + L.part);
    const zm::Mesh m = zm::make_mesh(*params);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    zm_status st = ZM_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = ZM_ERR_HIP;
    if (st == ZM_OK && zm::launch_tune_init(m, z, gam, s) != hipSuccess) st = ZM_ERR_HIP;
    double best_t = 1e300;
    zm::PairShape best_sh{};
    if (st == ZM_OK) {
        for (const zm::PairShape& sh : candidates(*params)) {
            auto launch = [&] {
                return params->precision == ZM_FP32_PAIRS
                           ? zm::launch_pairs_f32(m, sh, z, gam, part, nullptr, s)
                           : zm::launch_pairs_f64(m, sh, z, gam, part, nullptr, s);
            };
            if (launch() != hipSuccess) { st = ZM_ERR_HIP; break; }   // warm-up
            float times[3];
            bool ok = true;
            for (float& t : times) {
                ok = ok && hipEventRecord(e0, s) == hipSuccess && launch() == hipSuccess &&
                     hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&t, e0, e1) == hipSuccess;
            }
            if (!ok) { st = ZM_ERR_HIP; break; }
            std::sort(times, times + 3);
            if (times[1] < best_t) { best_t = times[1]; best_sh = sh; }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != ZM_OK) return st;
    zm_pair_tuning t{best_sh.R, best_sh.splits};
    zm_status r = zm_tuning_set(params->n1, params->n2, params->precision, &t);
    if (r != ZM_OK) return r;
    if (best) *best = t;
    if (best_ms) *best_ms = best_t;
    return ZM_OK;
}

size_t zm_batch_autotune_workspace_bytes(const zm_params* params, int32_t count)
{
    if (batch_tune_check(params, count)) return 0;
    return batch_tune_layout(params, count).total;
}

zm_status zm_batch_autotune(const zm_params* params, int32_t count, void* d_workspace,
                            size_t workspace_bytes, void* hip_stream, zm_pair_tuning* best,
                            double* best_ms)
{
    if (batch_tune_check(params, count)) return ZM_ERR_INVALID_ARG;
    const BatchTuneLayout L = batch_tune_layout(params, count);
    if (!zm::aligned(d_workspace) || workspace_bytes < L.total) return ZM_ERR_WORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    char* ws = reinterpret_cast<char*>(d_workspace);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return ZM_ERR_HIP;

    // distinct sizes, largest total pair work first; start from the shapes
    // new contexts would take now
    std::map<Key, double> work;
    for (int i = 0; i < count; ++i) {
        const double N = (double)params[i].n1 * params[i].n2;
        const double side = 2.0 * params[i].image_layers + 1.0;
        work[key_of(params[i])] += N * N * side * side;
    }
    std::vector<Key> keys;
    for (const auto& kv : work) keys.push_back(kv.first);
    std::stable_sort(keys.begin(), keys.end(),
                     [&](const Key& a, const Key& b) { return work[a] > work[b]; });
    std::map<Key, zm::PairShape> shape;
    std::map<Key, int> first;   // a member of each size (its params give the candidates)
    for (int i = 0; i < count; ++i) {
        const Key k = key_of(params[i]);
        if (!shape.count(k)) {
            shape[k] = zm::choose_pair_shape(params[i].n1, params[i].n2, params[i].precision);
            if (zm::fp32_shape_problem(params[i], shape[k])) shape[k] = batch_candidates(params[i])[0];
            first[k] = i;
        }
    }

    // synthetic inputs of every member
    std::vector<zm::Layout> layouts(count);
    std::vector<char*> bases(count, ws);
    for (int i = 0; i < count; ++i) {
        zm::Layout& l = layouts[i];
        std::memset(&l, 0, sizeof(l));
        l.y0 = l.y1 = l.y2 = L.z[i];
        l.gam = L.gam[i];
        l.part = L.part[i];
        l.q = l.tie = l.u = l.V = L.z[i];   // not touched by the pair sweep
        l.fold = L.fold[i];                 // cleared: the far forms are allowed
        const zm::Mesh m = zm::make_mesh(params[i]);
        if (zm::launch_tune_init(m, reinterpret_cast<double*>(ws + L.z[i]),
                                 reinterpret_cast<double*>(ws + L.gam[i]), s) != hipSuccess ||
            hipMemsetAsync(ws + L.fold[i], 0, zm::kFoldWords * sizeof(int), s) != hipSuccess)
            return ZM_ERR_HIP;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return ZM_ERR_HIP;
    }
    zm::InstDesc* dtable = reinterpret_cast<zm::InstDesc*>(ws + L.table);
    zm::WorkItem* ditems = reinterpret_cast<zm::WorkItem*>(ws + L.items);
    int* counters = reinterpret_cast<int*>(ws + L.counters);

    // time of one batched pair sweep with the current shapes (fastest of two
    // after a warm-up)
    auto time_sweep = [&](float* out) -> zm_status {
        std::vector<zm::PairShape> sh(count);
        for (int i = 0; i < count; ++i) sh[i] = shape[key_of(params[i])];
        zm::TableBuild tb;
        zm::build_tables(params, sh.data(), layouts.data(), bases.data(), nullptr, count, tb);
        if (tb.items.size() > L.max_items) return ZM_ERR_WORKSPACE;
        if (hipMemcpyAsync(dtable, tb.table.data(), sizeof(zm::InstDesc) * count,
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(ditems, tb.items.data(), sizeof(zm::WorkItem) * tb.items.size(),
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return ZM_ERR_HIP;
        zm::BatchLaunch bl{};
        bl.table = dtable;
        bl.count = count;
        bl.items = ditems;
        bl.ngroups = (int)tb.groups.size();
        for (int g = 0; g < bl.ngroups; ++g) bl.groups[g] = tb.groups[g];
        bl.counters = counters;
        bl.persistent_groups = 4 * (cus > 0 ? cus : 256);
        float t = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            float ms = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess || zm::launch_batch_pairs(bl, 0, s) != hipSuccess ||
                hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                return ZM_ERR_HIP;
            if (rep > 0) t = std::min(t, ms);   // rep 0 warms up
        }
        *out = t;
        return ZM_OK;
    };

    zm_status st = ZM_OK;
    float best_t = 0.f;
    st = time_sweep(&best_t);
    for (size_t k = 0; st == ZM_OK && k < keys.size(); ++k) {
        const Key key = keys[k];
        zm::PairShape keep = shape[key];
        for (const zm::PairShape& c : batch_candidates(params[first[key]])) {
            if (c.R == keep.R && c.splits == keep.splits) continue;
            shape[key] = c;
            float t = 0.f;
            st = time_sweep(&t);
            if (st != ZM_OK) break;
            if (t < best_t) { best_t = t; keep = c; }
        }
        shape[key] = keep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ZM_OK) return st;
    for (const Key& key : keys) {
        const zm_pair_tuning t{shape[key].R, shape[key].splits};
        const zm_status r = zm_tuning_set(std::get<0>(key), std::get<1>(key), std::get<2>(key), &t);
        if (r != ZM_OK) return r;
    }
    if (best)
        for (int i = 0; i < count; ++i) {
            const zm::PairShape& sh = shape[key_of(params[i])];
            best[i] = zm_pair_tuning{sh.R, sh.splits};
        }
    if (best_ms) *best_ms = best_t;
    return ZM_OK;
}

}  // extern "C"
