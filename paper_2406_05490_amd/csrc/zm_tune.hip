// Process-wide launch-shape table and the autotuner (zm_tuning_*,
// zm_autotune* in include/zm.h).
#include "zm.h"
#include "zm_host.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
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
                           ? zm::launch_pairs_f32(m, sh, z, gam, part, s)
                           : zm::launch_pairs_f64(m, sh, z, gam, part, s);
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

}  // extern "C"
