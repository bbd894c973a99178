// Host-side helpers shared by the single-instance and batched runtimes.
#pragma once

#include "zm.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>

namespace zm {

// Message zm_last_error(NULL) returns on this thread (zm_create and the
// allocation-free evaluation record why they refused a call).
void set_create_error(const std::string& msg);

constexpr size_t kAlign = 256;
constexpr int kMaxSide = 8192;
constexpr int kMaxImages = 16;

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace regions, all 256-byte aligned, in bytes from the base.
struct Layout {
    size_t y0, y1, y2;   // 5N doubles each (z1 z2 z3 w1 w2)
    size_t gam, q;       // 3N, N
    size_t part;         // max(splits, cutoff slots) * 3N
    size_t tie;          // 6N
    size_t u, V;         // 3N, N
    size_t flag;         // one int
    size_t fold;         // kFoldWords ints: tangent-map statistics, far-form flag
    // cutoff solver only (size 0 otherwise)
    size_t cut_keys[2], cut_vals[2];   // N unsigned each
    size_t cut_hist;                   // 256 * sort_blocks unsigned
    size_t cut_start, cut_end;         // nkeys int each
    size_t cut_bstart, cut_bend;       // target blocks, int each
    size_t cut_src;                    // 8N doubles
    size_t cut_counts;                 // kCutCountWords uint64
    size_t cut_kflag;                  // nkeys int
    // low-order model only (size 0 otherwise)
    size_t lo_a, lo_b;                 // N double2 each
    size_t lo_tw1, lo_tw2;             // n1, n2 double2
    size_t total;
};

inline bool has_cutoff(const zm_params& p) { return p.cutoff > 0.0; }

inline CutGrid cut_grid_of(const zm_params& p)
{
    return make_cut_grid(p.n1, p.n2, p.period1, p.period2, p.cutoff,
                         p.boundary != ZM_BOUNDARY_FREE);
}

inline Layout make_layout(const zm_params& p, const zm::PairShape& sh)
{
    const size_t N = (size_t)p.n1 * (size_t)p.n2;
    const size_t d = sizeof(double);
    const bool cut = has_cutoff(p);
    const CutGrid g = cut ? cut_grid_of(p) : CutGrid();
    const int slots = cut ? (g.planes > sh.splits ? g.planes : sh.splits) : sh.splits;
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    L.y0 = take(5 * N * d);
    L.y1 = take(5 * N * d);
    L.y2 = take(5 * N * d);
    L.gam = take(3 * N * d);
    L.q = take(N * d);
    L.part = take((size_t)slots * 3 * N * d);
    L.tie = take(6 * N * d);
    L.u = take(3 * N * d);
    L.V = take(N * d);
    L.flag = take(sizeof(int));
    L.fold = take(kFoldWords * sizeof(int));
    const size_t u4 = sizeof(unsigned);
    L.cut_keys[0] = take(cut ? N * u4 : 0);
    L.cut_keys[1] = take(cut ? N * u4 : 0);
    L.cut_vals[0] = take(cut ? N * u4 : 0);
    L.cut_vals[1] = take(cut ? N * u4 : 0);
    L.cut_hist = take(cut ? (size_t)256 * g.sort_blocks * u4 : 0);
    L.cut_start = take(cut ? (size_t)g.nkeys * sizeof(int) : 0);
    L.cut_end = take(cut ? (size_t)g.nkeys * sizeof(int) : 0);
    L.cut_bstart = take(cut ? (size_t)g.nb1 * g.nb2 * sizeof(int) : 0);
    L.cut_bend = take(cut ? (size_t)g.nb1 * g.nb2 * sizeof(int) : 0);
    L.cut_src = take(cut ? 8 * N * d : 0);
    L.cut_counts = take(cut ? kCutCountWords * sizeof(unsigned long long) : 0);
    L.cut_kflag = take(cut ? (size_t)g.nkeys * sizeof(int) : 0);
    const bool low = p.model == ZM_MODEL_LOW || p.model == ZM_MODEL_MEDIUM;   // FFT buffers
    const size_t c16 = 2 * sizeof(double);
    L.lo_a = take(low ? N * c16 : 0);
    L.lo_b = take(low ? N * c16 : 0);
    L.lo_tw1 = take(low ? (size_t)p.n1 * c16 : 0);
    L.lo_tw2 = take(low ? (size_t)p.n2 * c16 : 0);
    L.total = o;
    return L;
}

// FP32 pair form: sources are staged as FP32 offsets from a patch centre,
// so a pair's r carries an absolute error of about ulp(patch extent) while
// near pairs sit about one mesh spacing apart.  The form keeps its error
// bound (1e-5 normwise; 6.5e-7 measured at 36 spacings) while the patch
// extent stays within this many finest spacings; beyond it (very
// anisotropic meshes, e.g. 8192 x 8 on a square period) the FP32 form is
// refused and FP64 must be used.
constexpr double kF32MaxExtentSpacings = 128.0;

// Reason the FP32 pair form cannot serve these params with this shape, or
// nullptr (always nullptr for FP64).
inline const char* fp32_shape_problem(const zm_params& p, const zm::PairShape& sh)
{
    if (p.precision != ZM_FP32_PAIRS) return nullptr;
    const double h1 = p.period1 / p.n1, h2 = p.period2 / p.n2;
    const double cols = sh.cx < p.n1 ? sh.cx : p.n1;
    const double rows = sh.prow < p.n2 ? sh.prow : p.n2;
    const double ext = std::sqrt(cols * cols * h1 * h1 + rows * rows * h2 * h2);
    if (ext <= kF32MaxExtentSpacings * std::fmin(h1, h2)) return nullptr;
    return "the FP32 pair form needs patches within 128 finest mesh spacings (this mesh is too "
           "anisotropic for it); use FP64";
}

inline const char* validate(const zm_params* p)
{
    if (!p) return "params is NULL";
    if (p->n1 < 8 || p->n2 < 8) return "n1 and n2 must be >= 8";
    if (p->n1 > kMaxSide || p->n2 > kMaxSide) return "n1 and n2 must be <= 8192";
    if (!(std::isfinite(p->period1) && p->period1 > 0.0)) return "period1 must be finite and > 0";
    if (!(std::isfinite(p->period2) && p->period2 > 0.0)) return "period2 must be finite and > 0";
    if (!(std::isfinite(p->eps) && p->eps > 0.0)) return "eps must be finite and > 0";
    if (!(std::isfinite(p->dt) && p->dt > 0.0)) return "dt must be finite and > 0";
    if (!(std::isfinite(p->nu) && p->nu >= 0.0)) return "nu must be finite and >= 0";
    if (!std::isfinite(p->atwood)) return "atwood must be finite";
    if (!std::isfinite(p->gravity)) return "gravity must be finite";
    if (p->precision != ZM_FP64 && p->precision != ZM_FP32_PAIRS) return "unknown precision";
    if (p->image_layers < 0 || p->image_layers > kMaxImages) return "image_layers must be in [0, 16]";
    if (p->flags & ~(ZM_FLAG_CHECK_FINITE | ZM_FLAG_GRAPH)) return "unknown flag bits";
    if (p->model != ZM_MODEL_HIGH && p->model != ZM_MODEL_LOW && p->model != ZM_MODEL_MEDIUM)
        return "unknown model";
    if (p->model == ZM_MODEL_LOW && (p->cutoff != 0.0 || p->image_layers != 0))
        return "the low-order model takes no cutoff and no image layers";
    if (p->boundary != ZM_BOUNDARY_PERIODIC && p->boundary != ZM_BOUNDARY_FREE)
        return "unknown boundary";
    if (p->boundary == ZM_BOUNDARY_FREE && (p->model != ZM_MODEL_HIGH || p->image_layers != 0))
        return "a free sheet needs the high-order model and no image layers";
    if (p->reserved != 0) return "reserved must be 0";
    if (!(std::isfinite(p->cutoff) && p->cutoff >= 0.0)) return "cutoff must be finite and >= 0";
    if (p->cutoff > 0.0) {
        if (p->boundary == ZM_BOUNDARY_PERIODIC &&
            (p->cutoff > 0.45 * p->period1 || p->cutoff > 0.45 * p->period2))
            return "cutoff must be <= 0.45 min(period1, period2) on a periodic sheet";
        if (p->image_layers != 0) return "cutoff needs image_layers = 0";
    }
    return nullptr;
}

inline bool aligned(const void* p) { return p && ((uintptr_t)p % kAlign) == 0; }

inline bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Makes the context's device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline Mesh make_mesh(const zm_params& p)
{
    Mesh m;
    m.n1 = p.n1;
    m.n2 = p.n2;
    m.N = p.n1 * p.n2;
    m.K = p.image_layers;
    m.L1 = p.period1;
    m.L2 = p.period2;
    m.h1 = p.period1 / p.n1;
    m.h2 = p.period2 / p.n2;
    m.eps2 = p.eps * p.eps;
    m.coef = -(m.h1 * m.h2) / (4.0 * M_PI);
    m.atwood = p.atwood;
    m.gravity = p.gravity;
    m.nu = p.nu;
    m.dt = p.dt;
    m.periodic = p.boundary == ZM_BOUNDARY_FREE ? 0 : 1;
    m.pad_ = 0;
    return m;
}

}  // namespace zm
