// Allocation-free Birkhoff-Rott evaluation (zm_br_velocity_noalloc in
// include/zm.h), for callers that cannot allocate device memory at all.
//
// The evaluation runs the same kernels as zm_br_velocity on a context --
// k_surface, k_pairs (FP64 or FP32 form), k_ties for even sides, k_reduce --
// with their scratch (source strengths, q, tie corrections, per-split
// partial sums) carved from one file-scope device array instead of a caller
// workspace.  The array exists once per device the library runs on and lives
// until the process ends.  Host code never passes the array's name to a
// kernel: its device address is looked up once per device with
// hipGetSymbolAddress and kept.
#include "zm.h"
#include "zm_host.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>
#include <string>

static_assert(ZM_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) unsigned char scratch[ZM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use;
// the caller's device is current).
hipError_t scratch_of(int dev, char** out)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<char*>(g_scratch_ptr[dev]);
    return hipSuccess;
}

struct NoallocLayout {
    size_t fold, gam, q, tie, part, total;
};

NoallocLayout noalloc_layout(size_t N, bool ties, int splits)
{
    const size_t d = sizeof(double);
    NoallocLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = zm::align_up(o + bytes); return at; };
    // fold statistics: zero when the array is loaded, and cleared again by
    // the last surface workgroup of every call
    L.fold = take(zm::kFoldWords * sizeof(int));
    L.gam = take(3 * N * d);
    L.q = take(N * d);
    L.tie = take(ties ? 6 * N * d : 0);
    L.part = take((size_t)splits * 3 * N * d);
    L.total = o;
    return L;
}

zm_status reject(zm_status st, const std::string& msg)
{
    zm::set_create_error(msg);
    return st;
}

}  // namespace

extern "C" zm_status zm_br_velocity_noalloc(const zm_params* params, const double* d_z,
                                            const double* d_w, double* d_u, void* hip_stream)
{
    zm::set_create_error("");
    if (const char* why = zm::validate(params)) return reject(ZM_ERR_INVALID_ARG, why);
    if (params->cutoff > 0.0 || params->model == ZM_MODEL_LOW)
        return reject(ZM_ERR_UNSUPPORTED, "the allocation-free call evaluates the exact BR sum only "
                                          "(cutoff = 0, high or medium order)");
    if (!zm::aligned(d_z) || !zm::aligned(d_w) || !zm::aligned(d_u))
        return reject(ZM_ERR_INVALID_ARG, "pointers must be non-NULL and 256-byte aligned");
    const zm::Mesh m = zm::make_mesh(*params);
    const size_t N = (size_t)m.N, d = sizeof(double);
    if (zm::overlaps(d_u, 3 * N * d, d_z, 3 * N * d) || zm::overlaps(d_u, 3 * N * d, d_w, 2 * N * d))
        return reject(ZM_ERR_INVALID_ARG, "d_u overlaps an input");
    const bool ties = m.periodic && ((m.n1 % 2) == 0 || (m.n2 % 2) == 0);

    // The context's shape when its partial sums fit the scratch (bitwise the
    // same result as zm_br_velocity); otherwise the same targets per lane
    // with as many source ranges as fit (a different summation order).
    zm::PairShape sh = zm::choose_pair_shape(params->n1, params->n2, params->precision);
    const size_t fixed = noalloc_layout(N, ties, 0).total;
    if (noalloc_layout(N, ties, sh.splits).total > ZM_NOALLOC_SCRATCH_BYTES) {
        const size_t per_split = zm::align_up(3 * N * d);
        const size_t room = ZM_NOALLOC_SCRATCH_BYTES > fixed ? ZM_NOALLOC_SCRATCH_BYTES - fixed : 0;
        const int fit = (int)(room / per_split);
        if (fit < 1)
            return reject(ZM_ERR_CAPACITY,
                          "mesh too large for the allocation-free call: it needs " +
                              std::to_string(fixed + per_split) + " bytes of scratch, " +
                              std::to_string((size_t)ZM_NOALLOC_SCRATCH_BYTES) +
                              " are available (use a context with a workspace)");
        sh = zm::make_pair_shape(params->n1, params->n2, params->precision, sh.R,
                                 fit < sh.splits ? fit : sh.splits);
        // make_pair_shape rounds the range count; keep within the room
        while (sh.splits > 1 && noalloc_layout(N, ties, sh.splits).total > ZM_NOALLOC_SCRATCH_BYTES)
            sh = zm::make_pair_shape(params->n1, params->n2, params->precision, sh.R,
                                     sh.splits - 1);
    }
    if (const char* why = zm::fp32_shape_problem(*params, sh)) return reject(ZM_ERR_UNSUPPORTED, why);
    const NoallocLayout L = noalloc_layout(N, ties, sh.splits);
    if (L.total > ZM_NOALLOC_SCRATCH_BYTES)
        return reject(ZM_ERR_CAPACITY, "mesh too large for the allocation-free call");

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return reject(ZM_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return reject(ZM_ERR_UNSUPPORTED, "device index above 63");
    char* base = nullptr;
    e = scratch_of(dev, &base);
    if (e != hipSuccess)
        return reject(ZM_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));

    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    double* gam = reinterpret_cast<double*>(base + L.gam);
    double* q = reinterpret_cast<double*>(base + L.q);
    double* tie = reinterpret_cast<double*>(base + L.tie);
    double* part = reinterpret_cast<double*>(base + L.part);
    int* fold = reinterpret_cast<int*>(base + L.fold);
    e = zm::launch_surface(m, d_z, d_w, gam, q, fold, s);
    if (e == hipSuccess)
        e = params->precision == ZM_FP32_PAIRS
                ? zm::launch_pairs_f32(m, sh, d_z, gam, part, fold, s)
                : zm::launch_pairs_f64(m, sh, d_z, gam, part, fold, s);
    if (e == hipSuccess && ties) e = zm::launch_ties(m, d_z, gam, tie, s);
    if (e == hipSuccess)
        e = zm::launch_reduce(m, sh.splits, part, tie, q, d_z, d_u, nullptr, s, m.periodic != 0);
    if (e != hipSuccess) return reject(ZM_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
    return ZM_OK;
}
