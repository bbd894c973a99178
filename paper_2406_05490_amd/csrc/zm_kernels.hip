// Single-instance kernels: thin wrappers that map the launch grid onto the
// device bodies in zm_device.h, plus the launch-shape choice and launchers.
#include "zm_device.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace zm {
namespace {

using dev::kThreads;

// One point per thread.  PER: 1 periodic sheet, 0 free sheet (the stencils
// without the other boundary's branches).  Every workgroup adds its points'
// tangent-map statistics to the fold words; k_fold_finish, the next launch
// on the stream, turns them into this evaluation's flag (the kernel boundary
// orders every workgroup's atomics before its reads).
template <int PER>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_surface(Mesh m, const double* __restrict__ z,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ gam,
                                                      double* __restrict__ q,
                                                      int* __restrict__ fold)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    const dev::FoldStat st = dev::surface_point<PER>(m, p, z, w, gam, q);   // identity past N
    if (fold) dev::fold_accumulate(st, fold);
}

__global__ void k_fold_finish(int* __restrict__ fold)
{
    if (threadIdx.x == 0) dev::fold_finish(fold);
}

// Workgroups are dealt round-robin to the 8 XCDs.  The pair kernels give
// each XCD one contiguous run of the split-major (patch, split) work list, so
// that the workgroups an XCD runs at one time share a split and its sources
// stay in that XCD's L2 (dealt round-robin, every XCD would run patches of
// every split and read every split's sources).  A bijection of the grid.
constexpr int kXcds = 8;

__device__ __forceinline__ void pair_item(int& patch, int& split)
{
    const int total = (int)(gridDim.x * gridDim.y);
    const int L = (int)(blockIdx.x + gridDim.x * blockIdx.y);
    const int xcd = L % kXcds, per = total / kXcds, rem = total % kXcds;
    const int item = xcd * per + min(xcd, rem) + L / kXcds;
    patch = item % (int)gridDim.x;
    split = item / (int)gridDim.x;
}

template <int R, int PX>
__global__ __launch_bounds__(kThreads) void k_pairs_f64f(Mesh m, PairShape sh,
                                                         const double* __restrict__ z,
                                                         const double* __restrict__ gam,
                                                         double* __restrict__ part,
                                                         const int* __restrict__ fold)
{
    __shared__ dev::F64Tile lds;
    int patch, split;
    pair_item(patch, split);
    dev::pairs_f64f_block<R, PX>(m, sh, z, gam, part, patch, split, fold, lds);
}

template <int R, int PX>
__global__ __launch_bounds__(kThreads) void k_pairs_f32(Mesh m, PairShape sh,
                                                        const double* __restrict__ z,
                                                        const double* __restrict__ gam,
                                                        double* __restrict__ part,
                                                        const int* __restrict__ fold)
{
    __shared__ dev::F32Tile tile;
    int patch, split;
    pair_item(patch, split);
    dev::pairs_f32_block<R, PX>(m, sh, z, gam, part, patch, split, fold, tile);
}

// blockIdx.y = pass (0: tie column, 1: tie row); L threads per target
__global__ __launch_bounds__(kThreads) void k_ties(Mesh m, const double* __restrict__ z,
                                                   const double* __restrict__ gam,
                                                   double* __restrict__ tie)
{
    __shared__ double2 lds[3][kThreads];
    if (blockIdx.y == 0) dev::ties_block<0>(m, blockIdx.x, z, gam, tie, lds);
    else dev::ties_block<1>(m, blockIdx.x, z, gam, tie, lds);
}

__global__ __launch_bounds__(kThreads) void k_reduce(Mesh m, int splits,
                                                     const double* __restrict__ part,
                                                     const double* __restrict__ tie,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ z,
                                                     double* __restrict__ u,
                                                     double* __restrict__ V, int ties)
{
    dev::reduce_thread(m, blockIdx.x * kThreads + threadIdx.x, dev::reduce_lanes(m.N, splits), splits,
                       part, tie, q, z, u, V, ties != 0);
}

// y0 may alias out (see update_point), so neither carries __restrict__.
template <int PER>
__global__ __launch_bounds__(kThreads) void k_update(Mesh m, int stage, const double* y0_z,
                                                     const double* y0_w,
                                                     const double* __restrict__ ys_z,
                                                     const double* __restrict__ ys_w,
                                                     const double* __restrict__ u,
                                                     const double* __restrict__ V,
                                                     double* out_z, double* out_w,
                                                     int* __restrict__ nonfinite)
{
    dev::update_point<PER>(m, blockIdx.x * kThreads + threadIdx.x, stage, y0_z, y0_w, ys_z, ys_w,
                           u, V, out_z, out_w, nonfinite);
}

// Synthetic tuning input: a gently curved mesh with a smooth source strength.
__global__ __launch_bounds__(kThreads) void k_tune_init(Mesh m, double* __restrict__ z,
                                                        double* __restrict__ gam)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= m.N) return;
    const int i2 = p / m.n1, i1 = p - i2 * m.n1;
    const double x = -0.5 * m.L1 + i1 * m.h1, y = -0.5 * m.L2 + i2 * m.h2;
    const double cx = cos(6.283185307179586 * x / m.L1), cy = cos(6.283185307179586 * y / m.L2);
    z[p] = x;
    z[m.N + p] = y;
    z[2 * m.N + p] = 0.01 * cx * cy;
    gam[p] = cy;
    gam[m.N + p] = cx;
    gam[2 * m.N + p] = 0.1 * cx * cy;
}

inline unsigned blocks_for(int n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace


// ---------------------------------------------------------------------------
// launch shapes and launchers
// ---------------------------------------------------------------------------

PairShape make_pair_shape(int n1, int n2, int precision, int R, int splits)
{
    PairShape sh;
    sh.R = R;
    // compact patches keep patch-relative coordinates small
    (void)precision;
    sh.cx = (n1 >= 32) ? 32 : (n1 >= 16 ? 16 : 8);
    sh.prow = (kThreads / sh.cx) * sh.R;
    sh.px = (n1 + sh.cx - 1) / sh.cx;
    sh.py = (n2 + sh.prow - 1) / sh.prow;
    if (splits <= 0) {
        // default: >= 2048 workgroups (8 per CU on 256 CUs)
        const int patches = sh.px * sh.py;
        splits = (2048 + patches - 1) / patches;
    }
    if (splits > n2) splits = n2;
    if (splits < 1) splits = 1;
    sh.rows_per_split = (n2 + splits - 1) / splits;
    sh.splits = (n2 + sh.rows_per_split - 1) / sh.rows_per_split;
    return sh;
}

PairShape default_pair_shape(int n1, int n2, int precision)
{
    // From autotuner runs on MI355X (32^2 .. 1024^2): fewer targets per lane
    // on small meshes (more waves in flight); FP32 prefers 2 targets per lane
    // from 64^2 up, FP64 4 from 128^2 up; twice the default source splits
    // helps FP32 from 64^2 up and FP64 on mid-size meshes.
    const long N = (long)n1 * n2;
    int R;
    if (precision == 1) R = N >= 4096 ? 2 : 1;
    else R = N >= 16384 ? 4 : (N >= 9216 ? 2 : 1);
    const PairShape d = make_pair_shape(n1, n2, precision, R, 0);
    if (precision == 1 && N >= (1L << 20)) {
        // FP32 from 2^20 points up: about 32768 workgroups (at 1024^2, 16
        // source ranges of 64 rows).  Each workgroup then runs for a few
        // milliseconds instead of tens of them, which shortens the tail of
        // the launch: 3-4% faster at 1024^2 than 2 ranges.  The partial sums
        // take splits x N x 24 B, about 400 MB at any size.
        const int patches = d.px * d.py;
        const int s = std::min((32768 + patches - 1) / patches, std::max(1, n2 / 2));
        return make_pair_shape(n1, n2, precision, R, std::max(s, 2 * d.splits));
    }
    const bool mid = precision == 1 ? (N >= 4096) : (N >= 9216);
    return mid ? make_pair_shape(n1, n2, precision, R, 2 * d.splits) : d;
}

PairShape choose_pair_shape(int n1, int n2, int precision)
{
    int R = 0, splits = 0;
    if (lookup_tuning(n1, n2, precision, &R, &splits)) return make_pair_shape(n1, n2, precision, R, splits);
    return default_pair_shape(n1, n2, precision);
}

hipError_t launch_tune_init(const Mesh& m, double* z, double* gam, hipStream_t s)
{
    hipLaunchKernelGGL(k_tune_init, dim3(blocks_for(m.N)), dim3(kThreads), 0, s, m, z, gam);
    return hipGetLastError();
}

hipError_t launch_surface(const Mesh& m, const double* z, const double* w, double* gam, double* q,
                          int* fold, hipStream_t s)
{
    const int groups = blocks_for(m.N);
    if (m.periodic)
        hipLaunchKernelGGL(k_surface<1>, dim3(groups), dim3(kThreads), 0, s, m, z, w, gam, q, fold);
    else
        hipLaunchKernelGGL(k_surface<0>, dim3(groups), dim3(kThreads), 0, s, m, z, w, gam, q, fold);
    if (fold) hipLaunchKernelGGL(k_fold_finish, dim3(1), dim3(64), 0, s, fold);
    return hipGetLastError();
}

hipError_t launch_pairs_f64(const Mesh& m, const PairShape& sh, const double* z,
                            const double* gam, double* part, const int* fold, hipStream_t s)
{
    const dim3 grid((unsigned)(sh.px * sh.py), (unsigned)sh.splits);
    const dim3 blk(kThreads);
#define ZM_F64_CASE(RR, CC)                                                                       \
    else if (sh.R == RR && sh.cx == CC)                                                           \
        hipLaunchKernelGGL((k_pairs_f64f<RR, CC>), grid, blk, 0, s, m, sh, z, gam, part, fold);
    if (false) {}
    ZM_F64_CASE(1, 32) ZM_F64_CASE(1, 16) ZM_F64_CASE(1, 8) ZM_F64_CASE(2, 32)
    ZM_F64_CASE(2, 16) ZM_F64_CASE(2, 8) ZM_F64_CASE(4, 32) ZM_F64_CASE(4, 16)
    ZM_F64_CASE(4, 8)
    else return hipErrorInvalidConfiguration;
#undef ZM_F64_CASE
    return hipGetLastError();
}

hipError_t launch_pairs_f32(const Mesh& m, const PairShape& sh, const double* z,
                            const double* gam, double* part, const int* fold, hipStream_t s)
{
    const dim3 grid((unsigned)(sh.px * sh.py), (unsigned)sh.splits);
    const dim3 blk(kThreads);
#define ZM_F32_CASE(RR, CC)                                                                       \
    else if (sh.R == RR && sh.cx == CC)                                                           \
        hipLaunchKernelGGL((k_pairs_f32<RR, CC>), grid, blk, 0, s, m, sh, z, gam, part, fold);
    if (false) {}
    ZM_F32_CASE(1, 32) ZM_F32_CASE(1, 16) ZM_F32_CASE(1, 8) ZM_F32_CASE(2, 32)
    ZM_F32_CASE(2, 16) ZM_F32_CASE(2, 8) ZM_F32_CASE(4, 32) ZM_F32_CASE(4, 16)
    ZM_F32_CASE(4, 8)
    else return hipErrorInvalidConfiguration;
#undef ZM_F32_CASE
    return hipGetLastError();
}

hipError_t launch_ties(const Mesh& m, const double* z, const double* gam, double* tie,
                       hipStream_t s)
{
    const int blocks = dev::tie_blocks(m.n1, m.n2);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ties, dim3(blocks, 2), dim3(kThreads), 0, s, m, z, gam, tie);
    return hipGetLastError();
}

hipError_t launch_reduce(const Mesh& m, int splits, const double* part, const double* tie,
                         const double* q, const double* z, double* u, double* V, hipStream_t s,
                         bool ties)
{
    const int L = dev::reduce_lanes(m.N, splits);
    hipLaunchKernelGGL(k_reduce, dim3(blocks_for(m.N * L)), dim3(kThreads), 0, s, m, splits, part, tie,
                       q, z, u, V, ties ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_update(const Mesh& m, int stage, const double* y0_z, const double* y0_w,
                         const double* ys_z, const double* ys_w, const double* u, const double* V,
                         double* out_z, double* out_w, int* nonfinite, hipStream_t s)
{
    if (m.periodic)
        hipLaunchKernelGGL(k_update<1>, dim3(blocks_for(m.N)), dim3(kThreads), 0, s, m, stage, y0_z,
                           y0_w, ys_z, ys_w, u, V, out_z, out_w, nonfinite);
    else
        hipLaunchKernelGGL(k_update<0>, dim3(blocks_for(m.N)), dim3(kThreads), 0, s, m, stage, y0_z,
                           y0_w, ys_z, ys_w, u, V, out_z, out_w, nonfinite);
    return hipGetLastError();
}

}  // namespace zm
