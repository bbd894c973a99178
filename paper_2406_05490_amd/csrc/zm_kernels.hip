// Single-instance kernels: thin wrappers that map the launch grid onto the
// device bodies in zm_device.h, plus the launch-shape choice and launchers.
#include "zm_device.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

namespace zm {
namespace {

using dev::kThreads;

__global__ __launch_bounds__(kThreads) void k_surface(Mesh m, const double* __restrict__ z,
                                                      const double* __restrict__ w,
                                                      double* __restrict__ gam,
                                                      double* __restrict__ q)
{
    dev::surface_point(m, blockIdx.x * kThreads + threadIdx.x, z, w, gam, q);
}

template <int R, int CX>
__global__ __launch_bounds__(kThreads) void k_pairs_f64(Mesh m, PairShape sh,
                                                        const double* __restrict__ z,
                                                        const double* __restrict__ gam,
                                                        double* __restrict__ part)
{
    __shared__ double2 lds[2][3][kThreads];
    dev::pairs_f64_block<R, CX>(m, sh, z, gam, part, blockIdx.x, blockIdx.y, lds);
}

template <int R, int PX>
__global__ __launch_bounds__(kThreads) void k_pairs_f32(Mesh m, PairShape sh,
                                                        const double* __restrict__ z,
                                                        const double* __restrict__ gam,
                                                        double* __restrict__ part)
{
    __shared__ float4 lds0[2][kThreads];
    __shared__ float2 lds1[2][kThreads];
    dev::pairs_f32_block<R, PX>(m, sh, z, gam, part, blockIdx.x, blockIdx.y, lds0, lds1);
}

// blockIdx.y = pass (0: tie column, 1: tie row)
__global__ __launch_bounds__(kThreads) void k_ties(Mesh m, const double* __restrict__ z,
                                                   const double* __restrict__ gam,
                                                   double* __restrict__ tie)
{
    dev::ties_point(m, blockIdx.x * kThreads + threadIdx.x, blockIdx.y, z, gam, tie);
}

__global__ __launch_bounds__(kThreads) void k_reduce(Mesh m, int splits,
                                                     const double* __restrict__ part,
                                                     const double* __restrict__ tie,
                                                     const double* __restrict__ q,
                                                     const double* __restrict__ z,
                                                     double* __restrict__ u,
                                                     double* __restrict__ V)
{
    dev::reduce_point(m, blockIdx.x * kThreads + threadIdx.x, splits, part, tie, q, z, u, V);
}

// y0 may alias out (see update_point), so neither carries __restrict__.
__global__ __launch_bounds__(kThreads) void k_update(Mesh m, int stage, const double* y0_z,
                                                     const double* y0_w,
                                                     const double* __restrict__ ys_z,
                                                     const double* __restrict__ ys_w,
                                                     const double* __restrict__ u,
                                                     const double* __restrict__ V,
                                                     double* out_z, double* out_w,
                                                     int* __restrict__ nonfinite)
{
    dev::update_point(m, blockIdx.x * kThreads + threadIdx.x, stage, y0_z, y0_w, ys_z, ys_w, u,
                      V, out_z, out_w, nonfinite);
}

inline unsigned blocks_for(int n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace


// ---------------------------------------------------------------------------
// launch shapes and launchers
// ---------------------------------------------------------------------------

PairShape choose_pair_shape(int n1, int n2, int precision)
{
    PairShape sh;
    if (precision == 1) {
        // FP32 pairs: compact patches keep tile-relative coordinates small
        sh.R = ZM_PAIR32_R;
        sh.cx = (n1 >= 32) ? 32 : (n1 >= 16 ? 16 : 8);
    } else {
        sh.R = ZM_PAIR_R;
        sh.cx = (n1 >= 16) ? 16 : 8;
    }
    sh.prow = (kThreads / sh.cx) * sh.R;
    sh.px = (n1 + sh.cx - 1) / sh.cx;
    sh.py = (n2 + sh.prow - 1) / sh.prow;
    const int patches = sh.px * sh.py;
    // Aim for >= 2048 workgroups (8 per CU on 256 CUs) by splitting the
    // source rows; every split keeps at least one row.
    int splits = (2048 + patches - 1) / patches;
    if (splits > n2) splits = n2;
    if (splits < 1) splits = 1;
    sh.rows_per_split = (n2 + splits - 1) / splits;
    sh.splits = (n2 + sh.rows_per_split - 1) / sh.rows_per_split;
    return sh;
}

hipError_t launch_surface(const Mesh& m, const double* z, const double* w, double* gam, double* q,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_surface, dim3(blocks_for(m.N)), dim3(kThreads), 0, s, m, z, w, gam, q);
    return hipGetLastError();
}

hipError_t launch_pairs_f64(const Mesh& m, const PairShape& sh, const double* z,
                            const double* gam, double* part, hipStream_t s)
{
    const dim3 grid((unsigned)(sh.px * sh.py), (unsigned)sh.splits);
    constexpr int R = ZM_PAIR_R;
    if (sh.R == R && sh.cx == 16)
        hipLaunchKernelGGL((k_pairs_f64<R, 16>), grid, dim3(kThreads), 0, s, m, sh, z, gam, part);
    else if (sh.R == R && sh.cx == 8)
        hipLaunchKernelGGL((k_pairs_f64<R, 8>), grid, dim3(kThreads), 0, s, m, sh, z, gam, part);
    else
        return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

hipError_t launch_pairs_f32(const Mesh& m, const PairShape& sh, const double* z,
                            const double* gam, double* part, hipStream_t s)
{
    const dim3 grid((unsigned)(sh.px * sh.py), (unsigned)sh.splits);
    constexpr int R = ZM_PAIR32_R;
    if (sh.R == R && sh.cx == 32)
        hipLaunchKernelGGL((k_pairs_f32<R, 32>), grid, dim3(kThreads), 0, s, m, sh, z, gam, part);
    else if (sh.R == R && sh.cx == 16)
        hipLaunchKernelGGL((k_pairs_f32<R, 16>), grid, dim3(kThreads), 0, s, m, sh, z, gam, part);
    else if (sh.R == R && sh.cx == 8)
        hipLaunchKernelGGL((k_pairs_f32<R, 8>), grid, dim3(kThreads), 0, s, m, sh, z, gam, part);
    else
        return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

hipError_t launch_ties(const Mesh& m, const double* z, const double* gam, double* tie,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_ties, dim3(blocks_for(m.N), 2), dim3(kThreads), 0, s, m, z, gam, tie);
    return hipGetLastError();
}

hipError_t launch_reduce(const Mesh& m, int splits, const double* part, const double* tie,
                         const double* q, const double* z, double* u, double* V, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(blocks_for(m.N)), dim3(kThreads), 0, s, m, splits, part, tie,
                       q, z, u, V);
    return hipGetLastError();
}

hipError_t launch_update(const Mesh& m, int stage, const double* y0_z, const double* y0_w,
                         const double* ys_z, const double* ys_w, const double* u, const double* V,
                         double* out_z, double* out_w, int* nonfinite, hipStream_t s)
{
    hipLaunchKernelGGL(k_update, dim3(blocks_for(m.N)), dim3(kThreads), 0, s, m, stage, y0_z, y0_w,
                       ys_z, ys_w, u, V, out_z, out_w, nonfinite);
    return hipGetLastError();
}

}  // namespace zm
