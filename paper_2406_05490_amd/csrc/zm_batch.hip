// Batched kernels: many independent Z-Model instances advanced by one set of
// launches per RK3 stage.
//
// Every instance has a device descriptor (mesh, pair-kernel shape, buffer
// pointers).  Point-wise kernels run over the concatenated block ranges of
// all instances; a block finds its instance by binary search over the block
// offsets.  The pair sweep is one persistent launch per precision: each
// workgroup repeatedly takes the next (instance, target patch, source split)
// item from a device work list sorted longest first and runs the same body
// as the single-instance kernel, so every instance's arithmetic is identical
// alone and in a batch.
#include "zm_batch_internal.h"
#include "zm_device.h"

#include <hip/hip_runtime.h>

namespace zm {
namespace {

using dev::kThreads;

// Instance owning global block b: largest i with block_begin <= b.
__device__ __forceinline__ int find_instance(const InstDesc* __restrict__ T, int count, int b)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T[mid].block_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The same search over the tie kernel's block offsets.
__device__ __forceinline__ int find_tie_instance(const InstDesc* __restrict__ T, int count, int b)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T[mid].tie_block_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void kb_surface(const InstDesc* __restrict__ T, int count,
                                                       int stage)
{
    const int i = find_instance(T, count, blockIdx.x);
    const InstDesc& d = T[i];
    const int p = (blockIdx.x - d.block_begin) * kThreads + threadIdx.x;
    const double* ys = d.Y[stage];
    dev::surface_point(d.m, p, ys, ys + 3 * (size_t)d.m.N, d.gam, d.q);
}

__global__ __launch_bounds__(kThreads) void kb_ties(const InstDesc* __restrict__ T, int count,
                                                    int stage)
{
    __shared__ double2 lds[3][kThreads];
    const int i = find_tie_instance(T, count, blockIdx.x);
    const InstDesc& d = T[i];
    // blocks past this instance's own tie shape leave at once (uniformly)
    const int b = blockIdx.x - d.tie_block_begin;
    if (blockIdx.y == 0) dev::ties_block<0>(d.m, b, d.Y[stage], d.gam, d.tie, lds);
    else dev::ties_block<1>(d.m, b, d.Y[stage], d.gam, d.tie, lds);
}

// The same search over the reduction's block offsets.
__device__ __forceinline__ int find_reduce_instance(const InstDesc* __restrict__ T, int count, int b)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (T[mid].reduce_block_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void kb_reduce(const InstDesc* __restrict__ T, int count,
                                                      int stage)
{
    const int i = find_reduce_instance(T, count, blockIdx.x);
    const InstDesc& d = T[i];
    const int t = (blockIdx.x - d.reduce_block_begin) * kThreads + threadIdx.x;
    // one instance per block, so the lane count is uniform over the block
    dev::reduce_thread(d.m, t, dev::reduce_lanes(d.m.N, d.sh.splits), d.sh.splits, d.part, d.tie,
                       d.q, d.Y[stage], d.u, d.V, true);
}

__global__ __launch_bounds__(kThreads) void kb_update(const InstDesc* __restrict__ T, int count,
                                                      int stage)
{
    const int i = find_instance(T, count, blockIdx.x);
    const InstDesc& d = T[i];
    const int p = (blockIdx.x - d.block_begin) * kThreads + threadIdx.x;
    const size_t N = d.m.N;
    const double* ys = d.Y[stage];
    double* out = d.Y[(stage + 1) % 3];
    const double* y0 = d.Y[0];
    dev::update_point(d.m, p, stage, y0, y0 + 3 * N, ys, ys + 3 * N, d.u, d.V, out, out + 3 * N,
                      d.flag);
}

// Resets the work counter of a persistent launch (a kernel, not a memset, so
// it can sit inside a captured graph).
__global__ void kb_reset(int* __restrict__ counter)
{
    if (threadIdx.x == 0) counter[0] = 0;
}

// Persistent pair sweep over the FP64 items.  Exit: a workgroup leaves once
// the counter passes nitems, which every workgroup reaches.
template <int R>
__global__ __launch_bounds__(kThreads) void kb_pairs_f64(const InstDesc* __restrict__ T,
                                                         const WorkItem* __restrict__ items,
                                                         int nitems, int* __restrict__ counter,
                                                         int stage)
{
    __shared__ double2 lds[2][5][kThreads];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const InstDesc& d = T[w.inst];
        if (d.sh.cx == 32)
            dev::pairs_f64f_block<R, 32>(d.m, d.sh, d.Y[stage], d.gam, d.part, w.patch, w.split, lds);
        else if (d.sh.cx == 16)
            dev::pairs_f64f_block<R, 16>(d.m, d.sh, d.Y[stage], d.gam, d.part, w.patch, w.split, lds);
        else
            dev::pairs_f64f_block<R, 8>(d.m, d.sh, d.Y[stage], d.gam, d.part, w.patch, w.split, lds);
        // the body ends with a barrier, so `next` and the LDS tiles are free
    }
}

template <int R>
__global__ __launch_bounds__(kThreads) void kb_pairs_f32(const InstDesc* __restrict__ T,
                                                         const WorkItem* __restrict__ items,
                                                         int nitems, int* __restrict__ counter,
                                                         int stage)
{
    __shared__ dev::F32Tile tile;
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const InstDesc& d = T[w.inst];
        if (d.sh.cx == 32)
            dev::pairs_f32_block<R, 32>(d.m, d.sh, d.Y[stage], d.gam, d.part, w.patch, w.split,
                                        tile);
        else if (d.sh.cx == 16)
            dev::pairs_f32_block<R, 16>(d.m, d.sh, d.Y[stage], d.gam, d.part, w.patch, w.split,
                                        tile);
        else
            dev::pairs_f32_block<R, 8>(d.m, d.sh, d.Y[stage], d.gam, d.part, w.patch, w.split,
                                       tile);
    }
}

}  // namespace

int dev_tie_blocks(int n1, int n2) { return dev::tie_blocks(n1, n2); }
int dev_reduce_lanes(int N, int splits) { return dev::reduce_lanes(N, splits); }

hipError_t launch_batch_pairs(const BatchLaunch& b, int stage, hipStream_t s)
{
    const dim3 blk(kThreads);
    for (int g = 0; g < b.ngroups; ++g) {
        const PairGroup& G = b.groups[g];
        if (G.nitems == 0) continue;
        hipLaunchKernelGGL(kb_reset, dim3(1), dim3(64), 0, s, b.counters + g);
        const unsigned grid = (unsigned)(G.nitems < b.persistent_groups ? G.nitems
                                                                         : b.persistent_groups);
        const WorkItem* items = b.items + G.item_begin;
        int* ctr = b.counters + g;
        const int n = G.nitems;
        if (G.precision == 0) {
            if (G.R == 1) hipLaunchKernelGGL((kb_pairs_f64<1>), dim3(grid), blk, 0, s, b.table, items, n, ctr, stage);
            else if (G.R == 2) hipLaunchKernelGGL((kb_pairs_f64<2>), dim3(grid), blk, 0, s, b.table, items, n, ctr, stage);
            else hipLaunchKernelGGL((kb_pairs_f64<4>), dim3(grid), blk, 0, s, b.table, items, n, ctr, stage);
        } else {
            if (G.R == 1) hipLaunchKernelGGL((kb_pairs_f32<1>), dim3(grid), blk, 0, s, b.table, items, n, ctr, stage);
            else if (G.R == 2) hipLaunchKernelGGL((kb_pairs_f32<2>), dim3(grid), blk, 0, s, b.table, items, n, ctr, stage);
            else hipLaunchKernelGGL((kb_pairs_f32<4>), dim3(grid), blk, 0, s, b.table, items, n, ctr, stage);
        }
    }
    return hipGetLastError();
}

hipError_t launch_batch_stage(const BatchLaunch& b, int stage, hipStream_t s)
{
    if (b.count <= 0) return hipSuccess;
    const dim3 blk(kThreads);
    hipLaunchKernelGGL(kb_surface, dim3(b.total_blocks), blk, 0, s, b.table, b.count, stage);
    hipError_t e = launch_batch_pairs(b, stage, s);
    if (e != hipSuccess) return e;
    if (b.any_even)
        hipLaunchKernelGGL(kb_ties, dim3(b.total_tie_blocks, 2), blk, 0, s, b.table, b.count, stage);
    hipLaunchKernelGGL(kb_reduce, dim3(b.total_reduce_blocks), blk, 0, s, b.table, b.count, stage);
    hipLaunchKernelGGL(kb_update, dim3(b.total_blocks), blk, 0, s, b.table, b.count, stage);
    return hipGetLastError();
}

}  // namespace zm
