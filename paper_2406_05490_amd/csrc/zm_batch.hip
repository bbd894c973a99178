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
    const dev::FoldStat st = dev::surface_point(d.m, p, ys, ys + 3 * (size_t)d.m.N, d.gam, d.q);
    // every workgroup belongs to one instance: gather over that instance's
    dev::fold_gather(st, d.fold, d.blocks);
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

// Persistent pair sweep over the items of one group (FP64 pair form, R
// targets per lane, patches PX columns wide).  Exit: a workgroup leaves once
// the counter passes nitems, which every workgroup reaches.
template <int R, int PX>
__global__ __launch_bounds__(kThreads) void kb_pairs_f64(const InstDesc* __restrict__ T,
                                                         const WorkItem* __restrict__ items,
                                                         int nitems, int* __restrict__ counter,
                                                         int stage)
{
    __shared__ dev::F64Tile lds;
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        // the same item in every lane: read it into a scalar register so the
        // item and its descriptor are scalar loads (and scalar registers)
        const int it = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const InstDesc& d = T[w.inst];
        dev::pairs_f64f_block<R, PX>(d.m, d.sh, d.Y[stage], d.gam, d.part, w.patch, w.split, d.fold,
                                     lds);
        // the body ends with a barrier, so `next` and the LDS tiles are free
    }
}

// The same over FP32-form items; up to two targets per lane it keeps four
// waves per SIMD, as the single-instance kernel does.
template <int R, int PX>
__global__ __launch_bounds__(kThreads, R <= 2 ? 4 : 1) void kb_pairs_f32(
    const InstDesc* __restrict__ T, const WorkItem* __restrict__ items, int nitems,
    int* __restrict__ counter, int stage)
{
    __shared__ dev::F32Tile tile;
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        // the same item in every lane: read it into a scalar register so the
        // item and its descriptor are scalar loads (and scalar registers)
        const int it = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (it >= nitems) break;
        const WorkItem w = items[it];
        const InstDesc& d = T[w.inst];
        dev::pairs_f32_block<R, PX>(d.m, d.sh, d.Y[stage], d.gam, d.part, w.patch, w.split, d.fold,
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
#define ZM_KB_CASE(PREC, KER, RR, CC)                                                             \
        else if (G.precision == PREC && G.R == RR && G.px == CC)                                  \
            hipLaunchKernelGGL((KER<RR, CC>), dim3(grid), blk, 0, s, b.table, items, n, ctr, stage);
        if (false) {}
        ZM_KB_CASE(0, kb_pairs_f64, 1, 32) ZM_KB_CASE(0, kb_pairs_f64, 1, 16)
        ZM_KB_CASE(0, kb_pairs_f64, 1, 8) ZM_KB_CASE(0, kb_pairs_f64, 2, 32)
        ZM_KB_CASE(0, kb_pairs_f64, 2, 16) ZM_KB_CASE(0, kb_pairs_f64, 2, 8)
        ZM_KB_CASE(0, kb_pairs_f64, 4, 32) ZM_KB_CASE(0, kb_pairs_f64, 4, 16)
        ZM_KB_CASE(0, kb_pairs_f64, 4, 8)
        ZM_KB_CASE(1, kb_pairs_f32, 1, 32) ZM_KB_CASE(1, kb_pairs_f32, 1, 16)
        ZM_KB_CASE(1, kb_pairs_f32, 1, 8) ZM_KB_CASE(1, kb_pairs_f32, 2, 32)
        ZM_KB_CASE(1, kb_pairs_f32, 2, 16) ZM_KB_CASE(1, kb_pairs_f32, 2, 8)
        ZM_KB_CASE(1, kb_pairs_f32, 4, 32) ZM_KB_CASE(1, kb_pairs_f32, 4, 16)
        ZM_KB_CASE(1, kb_pairs_f32, 4, 8)
        else return hipErrorInvalidConfiguration;
#undef ZM_KB_CASE
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
