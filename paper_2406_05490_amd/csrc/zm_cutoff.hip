// Cutoff Birkhoff-Rott solver: the desingularised BR sum restricted to the
// sources whose nearest periodic image (on a free sheet: the source itself)
// lies within a 3D distance rc of the target (the paper's cutoff-based
// approximate integral, sec. 3.2.2).  The
// paper finds neighbours with a spatial search library over a 3D spatial
// mesh; on one GPU a periodic cell grid rebuilt every evaluation does the
// same job with a handful of kernels:
//
//   k_cut_prepare   cell of every point (x, y wrapped into the period cell;
//                   z is not binned: the interface is a sheet) -> sort key
//   radix sort      stable LSD sort of (key, point) in 8-bit digits:
//                   k_sort_hist (per-workgroup digit counts), k_sort_scan
//                   (exclusive offsets, digit-major), k_sort_scatter (stable
//                   ranks from wave ballots)
//   k_cut_bounds    first / one-past-last sorted index of every cell and of
//                   every target block
//   k_cut_gather    positions, source strengths and wrap counts in sorted
//                   order, one 64-byte record per point
//   k_cut_pairs     one wave per (target block, row of neighbour cells):
//                   each neighbour cell's sources are read with wave-uniform
//                   scalar loads and every target (lane) sums over them;
//                   the image-shift arithmetic is dropped where no wrap
//                   count is involved, and a source no lane accepts skips
//                   the kernel evaluation
//
// On a periodic sheet whose horizontal map alpha -> (x, y) is one-to-one
// (the surface kernel's fold statistics: det J2 of one sign at every point)
// the binning is skipped: every source a target can accept lies within
// rc / sigma_min(J2) of it in the index torus.  On a free sheet the same
// holds with 1 - max ||J2 - I|| in place of sigma_min while that deviation
// from the index grid stays below 1/2.  Where the window fits (always on a
// free sheet), k_cut_sten walks it per target: offsets shared by all lanes,
// each lane's source read from a band of the mesh staged in LDS, so a
// target tests about its own window (1.1 - 1.2 times the pairs it accepts
// on the paper's workloads).  A larger periodic window falls back to the
// patch window (k_cut_prepare's records, k_cut_win: one 8 x 8 patch of
// targets per wave, sources read with scalar loads).  The kernels of the
// paths not taken leave at once; their launches are capped at a few
// thousand workgroups.
//
// The inclusion test is evaluated exactly as the definition writes it
// (r_a = (z_i,a - z_j,a) - S_a L_a, then r1*r1 + r2*r2 + r3*r3 < rc*rc, no
// contraction), so every include / exclude decision is the same bit for bit
// as in any other implementation of that definition.  All integer work is
// exact and every floating-point sum runs in a fixed order: results are
// bitwise reproducible.
#include "zm_device.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace zm {
namespace {

using dev::kThreads;

__host__ __device__ inline int floordiv(int a, int n) { return a >= 0 ? a / n : -((-a + n - 1) / n); }

__host__ __device__ inline int cell_key(const CutGrid& g, int cx, int cy)
{
    const int bx = cx / g.B, lx = cx - bx * g.B;
    const int by = cy / g.B, ly = cy - by * g.B;
    return ((by * g.nb1 + bx) * g.B + ly) * g.B + lx;
}

// Bound on max ||J2 - I||_2^2 (fold[9]) below which a free sheet takes the
// index window: d = ||J2 - I|| < 1/2, so its window radius rc / (1 - d) is
// at most twice the radius at d = 0.
constexpr float kFreeMaxDev2 = 0.25f;

// Whether this evaluation takes the index-window path: a sheet whose tangent
// map keeps one orientation everywhere (fold[7]: the signs det J2 took, bit 0
// positive, bit 1 negative, bit 2 zero or not a number) and, periodic, has a
// positive sigma_min(J2)^2 (fold[5]) or, free, stays within kFreeMaxDev2 of
// the identity map (fold[9]: max ||J2 - I||^2).  Every kernel of either path
// reads it and the other path's kernels leave at once.
__device__ __forceinline__ bool window_path(const int* __restrict__ fold, int periodic)
{
    if (fold == nullptr) return false;
    const int sg = fold[7];
    if (sg != 1 && sg != 2) return false;
    return periodic ? __int_as_float(fold[5]) > 0.f : __int_as_float(fold[9]) < kFreeMaxDev2;
}

// Periodic grid: wrap count k (x - k L lies in the period cell [x0, x0 + L))
// and the cell of the wrapped coordinate, clamped against rounding at the
// cell edges.  Free sheet: k = 0 and the cell of x itself, clamped to the
// box [0, nc) (in double, before the conversion, so that any x, even one far
// outside the box, gives an index in range).  Clamping never increases the
// cell distance of two points, so every pair within rc still lies within m
// cells of each other; the edge cells only get fuller once the sheet has
// rolled out of the box.
__device__ inline void wrap_cell(bool periodic, double x, double x0, double L, double cw, int nc,
                                 int& k, int& c)
{
    if (!periodic) {
        const double f = floor((x - x0) / cw);
        k = 0;
        c = (int)fmin(fmax(f, 0.0), (double)(nc - 1));
        return;
    }
    const double f = floor((x - x0) / L);
    k = (int)f;
    const double xw = x - f * L;
    c = (int)floor((xw - x0) / cw);
    c = c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// ---- stable LSD radix sort of (key, value), 8 bits per pass -----------------
// Workgroup b owns the elements [b seg, (b + 1) seg); offsets are laid out
// digit-major (digit d of every workgroup before digit d + 1), which makes the
// scatter stable.

__global__ __launch_bounds__(kThreads) void k_sort_hist(const unsigned* __restrict__ keys, int n,
                                                        int shift, int seg,
                                                        unsigned* __restrict__ hist,
                                                        const int* __restrict__ fold, int periodic)
{
    if (window_path(fold, periodic)) return;
    __shared__ unsigned h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int begin = blockIdx.x * seg;
    const int end = min(n, begin + seg);
    for (int i = begin + (int)threadIdx.x; i < end; i += kThreads)
        atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    __syncthreads();
    hist[threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of total entries in place, one workgroup of 1024 threads,
// in tiles of 8 Ki entries: a tile is loaded into LDS with coalesced reads,
// each thread scans 8 consecutive entries, the thread sums are scanned in
// LDS with the running total of the previous tiles, and the tile is written
// back coalesced.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;

__global__ __launch_bounds__(kScanThreads) void k_sort_scan(unsigned* __restrict__ a, int total,
                                                            const int* __restrict__ fold,
                                                            int periodic)
{
    if (window_path(fold, periodic)) return;
    __shared__ unsigned tile[kScanThreads * kScanPer];
    __shared__ unsigned s[kScanThreads];
    __shared__ unsigned carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    for (int base = 0; base < total; base += kScanThreads * kScanPer) {
        const int n = min(kScanThreads * kScanPer, total - base);
        for (int q = t; q < kScanThreads * kScanPer; q += kScanThreads)
            tile[q] = q < n ? a[base + q] : 0u;
        __syncthreads();
        unsigned sum = 0;
        for (int q = 0; q < kScanPer; ++q) sum += tile[t * kScanPer + q];
        s[t] = sum;
        __syncthreads();
        for (int off = 1; off < kScanThreads; off <<= 1) {
            const unsigned v = t >= off ? s[t - off] : 0u;
            __syncthreads();
            s[t] += v;
            __syncthreads();
        }
        unsigned run = carry + s[t] - sum;   // exclusive prefix of this thread's entries
        for (int q = 0; q < kScanPer; ++q) {
            const unsigned v = tile[t * kScanPer + q];
            tile[t * kScanPer + q] = run;
            run += v;
        }
        __syncthreads();
        for (int q = t; q < n; q += kScanThreads) a[base + q] = tile[q];
        if (t == kScanThreads - 1) carry += s[t];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void k_sort_scatter(const unsigned* __restrict__ kin,
                                                           const unsigned* __restrict__ vin,
                                                           unsigned* __restrict__ kout,
                                                           unsigned* __restrict__ vout, int n,
                                                           int shift, int seg,
                                                           const unsigned* __restrict__ offs,
                                                           const int* __restrict__ fold,
                                                           int periodic)
{
    if (window_path(fold, periodic)) return;
    __shared__ unsigned base[256];
    __shared__ unsigned wcnt[kThreads / 64][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    base[tid] = offs[tid * gridDim.x + blockIdx.x];
    const int begin = blockIdx.x * seg;
    const int end = min(n, begin + seg);
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int c = begin; c < end; c += kThreads) {   // uniform over the workgroup
        for (int q = 0; q < kThreads / 64; ++q) wcnt[q][tid] = 0;
        __syncthreads();
        const int i = c + tid;
        const bool valid = i < end;
        const unsigned key = valid ? kin[i] : 0u;
        const unsigned d = (key >> shift) & 255u;
        // lanes of this wave with the same digit
        unsigned long long same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long ones = __ballot(valid && bit);
            same &= bit ? ones : ~ones;
        }
        const unsigned rank = (unsigned)__popcll(same & below);
        if (valid && rank == 0) wcnt[w][d] = (unsigned)__popcll(same);
        __syncthreads();
        if (valid) {
            unsigned pos = base[d] + rank;
            for (int q = 0; q < w; ++q) pos += wcnt[q][d];
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        unsigned add = 0;
        for (int q = 0; q < kThreads / 64; ++q) add += wcnt[q][tid];
        base[tid] += add;
        __syncthreads();
    }
}

// Zero the cell and block bounds and the wrap flags of the cell path (one
// launch for the five arrays: start, end, kflag have nkeys entries, bstart
// and bend one per target block).
__global__ __launch_bounds__(kThreads) void k_cut_clear(int* __restrict__ start,
                                                        int* __restrict__ end,
                                                        int* __restrict__ kflag,
                                                        int* __restrict__ bstart,
                                                        int* __restrict__ bend, int nkeys,
                                                        int nblk, const int* __restrict__ fold,
                                                        int periodic)
{
    if (window_path(fold, periodic)) return;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < nkeys) {
        start[i] = 0;
        end[i] = 0;
        kflag[i] = 0;
    }
    if (i < nblk) {
        bstart[i] = 0;
        bend[i] = 0;
    }
}

__global__ void k_fill_u64(unsigned long long* __restrict__ a, int n)
{
    if ((int)threadIdx.x < n) a[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(kThreads) void k_cut_bounds(CutGrid g, int n,
                                                         const unsigned* __restrict__ ks,
                                                         int* __restrict__ start, int* __restrict__ end,
                                                         int* __restrict__ bstart, int* __restrict__ bend,
                                                         const int* __restrict__ fold)
{
    if (window_path(fold, g.periodic)) return;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const unsigned bb = (unsigned)(g.B * g.B);
    const unsigned key = ks[i], blk = key / bb;
    if (i == 0 || ks[i - 1] != key) start[key] = i;
    if (i == 0 || ks[i - 1] / bb != blk) bstart[blk] = i;
    if (i == n - 1 || ks[i + 1] != key) end[key] = i + 1;
    if (i == n - 1 || ks[i + 1] / bb != blk) bend[blk] = i + 1;
}

__global__ __launch_bounds__(kThreads) void k_cut_gather(Mesh m, CutGrid g, const double* __restrict__ z,
                                                         const double* __restrict__ gam,
                                                         const unsigned* __restrict__ order,
                                                         double* __restrict__ src,
                                                         int* __restrict__ kflag,
                                                         const int* __restrict__ fold)
{
    if (window_path(fold, g.periodic)) return;
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const int N = m.N;
    if (i >= N) return;
    const int p = (int)order[i];
    const double x = z[p], y = z[N + p];
    int kx, ky, cx, cy;
    wrap_cell(g.periodic, x, g.x0, g.L1, g.cw1, g.nc1, kx, cx);
    wrap_cell(g.periodic, y, g.y0, g.L2, g.cw2, g.nc2, ky, cy);
    double* r = src + (size_t)i * 8;
    r[0] = x;
    r[1] = y;
    r[2] = z[2 * N + p];
    r[3] = gam[p];
    r[4] = gam[N + p];
    r[5] = gam[2 * N + p];
    r[6] = (double)kx;
    r[7] = (double)ky;
    if (kx != 0 || ky != 0) kflag[cell_key(g, cx, cy)] = 1;   // same value from every writer
}

// One wave per (target block, neighbour row, chunk slot).  Lane = one target
// of the block: the wave takes the block's chunks of 64 targets z, z + C,
// z + 2C, ... (C = g.chunks, about the mean number of chunks per block, so
// that there are many waves even when the blocks are few); the row's B + 2m
// cells are visited left to right,
// each cell's sources in sorted order.  Every lane of the wave reads the same
// source, so a source is one 64-byte record (x, y, z, g1, g2, g3, kx, ky)
// fetched with wave-uniform (scalar) loads and used straight from scalar
// registers: no LDS, no barriers.  A source in raw cell column cx_raw
// (before wrapping) is the image shifted by wx = floor(cx_raw / nc1)
// periods, so the image shift of the pair is S = k_i + wx - k_j (and the
// same along y).  On a free sheet nothing wraps: cells outside the grid are
// skipped, every wrap count is 0 and S = 0, so r = z_i - z_j exactly (the
// wave of a row outside the grid still writes its zero partial sums).
constexpr int kCutThreads = 64;
constexpr long kCutMaxGroups = 16384;   // workgroups of a cell-path or patch-window launch at most

// Targets per lane of the pair kernel: every scalar-loaded source record
// serves 64 TR targets, each slot of 64 skipping on its own.  TR = 2, 3, 4
// cut the loads per pair but measured no faster overall (768^2, rc =
// 0.0667: 2.72, 2.46, 2.72 against 2.55 ms; 512^2, rc = 1/6: 2.94, 3.10,
// 3.07 against 2.97 ms): the kernel is bound by the per-pair VALU work of
// the accepted slots more than by its loads, and more targets per lane
// lower the occupancy (165 VGPRs at TR = 3 against 45).
#ifndef ZM_CUT_TARGETS_PER_LANE
#define ZM_CUT_TARGETS_PER_LANE 1
#endif
constexpr int kCutTargetsPerLane = ZM_CUT_TARGETS_PER_LANE;

// Image-shift handling of one (wave, neighbour cell) visit:
//   kShiftNone     every target of the wave and every source of the cell has
//                  wrap count 0 and the cell is not wrapped: S = 0, r = d
//                  (d - 0 L is d bit for bit);
//   kShiftUniform  wrap counts all 0 but the cell is wrapped: S = (wx, wy)
//                  for every pair, S_a L_a formed once;
//   kShiftPerLane  S = k_i + w - k_j per pair;
//   kShiftExact    S = the integer nearest to d / L per pair (the definition
//                  itself; d * (1 / L) in place of d / L can only change S
//                  where d / L is within rounding of a half-integer, and
//                  then both images lie about L/2 > rc away and are
//                  rejected).
// All give the same r as the definition's r_a = d_a - S_a L_a.
enum { kShiftNone = 0, kShiftUniform = 1, kShiftPerLane = 2, kShiftExact = 3 };

struct CutTarget {
    double x, y, z;     // target position
    double Kx, Ky;      // k_i + wx, k_i + wy (per-lane shift mode)
    bool active;        // lane holds a real target
    uint64_t amask;     // lanes of the wave that hold real targets
};

// One source record in scalar registers.
struct SrcRec {
    double x, y, z, g1, g2, g3, k1, k2;
};

__device__ __forceinline__ SrcRec load_rec(const double* __restrict__ src, int j)
{
    const double* s = src + (size_t)j * 8;   // the same address in every lane
    return SrcRec{s[0], s[1], s[2], s[3], s[4], s[5], s[6], s[7]};
}

// One source against the lane's TR targets: d1 = x_i - x_j is formed by the
// caller.  Slot q of the wave (64 consecutive targets of the block) skips the
// kernel evaluation of a source none of its targets accepts (a wave-uniform
// branch: the accepted set, and so every sum, is unchanged).
template <int SHIFT, bool COUNT, int TR>
__device__ __forceinline__ void cut_pair(const Mesh& m, const CutGrid& g, const CutTarget (&t)[TR],
                                         const SrcRec& b, const double (&d1)[TR], double SL1,
                                         double SL2, double (&acc)[TR][3],
                                         unsigned long long& tested, unsigned long long& accepted)
{
#pragma clang fp contract(off)
    double r1[TR], r2[TR], r3[TR], dd[TR];
    bool in[TR];
    uint64_t any[TR];
#pragma unroll
    for (int q = 0; q < TR; ++q) {
        const double d2 = t[q].y - b.y;
        if (SHIFT == kShiftNone) {
            r1[q] = d1[q];
            r2[q] = d2;
        } else if (SHIFT == kShiftUniform) {
            r1[q] = d1[q] - SL1;
            r2[q] = d2 - SL2;
        } else if (SHIFT == kShiftExact) {
            const double S1 = rint(d1[q] * g.iL1), S2 = rint(d2 * g.iL2);
            r1[q] = d1[q] - S1 * g.L1;
            r2[q] = d2 - S2 * g.L2;
        } else {
            const double S1 = t[q].Kx - b.k1, S2 = t[q].Ky - b.k2;
            r1[q] = d1[q] - S1 * g.L1;
            r2[q] = d2 - S2 * g.L2;
        }
        r3[q] = t[q].z - b.z;
        dd[q] = r1[q] * r1[q] + r2[q] * r2[q] + r3[q] * r3[q];
        in[q] = dd[q] < g.rc2;
        any[q] = __builtin_amdgcn_ballot_w64(in[q]) & t[q].amask;
        if (COUNT) {   // whole-wave counts (scalar work, the same in every lane)
            tested += (unsigned long long)__popcll(t[q].amask);
            accepted += (unsigned long long)__popcll(any[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < TR; ++q) {
        if (any[q] == 0ull) continue;
        const double wgt = in[q] ? dev::inv_cube_sqrt(dd[q] + m.eps2) : 0.0;
        const double a1 = wgt * b.g1, a2 = wgt * b.g2, a3 = wgt * b.g3;
        acc[q][0] = fma(r2[q], a3, acc[q][0]);
        acc[q][0] = fma(-r3[q], a2, acc[q][0]);
        acc[q][1] = fma(r3[q], a1, acc[q][1]);
        acc[q][1] = fma(-r1[q], a3, acc[q][1]);
        acc[q][2] = fma(r1[q], a2, acc[q][2]);
        acc[q][2] = fma(-r2[q], a1, acc[q][2]);
    }
}

// Sum the sources [s0, s1) of one cell into the lane's accumulators, two at
// a time.  Scalar loads may return out of order, so a wait is always a wait
// for every load in flight: the next pair is issued only after the current
// pair has arrived (its first use sits before a scheduling barrier), which
// leaves a whole pair of evaluations to hide the next pair's latency.
template <int SHIFT, bool COUNT, int TR>
__device__ __forceinline__ void cut_cell(const Mesh& m, const CutGrid& g,
                                         const double* __restrict__ src, int s0, int s1,
                                         const CutTarget (&t)[TR], double SL1, double SL2,
                                         double (&acc)[TR][3], unsigned long long& tested,
                                         unsigned long long& accepted)
{
    if (s0 >= s1) return;
    const int last = s1 - 1;
    SrcRec p0 = load_rec(src, s0), p1 = load_rec(src, s0 + 1 < s1 ? s0 + 1 : last);
    for (int j = s0; j < s1; j += 2) {
#pragma clang fp contract(off)
        const SrcRec c0 = p0, c1 = p1;
        double d1a[TR], d1b[TR];
#pragma unroll
        for (int q = 0; q < TR; ++q) {
            d1a[q] = t[q].x - c0.x;   // the pair has arrived
            d1b[q] = t[q].x - c1.x;
        }
        __builtin_amdgcn_sched_barrier(0);
        p0 = load_rec(src, j + 2 < s1 ? j + 2 : last);
        p1 = load_rec(src, j + 3 < s1 ? j + 3 : last);
        __builtin_amdgcn_sched_barrier(0);
        cut_pair<SHIFT, COUNT, TR>(m, g, t, c0, d1a, SL1, SL2, acc, tested, accepted);
        if (j + 1 < s1) cut_pair<SHIFT, COUNT, TR>(m, g, t, c1, d1b, SL1, SL2, acc, tested, accepted);
    }
}

// Chunks of 64 TR targets: slot q of a chunk holds targets t0 + lane + 64 q.
template <bool COUNT, int TR>
__global__ __launch_bounds__(kCutThreads) void k_cut_pairs(Mesh m, CutGrid g,
                                                           const double* __restrict__ src,
                                                           const int* __restrict__ start,
                                                           const int* __restrict__ end,
                                                           const int* __restrict__ bstart,
                                                           const int* __restrict__ bend,
                                                           const int* __restrict__ kflag,
                                                           const unsigned* __restrict__ order,
                                                           double* __restrict__ part,
                                                           unsigned long long* __restrict__ counts,
                                                           const int* __restrict__ fold)
{
    if (window_path(fold, g.periodic)) return;   // uniform: the index-window path runs instead
    constexpr int CH = kCutThreads * TR;
    // Grid order as launched (block fastest), so that the 8 XCDs, which
    // take workgroups round robin, share every region of the mesh.  Giving
    // each XCD a contiguous range of blocks instead (neighbouring blocks read
    // mostly the same cells) measured 7% slower at 768^2 and 15% at 512^2.
    const int N = m.N;
    const int lane = threadIdx.x;
    // the reduction sums partial sums [0, planes); this path writes
    // [0, slots) below and zeroes the rest here
    {
        const long nz = (long)(g.planes - g.slots) * 3 * N;
        double* pz = part + (long)g.slots * 3 * N;
        for (long i = (long)blockIdx.x * kCutThreads + lane; i < nz; i += (long)gridDim.x * kCutThreads)
            pz[i] = 0.0;
    }
    const int nblk = g.nb1 * g.nb2;
    const long items = (long)nblk * g.slots * g.chunks;
    unsigned long long tested = 0, accepted = 0;
    // items (block, row, chunk), block fastest, strided over a capped grid
    for (long it = blockIdx.x; it < items; it += gridDim.x) {
        const int blk = (int)(it % nblk), row = (int)(it / nblk % g.slots);
        const int zc = (int)(it / ((long)nblk * g.slots));
        const int T0 = bstart[blk], T1 = bend[blk];
        if (T0 + zc * CH >= T1) continue;   // nothing left: uniform
        const int bx = blk % g.nb1, by = blk / g.nb1;
        const int cy_raw = by * g.B - g.m + row;
        const int wy = floordiv(cy_raw, g.nc2), cy = cy_raw - wy * g.nc2;
        const bool row_in = g.periodic || wy == 0;

        // chunks zc, zc + chunks, ...
        for (int t0 = T0 + zc * CH; t0 < T1; t0 += g.chunks * CH) {
            CutTarget t[TR];
            double kxi[TR], kyi[TR];
            bool any_k = false;
#pragma unroll
            for (int q = 0; q < TR; ++q) {
                const int i = t0 + lane + kCutThreads * q;
                t[q].active = i < T1;
                t[q].amask = __builtin_amdgcn_ballot_w64(t[q].active);
                const double* ti = src + (size_t)(t[q].active ? i : T0) * 8;
                t[q].x = ti[0];
                t[q].y = ti[1];
                t[q].z = ti[2];
                kxi[q] = ti[6];
                kyi[q] = ti[7];
                any_k = any_k || kxi[q] != 0.0 || kyi[q] != 0.0;
            }
            // every target of the wave unwrapped (inactive slots hold a real target of the block)
            const bool targets_k0 = __builtin_amdgcn_ballot_w64(any_k) == 0ull;
            double acc[TR][3];
#pragma unroll
            for (int q = 0; q < TR; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
            for (int col = 0; col < g.slots; ++col) {
                const int cx_raw = bx * g.B - g.m + col;
                const int wx = floordiv(cx_raw, g.nc1), cx = cx_raw - wx * g.nc1;
                if (!row_in || (!g.periodic && wx != 0)) continue;   // wave-uniform
                const int key = cell_key(g, cx, cy);
                const int s0 = start[key], s1 = end[key];
                if (targets_k0 && kflag[key] == 0) {
                    if (wx == 0 && wy == 0) {
                        cut_cell<kShiftNone, COUNT, TR>(m, g, src, s0, s1, t, 0.0, 0.0, acc, tested,
                                                        accepted);
                    } else {
                        const double SL1 = (double)wx * g.L1, SL2 = (double)wy * g.L2;
                        cut_cell<kShiftUniform, COUNT, TR>(m, g, src, s0, s1, t, SL1, SL2, acc, tested,
                                                           accepted);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < TR; ++q) {
                        t[q].Kx = kxi[q] + (double)wx;
                        t[q].Ky = kyi[q] + (double)wy;
                    }
                    cut_cell<kShiftPerLane, COUNT, TR>(m, g, src, s0, s1, t, 0.0, 0.0, acc, tested,
                                                       accepted);
                }
            }
            double* out = part + (size_t)row * 3 * N;
#pragma unroll
            for (int q = 0; q < TR; ++q) {
                if (t[q].active) {
                    const int p = (int)order[t0 + lane + kCutThreads * q];
                    out[p] = acc[q][0];
                    out[N + p] = acc[q][1];
                    out[2 * N + p] = acc[q][2];
                }
            }
        }
    }
    if (COUNT) {
        if (lane == 0) {
            atomicAdd(&counts[0], tested);
            atomicAdd(&counts[1], accepted);
            atomicOr(&counts[2], kCutPathCells);
        }
    }
}

// ---- index-window path ----------------------------------------------------

constexpr int kStThreads = 256;
constexpr int kXcds = 8;                               // XCDs the workgroups are dealt over
constexpr int kStBlk = 4;                              // tiles per side of a block of the work order
constexpr int kCUs = 256;                              // compute units of the device
constexpr int kMaxPlanes = 16;                         // partial sums per target at most
constexpr int kStTX = 32, kStTY = 16;                  // target tile (columns, rows)
constexpr int kStBh = 8, kStBw = 16;                   // offsets per band (rows, columns)
constexpr int kStRows = kStTY + kStBh - 1;             // staged source rows
constexpr int kStCols = kStTX - 2 + kStBw;             // staged source columns
constexpr int kStHalf = kStCols / 2;                   // entries per parity and row
constexpr int kStPad = kStHalf + 1;
constexpr int kStPer = (kStRows * kStCols + kStThreads - 1) / kStThreads;   // staged per lane
constexpr int kStPairsX = kStTX / 2;                  // lanes per target row (two targets each)
static_assert(kStPairsX * kStTY == kStThreads && kStTX % 2 == 0, "lane layout");
static_assert(kStBw % 2 == 0, "a band starts both parities");

// Index window of one evaluation (the same in every workgroup): alpha radius
// Ra (squared), row and column reach W2, W1 in spacings, and whether the
// seam counts give the image shifts.  A source whose nearest image lies
// within rc of a target is less than Ra = rc / sigma_min from it in alpha
// (sigma_min = min sigma_min(J2) over the sheet, fold[5]; plus a margin of 2%
// and one spacing for the discrete tangents).  Along the window the sources
// of one period copy (unwrapped column ju1 = j1 + w1 n1, row ju2 = j2 + w2 n2)
// have image shift S = (w1, w2) whenever sigma_max(J2) (fold[9]) times the
// largest alpha offset between a target and a window source stays below
// 0.45 min(L1, L2): the horizontal part of z_i - z_j - w L, the only part the
// shift depends on, is at most that long, so the nearest integer to d_a / L_a
// is w_a.
struct WinGeom {
    double Ra2;
    int W1, W2;
    bool by_seams;
};

__device__ inline WinGeom win_geom(const Mesh& m, const CutGrid& g, const int* __restrict__ fold)
{
    WinGeom w;
    // the least ratio of horizontal distance to index distance: sigma_min(J2)
    // on a periodic sheet, 1 - max ||J2 - I|| on a free one
    const double hdev = sqrt((double)__int_as_float(fold[9]));
    const double smin = g.periodic ? sqrt((double)__int_as_float(fold[5])) : 1.0 - hdev;
    const double Ra = sqrt(g.rc2) * 1.02 / smin;
    w.Ra2 = Ra * Ra;
    w.W2 = (int)ceil(Ra / m.h2) + 1;
    w.W1 = (int)ceil(Ra / m.h1) + 1;
    if (!g.periodic) {
        // no source of a free sheet lies farther than its side in index
        w.W1 = min(w.W1, m.n1);
        w.W2 = min(w.W2, m.n2);
        w.by_seams = true;   // no images: every shift is 0
        return w;
    }
    const double dmax = sqrt((double)(w.W1 + 8) * (w.W1 + 8) * m.h1 * m.h1 +
                             (double)(w.W2 + 8) * (w.W2 + 8) * m.h2 * m.h2);
    w.by_seams = hdev * dmax < 0.45 * fmin(g.L1, g.L2);
    return w;
}

// Columns either side of a target that the window takes in the row dy
// spacings away (the chord of the radius-Ra disc, plus one spacing).
__device__ inline int win_chord(const Mesh& m, const WinGeom& w, int dy)
{
    const double ry = (double)dy * m.h2;
    const double half = w.Ra2 > ry * ry ? sqrt(w.Ra2 - ry * ry) : 0.0;
    return (int)ceil(half / m.h1) + 1;
}

// Whether the per-target stencil (k_cut_sten) takes the evaluation: on a
// periodic sheet the seam counts give the shifts and no target's window holds
// a source twice (its 2 W1 + 2 columns and 2 W2 + 1 rows fit the period);
// a free sheet has neither images nor wraps, and always fits.  Otherwise the
// patch-window kernel (k_cut_win) does.
__device__ inline bool sten_fits(const Mesh& m, const WinGeom& w)
{
    if (!m.periodic) return true;
    return w.by_seams && 2 * w.W1 + 2 <= m.n1 && 2 * w.W2 + 1 <= m.n2 && m.n1 >= kStCols &&
           m.n2 >= kStRows;
}

// First pass over the points, per path: the cell path's sort keys (cell
// of every point, x and y wrapped into the period cell; z is not binned:
// the interface is a sheet) and point indices; the patch window's records
// (x, y, z, g1, g2, g3, 0, 0) in index order; nothing for the stencil, which
// reads the planes.
__global__ __launch_bounds__(kThreads) void k_cut_prepare(Mesh m, CutGrid g,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ gam,
                                                          unsigned* __restrict__ keys,
                                                          unsigned* __restrict__ vals,
                                                          double* __restrict__ src,
                                                          const int* __restrict__ fold)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    const int N = m.N;
    if (!window_path(fold, g.periodic)) {
        if (p >= N) return;
        int kx, ky, cx, cy;
        wrap_cell(g.periodic, z[p], g.x0, g.L1, g.cw1, g.nc1, kx, cx);
        wrap_cell(g.periodic, z[N + p], g.y0, g.L2, g.cw2, g.nc2, ky, cy);
        keys[p] = (unsigned)cell_key(g, cx, cy);
        vals[p] = (unsigned)p;
        return;
    }
    if (sten_fits(m, win_geom(m, g, fold))) return;
    if (p >= N) return;
    double* r = src + (size_t)p * 8;
    r[0] = z[p];
    r[1] = z[N + p];
    r[2] = z[2 * N + p];
    r[3] = gam[p];
    r[4] = gam[N + p];
    r[5] = gam[2 * N + p];
    r[6] = 0.0;
    r[7] = 0.0;
}

// Patch window, for windows too large for the stencil: one wave per (8 x 8
// patch of targets, row group).  Lane = one target (t1, t2) = (c0 + lane % 8,
// r0 + lane / 8); the window is every source whose alpha distance to the
// patch's rectangle is at most Ra, rows of it split over the slots, each
// source read once for all 64 lanes.  Without the seam-count rule S is
// formed per pair from its definition; a window wider than the period takes
// every column (row) once.
template <bool COUNT>
__global__ __launch_bounds__(kCutThreads) void k_cut_win(Mesh m, CutGrid g,
                                                         const double* __restrict__ src,
                                                         double* __restrict__ part,
                                                         unsigned long long* __restrict__ counts,
                                                         const int* __restrict__ fold)
{
    if (!window_path(fold, g.periodic)) return;   // uniform: the cell path runs instead
    const WinGeom wg = win_geom(m, g, fold);
    if (sten_fits(m, wg)) return;                 // uniform: the stencil runs instead
    const int n1 = m.n1, n2 = m.n2, N = m.N;
    const int lane = threadIdx.x;
    const int pc = (n1 + 7) / 8, npatch = pc * ((n2 + 7) / 8);
    const long items = (long)npatch * g.planes;
    unsigned long long tested = 0, accepted = 0;
    // items (patch, slot), patch fastest, strided over a capped grid
    for (long it = blockIdx.x; it < items; it += gridDim.x) {
        const int patch = (int)(it % npatch), slot = (int)(it / npatch);
        const int c0 = (patch % pc) * 8, r0 = (patch / pc) * 8;
        const int t1 = c0 + (lane & 7), t2 = r0 + (lane >> 3);

        CutTarget t[1];
        t[0].active = t1 < n1 && t2 < n2;
        t[0].amask = __builtin_amdgcn_ballot_w64(t[0].active);
        const int p = t[0].active ? t2 * n1 + t1 : r0 * n1 + c0;   // idle lanes hold a real target
        const double* tr = src + (size_t)p * 8;
        t[0].x = tr[0];
        t[0].y = tr[1];
        t[0].z = tr[2];
        t[0].Kx = t[0].Ky = 0.0;

        const int W2 = wg.W2;
        const bool by_seams = wg.by_seams;
        int rlo = r0 - W2, nrows = 8 + 2 * W2;
        // a window taller than the period takes every row once; a row's
        // distance from the patch is then its distance in the torus
        const bool all_rows = nrows >= n2;
        if (all_rows) nrows = n2;
        const int per = (nrows + g.planes - 1) / g.planes;
        const int ra = rlo + slot * per, rb = min(rlo + nrows, ra + per);
        const double Ra2 = wg.Ra2;
        auto row_gap = [&](int ju) { return ju < r0 ? r0 - ju : (ju > r0 + 7 ? ju - (r0 + 7) : 0); };

        double acc[1][3] = {{0.0, 0.0, 0.0}};
        for (int ju2 = ra; ju2 < rb; ++ju2) {
            const int w2 = floordiv(ju2, n2), j2 = ju2 - w2 * n2;
            int dy = row_gap(ju2);
            if (all_rows) dy = min(dy, min(row_gap(ju2 + n2), row_gap(ju2 - n2)));
            const double ry = dy * m.h2;
            const double half = Ra2 > ry * ry ? sqrt(Ra2 - ry * ry) : 0.0;
            const int dxm = (int)ceil(half / m.h1) + 1;
            int clo = c0 - dxm, ncols = 8 + 2 * dxm;
            if (ncols > n1) ncols = n1;               // every column once
            // the row's columns [clo, clo + ncols) in pieces of one period copy
            int a = clo;
            const int e = clo + ncols;
            while (a < e) {
                const int w1 = floordiv(a, n1);
                const int b = min(e, (w1 + 1) * n1);
                const int s0 = j2 * n1 + (a - w1 * n1), s1 = s0 + (b - a);
                if (!by_seams)
                    cut_cell<kShiftExact, COUNT, 1>(m, g, src, s0, s1, t, 0.0, 0.0, acc, tested,
                                                    accepted);
                else if (w1 == 0 && w2 == 0)
                    cut_cell<kShiftNone, COUNT, 1>(m, g, src, s0, s1, t, 0.0, 0.0, acc, tested,
                                                   accepted);
                else
                    cut_cell<kShiftUniform, COUNT, 1>(m, g, src, s0, s1, t, (double)w1 * g.L1,
                                                      (double)w2 * g.L2, acc, tested, accepted);
                a = b;
            }
        }
        if (t[0].active) {
            double* out = part + (size_t)slot * 3 * N;
            out[p] = acc[0][0];
            out[N + p] = acc[0][1];
            out[2 * N + p] = acc[0][2];
        }
    }
    if (COUNT) {
        if (lane == 0) {
            atomicAdd(&counts[0], tested);
            atomicAdd(&counts[1], accepted);
            atomicOr(&counts[2], kCutPathWindow);
        }
    }
}

// Per-target stencil: a workgroup of 256 lanes takes a 32 x 16 tile of
// targets, two horizontally adjacent targets per lane ((C0 + 2a + k, R0 + b),
// a = lane % 16, b = lane / 16, k = 0, 1), and walks offsets (dy, sx) that
// are the same in every lane: the lane's source is the point at (C0 + 2a +
// sx, R0 + b + dy), its first target's offset is (sx, dy), its second's
// (sx - 1, dy).  Offsets run over every row |dy| <= W2 and, in row dy, the
// columns -chord(dy) .. chord(dy) + 1, so each target meets every source of
// its own window and no other: the tests per target are about the disc of
// radius Ra rather than its union over a patch.  The sources of a band of
// kStBh x kStBw offsets are staged in LDS (the band's 23 rows x 46 columns,
// split by column parity so that consecutive lanes read consecutive
// entries); bands no row of the disc reaches are skipped and the others are
// dealt round-robin to the slots.  Every source is one period copy away from
// its wrapped index (w1, w2 in -1 .. 1), which is its image shift; bands that
// cross no seam skip the shift arithmetic (S = 0, r = d bit for bit).
// Two doubles as one native vector (staged records stay in registers; the
// HIP vector wrapper type keeps them in private memory when copied through
// an array).
typedef double dv2 __attribute__((ext_vector_type(2)));

struct StTile {
    dv2 xy[2][kStRows][kStPad];
    dv2 zg[2][kStRows][kStPad];   // (z, g1)
    dv2 gg[2][kStRows][kStPad];   // (g2, g3)
    int chord[kStBh];             // win_chord of the band's rows dy0 .. dy0 + kStBh - 1
};

// Stencil workgroups resident per CU (bounded by the 160 KiB of LDS).
constexpr long kStGroupsPerCU = (160L * 1024) / (long)sizeof(StTile);
static_assert(kStGroupsPerCU >= 1, "a staged band must fit the LDS");

// Coordinate of a free sheet's off-mesh sources in a staged band: far enough
// that no pair with a mesh point is accepted, small enough that the squared
// distance stays finite.
constexpr double kStFar = 1e150;

// One source against the lane's two targets (cut_pair's sums): a source that
// no lane accepts for either target is skipped; otherwise both targets take
// the kernel weight through the accept select in one block (the two
// reciprocal square roots overlap), an unaccepted pair adding exact zeros.
template <bool SEAM, bool COUNT>
__device__ __forceinline__ void sten_pair(const Mesh& m, const CutGrid& g, const CutTarget (&t)[2],
                                          const SrcRec& b, const double (&d1)[2], double SL1,
                                          double SL2, double (&acc)[2][3],
                                          unsigned long long& tested, unsigned long long& accepted)
{
#pragma clang fp contract(off)
    double r1[2], r2[2], r3[2], dd[2];
    bool in[2];
    uint64_t any[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double d2 = t[q].y - b.y;
        r1[q] = SEAM ? d1[q] - SL1 : d1[q];
        r2[q] = SEAM ? d2 - SL2 : d2;
        r3[q] = t[q].z - b.z;
        dd[q] = r1[q] * r1[q] + r2[q] * r2[q] + r3[q] * r3[q];
        in[q] = dd[q] < g.rc2;
        any[q] = __builtin_amdgcn_ballot_w64(in[q]) & t[q].amask;
        // whole-wave count (scalar work); the tested pairs are counted per row
        if (COUNT) accepted += (unsigned long long)__popcll(any[q]);
    }
    if ((any[0] | any[1]) == 0ull) return;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        double wgt = dev::inv_cube_sqrt(dd[q] + m.eps2);
        wgt = in[q] ? wgt : 0.0;
        const double a1 = wgt * b.g1, a2 = wgt * b.g2, a3 = wgt * b.g3;
        acc[q][0] = fma(r2[q], a3, acc[q][0]);
        acc[q][0] = fma(-r3[q], a2, acc[q][0]);
        acc[q][1] = fma(r3[q], a1, acc[q][1]);
        acc[q][1] = fma(-r1[q], a3, acc[q][1]);
        acc[q][2] = fma(r1[q], a2, acc[q][2]);
        acc[q][2] = fma(-r2[q], a1, acc[q][2]);
    }
}

template <bool SEAM, bool COUNT>
__device__ __forceinline__ void sten_band(const Mesh& m, const CutGrid& g, const WinGeom& wg,
                                          const StTile& T, int C0, int R0, int a, int b, int dy0,
                                          int dx0, const CutTarget (&t)[2], double (&acc)[2][3],
                                          unsigned long long& tested, unsigned long long& accepted)
{
    const int dyhi = min(dy0 + kStBh, wg.W2 + 1);
    for (int dy = dy0; dy < dyhi; ++dy) {
        // the same value in every lane (staged with the band)
        const int dm = __builtin_amdgcn_readfirstlane(T.chord[dy - dy0]);
        const int slo = max(dx0, -dm), shi = min(dx0 + kStBw, dm + 2);
        if (slo >= shi) continue;
        // every step of the row tests each active target once
        if (COUNT)
            tested += (unsigned long long)(shi - slo) *
                      (unsigned long long)(__popcll(t[0].amask) + __popcll(t[1].amask));
        const int rr = b + dy - dy0;
        // an active target's source lies less than one period outside the
        // mesh, so its wrap count is -1, 0 or 1 and S L is -L, 0 or L exactly
        // (idle lanes' shifts are never used)
        double SL2 = 0.0;
        if (SEAM) {
            const int r = R0 + b + dy;
            SL2 = r < 0 ? -g.L2 : (r >= m.n2 ? g.L2 : 0.0);
        }
        // offset o = sx - dx0 reads entry a + o / 2 of parity plane o & 1.
        // In runs of four steps each step's source is read before the step
        // ahead of it evaluates, so the LDS latency overlaps arithmetic.
        struct Rec { dv2 xy, zg, gg; };
        auto fetch = [&](int par, int hc) {
            return Rec{T.xy[par][rr][hc], T.zg[par][rr][hc], T.gg[par][rr][hc]};
        };
        auto step = [&](int sx, const Rec& r) {
#pragma clang fp contract(off)
            const SrcRec rec{r.xy.x, r.xy.y, r.zg.x, r.zg.y, r.gg.x, r.gg.y, 0.0, 0.0};
            double SL1 = 0.0;
            if (SEAM) {
                const int c = C0 + 2 * a + sx;
                SL1 = c < 0 ? -g.L1 : (c >= m.n1 ? g.L1 : 0.0);
            }
            double d1[2];
            d1[0] = t[0].x - rec.x;
            d1[1] = t[1].x - rec.x;
            sten_pair<SEAM, COUNT>(m, g, t, rec, d1, SL1, SL2, acc, tested, accepted);
        };
        int sx = slo;
        if ((sx - dx0) & 1) {
            step(sx, fetch(1, a + ((sx - dx0) >> 1)));
            ++sx;
        }
        for (; sx + 3 < shi; sx += 4) {   // two entries of each parity
            const int hc = a + ((sx - dx0) >> 1);
            const Rec r0 = fetch(0, hc);
            const Rec r1 = fetch(1, hc);
            step(sx, r0);
            const Rec r2 = fetch(0, hc + 1);
            step(sx + 1, r1);
            const Rec r3 = fetch(1, hc + 1);
            step(sx + 2, r2);
            step(sx + 3, r3);
        }
        for (; sx + 1 < shi; sx += 2) {
            const int hc = a + ((sx - dx0) >> 1);
            const Rec r0 = fetch(0, hc);
            const Rec r1 = fetch(1, hc);
            step(sx, r0);
            step(sx + 1, r1);
        }
        if (sx < shi) step(sx, fetch(0, a + ((sx - dx0) >> 1)));
    }
}

// PER: the boundary kind the launch was chosen for (1 periodic, 0 free), so
// that each instance stages one kind of band.
template <bool COUNT, bool PER>
__global__ __launch_bounds__(kStThreads) void k_cut_sten(Mesh m, CutGrid g,
                                                         const double* __restrict__ z,
                                                         const double* __restrict__ gam,
                                                         double* __restrict__ part,
                                                         unsigned long long* __restrict__ counts,
                                                         const int* __restrict__ fold)
{
    if (!window_path(fold, g.periodic)) return;   // uniform: the cell path runs instead
    const WinGeom wg = win_geom(m, g, fold);
    if (!sten_fits(m, wg)) return;                // uniform: the patch window runs instead
    __shared__ StTile T;
    const int n1 = m.n1, n2 = m.n2, N = m.N;
    constexpr bool periodic = PER;
    const int tiles1 = (n1 + kStTX - 1) / kStTX;
    // workgroups are dealt round-robin to the XCDs: give each XCD one
    // contiguous run of (tile, slot) items so that the windows of the tiles it
    // works on at one time overlap in its L2; items run over blocks of
    // kStBlk x kStBlk tiles, the tiles of a block, then the slots
    const int tiles2 = (n2 + kStTY - 1) / kStTY;
    const int blocks1 = (tiles1 + kStBlk - 1) / kStBlk;
    const int total = (int)gridDim.x;
    const int L = (int)blockIdx.x;
    const int xcd = L % kXcds, per = total / kXcds, rem = total % kXcds;
    const int item = xcd * per + min(xcd, rem) + L / kXcds;
    const int slot = item % g.planes, bt = item / g.planes;
    const int blk = bt / (kStBlk * kStBlk), in = bt - blk * (kStBlk * kStBlk);
    const int tx = (blk % blocks1) * kStBlk + in % kStBlk, ty = (blk / blocks1) * kStBlk + in / kStBlk;
    if (tx >= tiles1 || ty >= tiles2) return;     // the ragged edge of the block grid
    const int C0 = tx * kStTX, R0 = ty * kStTY;
    const int tid = threadIdx.x, a = tid % kStPairsX, b = tid / kStPairsX;

    CutTarget t[2];
    int tp[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int c = C0 + 2 * a + k, r = R0 + b;
        t[k].active = c < n1 && r < n2;
        t[k].amask = __builtin_amdgcn_ballot_w64(t[k].active);
        tp[k] = t[k].active ? r * n1 + c : 0;   // idle lanes hold a real target
        t[k].x = z[tp[k]];
        t[k].y = z[N + tp[k]];
        t[k].z = z[2 * N + tp[k]];
        t[k].Kx = t[k].Ky = 0.0;
    }

    unsigned long long tested = 0, accepted = 0;
    double acc[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    int band = 0;
    for (int dy0 = -wg.W2; dy0 <= wg.W2; dy0 += kStBh) {
        // the band's row nearest dy = 0 has the longest chord
        const int dyn = dy0 > 0 ? dy0 : min(dy0 + kStBh - 1, 0);
        const int dm = win_chord(m, wg, dyn);
        for (int dx0 = -wg.W1; dx0 <= wg.W1 + 1; dx0 += kStBw) {
            if (max(dx0, -dm) >= min(dx0 + kStBw, dm + 2)) continue;   // outside the disc
            // a free sheet's bands whose sources all lie off the mesh
            if (!periodic && (R0 + dy0 + kStRows <= 0 || R0 + dy0 >= n2 ||
                              C0 + dx0 + kStCols <= 0 || C0 + dx0 >= n1))
                continue;
            if (band++ % g.planes != slot) continue;
            // stage the band's sources: every load is issued before the
            // first LDS write (one round trip per band).  Periodic: the
            // band's first row and column are wrapped once, the rest by
            // subtraction.  Free: a source off the mesh is staged as a point
            // kStFar away with zero strength, which no target accepts (its
            // squared distance stays finite, its weight is selected away and
            // its terms add exact zeros)
            int rb = R0 + dy0, cb = C0 + dx0;
            if (periodic) {
                rb -= floordiv(rb, n2) * n2;
                cb -= floordiv(cb, n1) * n1;
            }
            dv2 v[kStPer][3];
#pragma unroll
            for (int i = 0; i < kStPer; ++i) {
                const int e = tid + i * kStThreads;
                const int ee = e < kStRows * kStCols ? e : 0;
                const int rr = ee / kStCols, cr = ee - rr * kStCols;
                int r = rb + rr, c = cb + cr;
                bool on = true;
                if (periodic) {
                    r = r >= n2 ? r - n2 : r;   // one period at most: n2 >= kStRows, n1 >= kStCols
                    c = c >= n1 ? c - n1 : c;
                } else {
                    on = r >= 0 && r < n2 && c >= 0 && c < n1;
                }
                const int j = on ? r * n1 + c : 0;
                v[i][0] = on ? dv2{z[j], z[N + j]} : dv2{kStFar, kStFar};
                v[i][1] = on ? dv2{z[2 * N + j], gam[j]} : dv2{kStFar, 0.0};
                v[i][2] = on ? dv2{gam[N + j], gam[2 * N + j]} : dv2{0.0, 0.0};
            }
            __syncthreads();   // the previous band's reads are done
#pragma unroll
            for (int i = 0; i < kStPer; ++i) {
                const int e = tid + i * kStThreads;
                if (e < kStRows * kStCols) {
                    const int rr = e / kStCols, cr = e - rr * kStCols;
                    const int par = cr & 1, hc = cr >> 1;
                    T.xy[par][rr][hc] = v[i][0];
                    T.zg[par][rr][hc] = v[i][1];
                    T.gg[par][rr][hc] = v[i][2];
                }
            }
            // the rows' chords (a square root and a division each), once per
            // band instead of once per row in every wave
            if (tid < kStBh) T.chord[tid] = win_chord(m, wg, dy0 + tid);
            __syncthreads();
            const bool seam = periodic && (C0 + dx0 < 0 || C0 + dx0 + kStCols > n1 ||
                                           R0 + dy0 < 0 || R0 + dy0 + kStRows > n2);
            if (seam)
                sten_band<true, COUNT>(m, g, wg, T, C0, R0, a, b, dy0, dx0, t, acc, tested,
                                       accepted);
            else
                sten_band<false, COUNT>(m, g, wg, T, C0, R0, a, b, dy0, dx0, t, acc, tested,
                                        accepted);
        }
    }
    double* out = part + (size_t)slot * 3 * N;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (!t[k].active) continue;
        out[tp[k]] = acc[k][0];
        out[N + tp[k]] = acc[k][1];
        out[2 * N + tp[k]] = acc[k][2];
    }
    if (COUNT) {
        if ((tid & 63) == 0) {
            atomicAdd(&counts[0], tested);
            atomicAdd(&counts[1], accepted);
            atomicOr(&counts[2], kCutPathStencil);
        }
    }
}

inline unsigned grid_for(long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

CutGrid make_cut_grid(int n1, int n2, double L1, double L2, double rc, bool periodic)
{
    CutGrid g;
    g.m = 2;
    g.periodic = periodic ? 1 : 0;
    g.pad_ = 0;
    // cells no smaller than rc / m (with a margin against rounding at the
    // cell edges) and no smaller than the mean mesh spacing
    const double grow = 1.0 + 1e-9;
    g.nc1 = std::max(1, std::min(n1, (int)std::floor(g.m * L1 / (rc * grow))));
    g.nc2 = std::max(1, std::min(n2, (int)std::floor(g.m * L2 / (rc * grow))));
    g.cw1 = L1 / g.nc1;
    g.cw2 = L2 / g.nc2;
    // target blocks of B x B cells hold >= ~128 points on average
    const double per_cell = (double)n1 * n2 / ((double)g.nc1 * g.nc2);
    g.B = std::max(1, (int)std::ceil(std::sqrt(128.0 / per_cell)));
    g.B = std::min(g.B, std::min(g.nc1, g.nc2));
    g.nb1 = (g.nc1 + g.B - 1) / g.B;
    g.nb2 = (g.nc2 + g.B - 1) / g.B;
    g.nkeys = g.nb1 * g.nb2 * g.B * g.B;
    g.key_bits = 1;
    while ((1L << g.key_bits) < (long)g.nkeys) ++g.key_bits;
    g.slots = g.B + 2 * g.m;
    // the index-window kernels split each target's sources over more
    // partial sums when the mesh has few stencil tiles, so that a launch
    // holds about eight rounds of resident workgroups (three per CU)
    const long tiles = (long)((n1 + kStTX - 1) / kStTX) * ((n2 + kStTY - 1) / kStTY);
    const long want = (8L * kStGroupsPerCU * kCUs + tiles - 1) / tiles;
    g.planes = (int)std::max<long>(g.slots, std::min<long>(want, kMaxPlanes));
    const long N = (long)n1 * n2;
    const long per_block = (N + (long)g.nb1 * g.nb2 - 1) / ((long)g.nb1 * g.nb2);
    g.tr = kCutTargetsPerLane;
    g.chunks = (int)std::max(1L, std::min(65535L, (per_block + 64L * g.tr - 1) / (64L * g.tr)));
    g.sort_blocks = (int)std::max(1L, std::min(1024L, (N + 1023) / 1024));
    g.x0 = -0.5 * L1;
    g.y0 = -0.5 * L2;
    g.L1 = L1;
    g.L2 = L2;
    g.rc2 = rc * rc;
    g.iL1 = 1.0 / L1;
    g.iL2 = 1.0 / L2;
    return g;
}

hipError_t launch_cut_cells(const Mesh& m, const CutGrid& g, const double* z, const double* gam,
                            const CutBuffers& b, const int* fold, int* sorted_half, hipStream_t s)
{
    const int N = m.N;
    const dim3 blk(kThreads);
    const int per = g.periodic;
    hipLaunchKernelGGL(k_cut_prepare, dim3(grid_for(N)), blk, 0, s, m, g, z, gam, b.keys[0],
                       b.vals[0], b.src, fold);
    const int G = g.sort_blocks;
    const int seg = ((N + G - 1) / G + kThreads - 1) / kThreads * kThreads;
    int cur = 0;
    for (int shift = 0; shift < g.key_bits; shift += 8) {
        hipLaunchKernelGGL(k_sort_hist, dim3(G), blk, 0, s, b.keys[cur], N, shift, seg, b.hist, fold,
                           per);
        hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(kScanThreads), 0, s, b.hist, 256 * G, fold, per);
        hipLaunchKernelGGL(k_sort_scatter, dim3(G), blk, 0, s, b.keys[cur], b.vals[cur],
                           b.keys[cur ^ 1], b.vals[cur ^ 1], N, shift, seg, b.hist, fold, per);
        cur ^= 1;
    }
    const int nblk = g.nb1 * g.nb2;
    hipLaunchKernelGGL(k_cut_clear, dim3(grid_for(std::max(g.nkeys, nblk))), blk, 0, s, b.start,
                       b.end, b.kflag, b.bstart, b.bend, g.nkeys, nblk, fold, per);
    hipLaunchKernelGGL(k_cut_bounds, dim3(grid_for(N)), blk, 0, s, g, N, b.keys[cur], b.start,
                       b.end, b.bstart, b.bend, fold);
    hipLaunchKernelGGL(k_cut_gather, dim3(grid_for(N)), blk, 0, s, m, g, z, gam, b.vals[cur], b.src,
                       b.kflag, fold);
    *sorted_half = cur;
    return hipGetLastError();
}

hipError_t launch_cut_pairs(const Mesh& m, const CutGrid& g, const double* z, const double* gam,
                            const CutBuffers& b, int sorted_half, double* part, bool count,
                            const int* fold, hipStream_t s)
{
    // capped grids: the kernels of the path not taken launch few workgroups
    const long cell_items = (long)g.nb1 * g.nb2 * g.slots * g.chunks;
    const dim3 grid((unsigned)std::min<long>(cell_items, kCutMaxGroups));
    const unsigned* order = b.vals[sorted_half];
    if (count)
        hipLaunchKernelGGL((k_cut_pairs<true, kCutTargetsPerLane>), grid, dim3(kCutThreads), 0, s, m,
                           g, b.src, b.start, b.end, b.bstart, b.bend, b.kflag, order, part,
                           b.counts, fold);
    else
        hipLaunchKernelGGL((k_cut_pairs<false, kCutTargetsPerLane>), grid, dim3(kCutThreads), 0, s,
                           m, g, b.src, b.start, b.end, b.bstart, b.bend, b.kflag, order, part,
                           b.counts, fold);
    // the index-window path: patch window or per-target stencil (the
    // workgroups of the kernels not taking the evaluation leave at once)
    const long win_items = (long)((m.n1 + 7) / 8) * ((m.n2 + 7) / 8) * g.planes;
    const dim3 wgrid((unsigned)std::min<long>(win_items, kCutMaxGroups));
    if (count)
        hipLaunchKernelGGL((k_cut_win<true>), wgrid, dim3(kCutThreads), 0, s, m, g, b.src, part,
                           b.counts, fold);
    else
        hipLaunchKernelGGL((k_cut_win<false>), wgrid, dim3(kCutThreads), 0, s, m, g, b.src, part,
                           b.counts, fold);
    const int bl1 = ((m.n1 + kStTX - 1) / kStTX + kStBlk - 1) / kStBlk;
    const int bl2 = ((m.n2 + kStTY - 1) / kStTY + kStBlk - 1) / kStBlk;
    const dim3 sgrid((unsigned)(bl1 * bl2 * kStBlk * kStBlk * g.planes));
#define ZM_STEN_LAUNCH(C, P)                                                                      \
    hipLaunchKernelGGL((k_cut_sten<C, P>), sgrid, dim3(kStThreads), 0, s, m, g, z, gam, part,     \
                       b.counts, fold)
    if (m.periodic) {
        if (count) ZM_STEN_LAUNCH(true, true);
        else ZM_STEN_LAUNCH(false, true);
    } else {
        if (count) ZM_STEN_LAUNCH(true, false);
        else ZM_STEN_LAUNCH(false, false);
    }
#undef ZM_STEN_LAUNCH
    return hipGetLastError();
}

hipError_t launch_cut_count_reset(unsigned long long* counts, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, counts, kCutCountWords);
    return hipGetLastError();
}

}  // namespace zm
