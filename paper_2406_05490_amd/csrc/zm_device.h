// Device-side bodies of the Z-Model kernels, shared by the single-instance
// kernels (zm_kernels.hip) and the batched ones (zm_batch.hip) so that an
// instance computes exactly the same arithmetic alone and in a batch.
//
// Data layout: structure-of-arrays float64 planes in HBM, point index
// p = i2 * n1 + i1.  Workgroups are 256 threads (four 64-wide waves).
//
//   surface_point     tangents T_a (5-point, periodic, seam-corrected), source
//                     strength gamma = w1 T2 - w2 T1, q = |gamma|^2/|T1 x T2|^2.
//   pairs_f64f_block  one (target patch, source row range) of the all-pairs
//                     Birkhoff-Rott sweep in FP64: sources staged 256 at a
//                     time through LDS (coalesced plane loads, double
//                     buffered) as patch-relative coordinates, read back as
//                     wave-wide broadcasts; factored pair arithmetic on the
//                     VALU; per-target sums blocked per row segment.
//   pairs_f32_block   the same in FP32 pair arithmetic (direct form) with
//                     FP64 per-target sums.
//   ties_block        split-tie correction for even n_a (tie line staged in LDS).
//   reduce_group      fixed-order sum over source splits and tie passes,
//                     scale, Bernoulli potential V.
//   update_point      D V (+ nu Lap w) and the SSP-RK3 stage combination.
#pragma once

#include "zm_internal.h"

#include <hip/hip_runtime.h>

namespace zm {
namespace dev {

constexpr int kThreads = 256;

// Source-loop unroll depth and targets per lane of the pair kernel.
#ifndef ZM_PAIR_UNROLL
#define ZM_PAIR_UNROLL 2
#endif


// Periodic neighbour index along one axis; sets wrap to -1/0/+1.
__device__ __forceinline__ int nbr(int i, int d, int n, int& wrap)
{
    int j = i + d;
    wrap = 0;
    if (j < 0) { j += n; wrap = -1; }
    else if (j >= n) { j -= n; wrap = 1; }
    return j;
}

// Value of a line g(0..n-1) (g[k * stride]) at j in [-2, n+1]; outside the
// line (free boundary) the ghost value of a cubic extrapolation from the four
// nearest points: g(-1) = 4 g0 - 6 g1 + 4 g2 - g3,
// g(-2) = 10 g0 - 20 g1 + 15 g2 - 4 g3, and the mirror images at the far end.
__device__ __forceinline__ double line_at(const double* __restrict__ g, size_t stride, int n, int j)
{
    if (j >= 0 && j < n) return g[(size_t)j * stride];
    const bool lo = j < 0;
    const size_t s = stride;
    const double g0 = lo ? g[0] : g[(size_t)(n - 1) * s];
    const double g1 = lo ? g[s] : g[(size_t)(n - 2) * s];
    const double g2 = lo ? g[2 * s] : g[(size_t)(n - 3) * s];
    const double g3 = lo ? g[3 * s] : g[(size_t)(n - 4) * s];
    const bool first = (j == -1) || (j == n);
    return first ? 4.0 * g0 - 6.0 * g1 + 4.0 * g2 - g3
                 : 10.0 * g0 - 20.0 * g1 + 15.0 * g2 - 4.0 * g3;
}

// The four 5-point neighbours (offsets -2, -1, +1, +2) of index i on the line
// g (g[k * stride], n points).  Periodic: wrapped, plus `shift` per wrap (the
// seam correction of the matching coordinate, 0 otherwise).  Free:
// extrapolated ghosts.
__device__ __forceinline__ void stencil4(bool periodic, const double* __restrict__ g, size_t stride,
                                         int n, int i, double shift, double v[4])
{
    const int offs[4] = {-2, -1, 1, 2};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (periodic) {
            int w;
            const int j = nbr(i, offs[k], n, w);
            v[k] = g[(size_t)j * stride];
            if (w != 0) v[k] = v[k] + (double)w * shift;
        } else {
            v[k] = line_at(g, stride, n, i + offs[k]);
        }
    }
}

__device__ __forceinline__ double d1_5pt(double fm2, double fm1, double fp1, double fp2, double h)
{
    return (8.0 * (fp1 - fm1) - (fp2 - fm2)) / (12.0 * h);
}

__device__ __forceinline__ double d2_5pt(double fm2, double fm1, double f0, double fp1, double fp2,
                                         double h)
{
    return (-fp2 + 16.0 * fp1 - 30.0 * f0 + 16.0 * fm1 - fm2) / (12.0 * h * h);
}

// w = (|r|^2 + eps^2)^(-3/2) from s = |r|^2 + eps^2.  The hardware reciprocal
// square root y0 = s^(-1/2) (1 + d) had |d| <= 2^-24 in a probe over every
// binade on gfx950 (a measurement; no bound is documented).  With
// e = 1 - s y0^2 = -(2d + d^2), |e| <= 2^-23, the exact value is
// y0^3 (1 - e)^(-3/2) = y0^3 (1 + 3e/2 + 15e^2/8 + ...), so the first-order
// correction w = y0^3 (1 + 3e/2) is low by 15 e^2 / 8 <= 2.7e-14 relative
// (plus a few ulp of rounding), a one-signed bias per pair.
__device__ __forceinline__ double inv_cube_sqrt(double s)
{
    const double y0 = __builtin_amdgcn_rsq(s);
    const double y2 = y0 * y0;
    const double e = fma(-s, y2, 1.0);
    const double w0 = y2 * y0;
    return fma(w0 * e, 1.5, w0);
}

// ---------------------------------------------------------------------------
// surface derivatives
// ---------------------------------------------------------------------------

// Boundary kind of a stencil: PER = 1 periodic, 0 free, -1 read from the
// mesh at run time (both stencils compiled in).
template <int PER>
__device__ __forceinline__ bool periodic_of(const Mesh& m)
{
    return PER < 0 ? m.periodic != 0 : PER != 0;
}

// Tangents T1 = D1 z, T2 = D2 z at point p (5-point; seam-corrected on a
// periodic sheet, extrapolated ghosts on a free one).
template <int PER = -1>
__device__ __forceinline__ void tangents_at(const Mesh& m, int p, const double* __restrict__ z,
                                            double T1[3], double T2[3])
{
    const int N = m.N;
    const int i2 = p / m.n1;
    const int i1 = p - i2 * m.n1;
    const bool per = periodic_of<PER>(m);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* f = z + (size_t)c * N;
        double a[4], b[4];
        stencil4(per, f + (size_t)i2 * m.n1, 1, m.n1, i1, c == 0 ? m.L1 : 0.0, a);
        stencil4(per, f + i1, (size_t)m.n1, m.n2, i2, c == 1 ? m.L2 : 0.0, b);
        T1[c] = d1_5pt(a[0], a[1], a[2], a[3], m.h1);
        T2[c] = d1_5pt(b[0], b[1], b[2], b[3], m.h2);
    }
}

// ---- fold statistics of the sheet -------------------------------------------
//
// The pair kernels' far forms expand |r|^2 + eps^2 as |a|^2 + (|b|^2 + eps^2 -
// 2 a.b), whose rounding is about ((|a| + |b|) / |r|)^2 ulp, and pick the
// sources that take it by their index distance from the target patch: every
// source at least one patch half-extent e beyond the patch.  That bounds the
// ratio only while index distance bounds physical distance.  With the
// tangent map J3 = (T1, T2) and its horizontal part J2 (the x, y rows):
// while det J2 keeps one sign (and is not 0) at every point the horizontal
// map alpha -> (x, y) is a covering of the period cell of degree +-1, i.e.
// one-to-one, so
// the horizontal distance of two points is at least sigma_min(J2) times their
// index distance (the straight horizontal segment between them pulls back
// to a path at least that long); and a target lies within sigma_max(J3) e of
// the patch centre.  So |r| >= sigma_min e, |a| <= sigma_max e and
// (|a| + |b|) / |r| <= 1 + 2 sigma_max / sigma_min: with sigma_max <= 4
// sigma_min everywhere the far forms stay within 81 ulp.  A sheet that
// folds (det J2 changes sign or vanishes: overturned, rolled up) or stretches beyond
// that ratio takes exact r for every pair instead (the same sums with more
// operations per pair).  The surface kernel gathers min sigma_min(J2)^2,
// max sigma_max(J3)^2, max sigma_max(J2)^2 and the signs det J2 takes over
// the mesh; a one-thread kernel after it (for a batch: the instance's last
// workgroup) turns them into the flag the pair kernels read and clears the
// gathered values for the next evaluation.
//
// fold[0]: max of (bits(+inf) - bits(min sigma_min^2)) (0 = nothing seen)
// fold[1]: max of bits(max sigma_max^2)
// fold[2]: signs of det J2 seen (bits as in fold_stat)
// fold[3]: workgroups done (batched surface kernel only)
// fold[4]: 1 = the far forms are off for this evaluation (read by the pair kernels)
// fold[5], fold[6], fold[7]: this evaluation's min sigma_min(J2)^2 and max
//          sigma_max(J3)^2 (float bits) and det J2 signs, kept after the
//          gathered values are cleared (the cutoff solver's index windows read
//          fold[5] and fold[7])
// fold[8]: max of bits(max hdev), where hdev is sigma_max(J2)^2 on a periodic
//          sheet and ||J2 - I||_2^2 on a free one
// fold[9]: this evaluation's max hdev (float bits), kept for the cutoff
//          solver: its image-shift rule (periodic) or its index-window bound
//          (free sheet: on the convex index rectangle, ||J2 - I|| <= d at
//          every point gives |x(a) - x(b)| >= (1 - d) |a - b| for the
//          horizontal map, by integrating J2 along the straight segment)
// (kFoldWords = 10 ints in all, zm_internal.h)
constexpr float kFoldMaxStretch2 = 16.f;   // (sigma_max / sigma_min)^2 allowed

struct FoldStat {
    float smin2, smax2;   // sigma_min(J2)^2, sigma_max(J3)^2
    float hmax2;          // periodic: sigma_max(J2)^2; free: ||J2 - I||_2^2
    int folded;
};

// Called by every thread of a workgroup (256 threads): the workgroup's
// points' statistics are combined and added to fold[0], [1], [2] and [8] with
// atomics, each only where it would change the word (within an evaluation
// the words only grow, so a value read here is a lower bound of the final
// one).
__device__ __forceinline__ void fold_accumulate(FoldStat st, int* __restrict__ fold)
{
    __shared__ float smin_w[kThreads / 64], smax_w[kThreads / 64], hmax_w[kThreads / 64];
    __shared__ int fold_w[kThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        st.smin2 = fminf(st.smin2, __shfl_xor(st.smin2, off, 64));
        st.smax2 = fmaxf(st.smax2, __shfl_xor(st.smax2, off, 64));
        st.hmax2 = fmaxf(st.hmax2, __shfl_xor(st.hmax2, off, 64));
        st.folded |= __shfl_xor(st.folded, off, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        smin_w[wv] = st.smin2;
        smax_w[wv] = st.smax2;
        hmax_w[wv] = st.hmax2;
        fold_w[wv] = st.folded;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    float a = smin_w[0], b = smax_w[0], c = hmax_w[0];
    int f = fold_w[0];
#pragma unroll
    for (int k = 1; k < kThreads / 64; ++k) {
        a = fminf(a, smin_w[k]);
        b = fmaxf(b, smax_w[k]);
        c = fmaxf(c, hmax_w[k]);
        f |= fold_w[k];
    }
    const int inf_bits = __float_as_int(__builtin_inff());
    auto peek = [&](int i) { return __hip_atomic_load(&fold[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); };
    const int v0 = inf_bits - __float_as_int(a), v1 = __float_as_int(b), v8 = __float_as_int(c);
    if (v0 > peek(0)) atomicMax(&fold[0], v0);   // a, b, c >= 0: bit order = value order
    if (v1 > peek(1)) atomicMax(&fold[1], v1);
    if (v8 > peek(8)) atomicMax(&fold[8], v8);
    if (f & ~peek(2)) atomicOr(&fold[2], f);
}

// One thread, once every workgroup has added its values: the flag the pair
// kernels read, this evaluation's values, and the gathered words cleared for
// the next evaluation.
__device__ __forceinline__ void fold_finish(int* __restrict__ fold)
{
    const int inf_bits = __float_as_int(__builtin_inff());
    const float smin2 = __int_as_float(inf_bits - atomicAdd(&fold[0], 0));
    const float smax2 = __int_as_float(atomicAdd(&fold[1], 0));
    const float hmax2 = __int_as_float(atomicAdd(&fold[8], 0));
    const int sg = atomicAdd(&fold[2], 0);
    const bool off = (sg & 3) == 3 || (sg & 4) != 0 || !(smax2 <= kFoldMaxStretch2 * smin2);
    atomicExch(&fold[4], off ? 1 : 0);
    atomicExch(&fold[5], __float_as_int(smin2));
    atomicExch(&fold[6], __float_as_int(smax2));
    atomicExch(&fold[7], sg);
    atomicExch(&fold[9], __float_as_int(hmax2));
    atomicExch(&fold[0], 0);
    atomicExch(&fold[1], 0);
    atomicExch(&fold[2], 0);
    atomicExch(&fold[3], 0);
    atomicExch(&fold[8], 0);
}

// fold_accumulate and fold_finish in one launch (the batched surface
// kernel, whose instances each own a range of its workgroups): the last
// workgroup of an instance (of `groups` in all), counted in fold[3] after a
// fence, finishes it.
__device__ __forceinline__ void fold_gather(FoldStat st, int* __restrict__ fold, int groups)
{
    fold_accumulate(st, fold);
    if (threadIdx.x != 0) return;
    __threadfence();
    if (atomicAdd(&fold[3], 1) != groups - 1) return;
    // last workgroup: every other one has added its values (fenced above)
    fold_finish(fold);
}

__device__ __forceinline__ FoldStat fold_merge(FoldStat a, FoldStat b)
{
    return FoldStat{fminf(a.smin2, b.smin2), fmaxf(a.smax2, b.smax2), fmaxf(a.hmax2, b.hmax2),
                    a.folded | b.folded};
}

// Tangent-map statistics of one point (identity values for p >= N).
// folded: bit 0 det J2 > 0, bit 1 det J2 < 0, bit 2 neither (0 or NaN).
__device__ __forceinline__ FoldStat fold_stat(const double T1[3], const double T2[3], double det2,
                                              bool periodic)
{
    const float x1 = (float)T1[0], y1 = (float)T1[1], z1 = (float)T1[2];
    const float x2 = (float)T2[0], y2 = (float)T2[1], z2 = (float)T2[2];
    const float det = (float)det2;
    const float s2 = x1 * x1 + x2 * x2 + y1 * y1 + y2 * y2;
    const float s3 = s2 + z1 * z1 + z2 * z2;
    const float n1 = y1 * z2 - z1 * y2, n2 = z1 * x2 - x1 * z2;
    const float nn = n1 * n1 + n2 * n2 + det * det;   // |T1 x T2|^2
    FoldStat st;
    st.smin2 = 0.5f * (s2 - __builtin_amdgcn_sqrtf(fmaxf(s2 * s2 - 4.f * det * det, 0.f)));
    st.smax2 = 0.5f * (s3 + __builtin_amdgcn_sqrtf(fmaxf(s3 * s3 - 4.f * nn, 0.f)));
    if (periodic) {
        st.hmax2 = 0.5f * (s2 + __builtin_amdgcn_sqrtf(fmaxf(s2 * s2 - 4.f * det * det, 0.f)));
    } else {
        // J2 - I = [[x1 - 1, x2], [y1, y2 - 1]]: its largest singular value squared
        const float a11 = x1 - 1.f, a22 = y2 - 1.f;
        const float f = a11 * a11 + x2 * x2 + y1 * y1 + a22 * a22;
        const float da = a11 * a22 - x2 * y1;
        st.hmax2 = 0.5f * (f + __builtin_amdgcn_sqrtf(fmaxf(f * f - 4.f * da * da, 0.f)));
    }
    st.folded = det2 > 0.0 ? 1 : (det2 < 0.0 ? 2 : 4);
    return st;
}

template <int PER = -1>
__device__ __forceinline__ FoldStat surface_point(const Mesh& m, int p, const double* __restrict__ z,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ gam, double* __restrict__ q)
{
    if (p >= m.N) return FoldStat{__builtin_inff(), 0.f, 0.f, 0};
    const int N = m.N;
    double T1[3], T2[3];
    tangents_at<PER>(m, p, z, T1, T2);
    const double w1 = w[p], w2 = w[N + p];
    const double g1 = w1 * T2[0] - w2 * T1[0];
    const double g2 = w1 * T2[1] - w2 * T1[1];
    const double g3 = w1 * T2[2] - w2 * T1[2];
    gam[p] = g1;
    gam[N + p] = g2;
    gam[2 * N + p] = g3;
    const double c1 = T1[1] * T2[2] - T1[2] * T2[1];
    const double c2 = T1[2] * T2[0] - T1[0] * T2[2];
    const double c3 = T1[0] * T2[1] - T1[1] * T2[0];
    q[p] = (g1 * g1 + g2 * g2 + g3 * g3) / (c1 * c1 + c2 * c2 + c3 * c3);
    return fold_stat(T1, T2, c3, periodic_of<PER>(m));
}

// ---------------------------------------------------------------------------
// periodic image bookkeeping
// ---------------------------------------------------------------------------

// Image bookkeeping along one axis for target index i on n points:
// sources j < b sit at shift s_lo, sources j >= b at s_hi = s_lo - 1.  The
// source at j == b has offset exactly -n/2 when n is even (a tie).
struct AxisImg {
    int b;
    int s_lo;
};

__device__ __forceinline__ AxisImg axis_img(int i, int n);

// axis_img on a mesh: a free sheet has no images (every source at shift 0,
// the breakpoint past the end of the axis).
__device__ __forceinline__ AxisImg axis_img_m(const Mesh& m, int i, int n)
{
    if (!m.periodic) {
        AxisImg a;
        a.b = n;
        a.s_lo = 0;
        return a;
    }
    return axis_img(i, n);
}

__device__ __forceinline__ AxisImg axis_img(int i, int n)
{
    const int H = n >> 1;
    AxisImg a;
    a.b = (i >= H) ? i - H : i + n - H;
    a.s_lo = (i >= H) ? 1 : 0;
    return a;
}

// Unscaled contributions of sources [k0, k0 + cnt) of the current LDS tile,
// all in one source row and one column segment, to the lane's R targets.
// CORE: every target of the lane has a fixed image shift over the segment,
// already folded into xt.  Otherwise (seam band) the axis-1 shift is chosen
// per source: sources with column < b1 sit at shift Sx_lo, the others at
// Sx_hi.
// ---------------------------------------------------------------------------
// all-pairs BR sweep, FP32 pair arithmetic, FP64 per-target sums
// ---------------------------------------------------------------------------
//
// Coordinates are tile-relative: the workgroup takes the FP64 position c of
// a target near the middle of its patch, and every staged source is stored
// as the FP32 rounding of (z_j + S_c(j) L - c), where S_c(j) is the source's
// periodic image seen from that centre target.  Near pairs therefore
// subtract small numbers (error ~ ulp of the patch extent, not of the
// domain).  A lane's own image differs from the centre's only for sources in
// the antipodal band (columns / rows where some patch target's image
// breakpoint lies); there the difference (a whole period) is added per
// source.  Pair terms and per-row partial sums are FP32; every row's partial
// is added into FP64 per-target accumulators.

// Away from the patch the same factored sum as the FP64 kernel is used
// (a x sum w g - sum w c with c = b x g formed once per staged source), and
// |a - b|^2 + eps^2 is expanded as |a|^2 + (|b|^2 + eps^2 - 2 a.b) with -2b
// and |b|^2 + eps^2 staged per source: 12 VALU operations and the rsqrt per
// pair instead of 17.  Outside a near box of one patch half-extent around
// the patch |r| >= |a|, so the expansion's rounding stays below
// (1 + 2|a|/|r|)^2 <= 9 ulp of |r|^2 + eps^2, and the factored terms, at most
// about twice the direct term, add at most about twice its rounding: a few
// 1e-7 relative per far pair, against the 1e-5 the FP32 form is held to.
// Inside the near box, in the antipodal band and for extra image layers the
// direct form is used.

#ifndef ZM_PAIR32_UNROLL
#define ZM_PAIR32_UNROLL 2
#endif
#ifndef ZM_F32_FACTORED
#define ZM_F32_FACTORED 1
#endif

// Near box half-width beyond the patch, in patch half-extents.
#ifndef ZM_F32_NEAR_EXTENTS
#define ZM_F32_NEAR_EXTENTS 1.0
#endif
constexpr double kF32NearExtents = ZM_F32_NEAR_EXTENTS;

// Staged FP32 sources, double buffered: (bx, by, bz, g1), (g2, g3, c1, c2), c3.
struct F32Tile {
    float4 a[2][kThreads];
    float4 b[2][kThreads];
    float2 c[2][kThreads];   // (c3, |b|^2 + eps^2)
};

// MODE 0: direct form; 1: direct form with the antipodal-band image
// correction; 2: factored form.  The row's partial is a x G - C: the
// factored form adds w g to G and w c to C, the direct form subtracts
// w (r x g) from C.
template <int R, int MODE>
__device__ __forceinline__ void pair_segment_f32(const F32Tile& T, int buf, int k0, int cnt,
                                                 int j1s, int b1, int s1lo, int bc1, int sc1lo,
                                                 float L1, float dm1, const float* ax,
                                                 const float* ay, const float* az, float eps2,
                                                 float (*G)[3], float (*C)[3])
{
    float mx[R], my[R], mz[R], aa[R];   // -2 a and |a|^2 (far-field form only)
    if (MODE == 2) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            mx[r] = -2.f * ax[r];
            my[r] = -2.f * ay[r];
            mz[r] = -2.f * az[r];
            aa[r] = fmaf(ax[r], ax[r], fmaf(ay[r], ay[r], az[r] * az[r]));
        }
    }
#pragma unroll ZM_PAIR32_UNROLL
    for (int c = 0; c < cnt; ++c) {
        const float4 v0 = T.a[buf][k0 + c];
        const float4 v1 = T.b[buf][k0 + c];
        float bx = v0.x;
        if (MODE == 1) {
            const int jj = j1s + c;
            const int si = (jj < b1) ? s1lo : s1lo - 1;
            const int sc = (jj < bc1) ? sc1lo : sc1lo - 1;
            bx = fmaf((float)(si - sc), L1, bx) + dm1;
        }
        const float by = v0.y, bz = v0.z;
        const float g1 = v0.w, g2 = v1.x, g3 = v1.y;
        if (MODE == 2) {
            const float2 cb = T.c[buf][k0 + c];
            const float c1 = v1.z, c2 = v1.w, c3 = cb.x, bb = cb.y;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // |a - b|^2 + eps^2 = |a|^2 + (|b|^2 + eps^2 - 2 a.b): outside the
                // near box (|r| >= |a|) the expansion's rounding stays within
                // (1 + 2|a|/|r|)^2 <= 9 ulp
                const float s = fmaf(mz[r], bz, fmaf(my[r], by, fmaf(mx[r], bx, bb))) + aa[r];
                const float y = __builtin_amdgcn_rsqf(s);
                const float wgt = y * y * y;
                G[r][0] = fmaf(wgt, g1, G[r][0]);
                G[r][1] = fmaf(wgt, g2, G[r][1]);
                G[r][2] = fmaf(wgt, g3, G[r][2]);
                C[r][0] = fmaf(wgt, c1, C[r][0]);
                C[r][1] = fmaf(wgt, c2, C[r][1]);
                C[r][2] = fmaf(wgt, c3, C[r][2]);
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float r1 = ax[r] - bx;
                const float r2 = ay[r] - by;
                const float r3 = az[r] - bz;
                const float s = fmaf(r1, r1, fmaf(r2, r2, fmaf(r3, r3, eps2)));
                const float y = __builtin_amdgcn_rsqf(s);
                const float wgt = y * y * y;
                const float a1 = wgt * g1, a2 = wgt * g2, a3 = wgt * g3;
                // the row's sum is a x G - C: a direct term d enters as C -= d
                C[r][0] = fmaf(-r2, a3, C[r][0]);
                C[r][0] = fmaf(r3, a2, C[r][0]);
                C[r][1] = fmaf(-r3, a1, C[r][1]);
                C[r][1] = fmaf(r1, a3, C[r][1]);
                C[r][2] = fmaf(-r1, a2, C[r][2]);
                C[r][2] = fmaf(r2, a1, C[r][2]);
            }
        }
    }
}

// Position of column a relative to the periodic interval [lo, lo + len) of
// an n-column axis: whether a lies inside, and how many columns from a on
// keep that state.
__device__ __forceinline__ int interval_run(int a, int lo, int len, int n, bool& inside)
{
    int d = a - lo;
    if (d < 0) d += n;
    inside = d < len;
    return inside ? len - d : n - d;
}

// Workgroup = target patch of PX columns x (256/PX)*R rows (lane = one
// column, R rows 256/PX apart) x one range of source rows.
template <int R, int PX>
__device__ __forceinline__ void pairs_f32_block(const Mesh& m, const PairShape& sh,
                                                const double* __restrict__ z,
                                                const double* __restrict__ gam,
                                                double* __restrict__ part, int patch, int split,
                                                const int* __restrict__ fold, F32Tile& T)
{
    constexpr int RY = kThreads / PX;
    constexpr int PY = RY * R;

    const int N = m.N, n1 = m.n1, n2 = m.n2;
    const int tid = threadIdx.x;
    const int ptx = patch % sh.px;
    const int pty = patch / sh.px;
    const int row_begin = split * sh.rows_per_split;
    const int row_end = min(n2, row_begin + sh.rows_per_split);
    if (row_begin >= row_end) return;  // uniform over the workgroup

    // ---- patch centre ----------------------------------------------------
    const int c0 = ptx * PX, r0 = pty * PY;
    const int ci1 = min(c0 + PX / 2, n1 - 1), ci2 = min(r0 + PY / 2, n2 - 1);
    const int pc = ci2 * n1 + ci1;
    const double cx = z[pc], cy = z[N + pc], cz = z[2 * N + pc];
    const AxisImg cimg1 = axis_img_m(m, ci1, n1), cimg2 = axis_img_m(m, ci2, n2);
    // antipodal band along axis 1: breakpoints of columns c0 .. c0+PX-1
    // (none on a free sheet)
    const int band_lo = axis_img_m(m, c0, n1).b;
    const int band_len = !m.periodic ? 0 : (PX >= n1 ? n1 : PX);

    // near box: patch widened by kF32NearExtents patch half-extents
    const double ext = 0.5 * sqrt((double)(PX * PX) * m.h1 * m.h1 + (double)(PY * PY) * m.h2 * m.h2);
    const int d1 = (int)ceil(kF32NearExtents * ext / m.h1);
    const int d2 = (int)ceil(kF32NearExtents * ext / m.h2);
    const int near1_len = PX + 2 * d1 >= n1 ? n1 : PX + 2 * d1;
    const int near1_lo = ((c0 - d1) % n1 + n1) % n1;
    const int near2_len = PY + 2 * d2 >= n2 ? n2 : PY + 2 * d2;
    const int near2_lo = ((r0 - d2) % n2 + n2) % n2;

    // ---- targets of this lane --------------------------------------------
    const int col = c0 + (tid % PX);
    const int rowg = tid / PX;
    const bool col_ok = col < n1;
    const int i1 = col_ok ? col : ci1;
    const AxisImg ax1 = axis_img_m(m, i1, n1);
    float ax[R], az[R], ay[R];
    double ayd[R];
    int b2[R], s2lo[R], pidx[R];
    bool valid[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = r0 + rowg + RY * k;
        valid[k] = col_ok && (r < n2);
        const int i2 = (r < n2) ? r : ci2;
        pidx[k] = i2 * n1 + i1;
        ax[k] = (float)(z[pidx[k]] - cx);
        ayd[k] = z[N + pidx[k]] - cy;
        az[k] = (float)(z[2 * N + pidx[k]] - cz);
        ay[k] = (float)ayd[k];
        const AxisImg a2 = axis_img_m(m, i2, n2);
        b2[k] = a2.b;
        s2lo[k] = a2.s_lo;
    }
    double acc[R][3];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k][0] = acc[k][1] = acc[k][2] = 0.0;

    const int src_begin = row_begin * n1;
    const int src_end = row_end * n1;
    const int ntiles = (src_end - src_begin + kThreads - 1) / kThreads;
    const int side = 2 * m.K + 1;
    const int total = ntiles * side * side;
    const float L1f = (float)m.L1;
    const float eps2f = (float)m.eps2;
    // the sheet's tangent map keeps index distance a bound on distance (see
    // the fold statistics above): the far forms may be used this evaluation
    const bool far_ok = fold == nullptr || fold[4] == 0;

    // ---- staging: source j relative to the centre, centre's image --------
    float4 st0, st1;
    float2 st2;
    auto load_tile = [&](int t) {
        const int tile = t % ntiles;
        const int j = src_begin + tile * kThreads + tid;
        if (j < src_end) {
            const int j2 = j / n1, j1 = j - j2 * n1;
            const int sc1 = (j1 < cimg1.b) ? cimg1.s_lo : cimg1.s_lo - 1;
            const int sc2 = (j2 < cimg2.b) ? cimg2.s_lo : cimg2.s_lo - 1;
            const double bx = (z[j] + (double)sc1 * m.L1) - cx;
            const double by = (z[N + j] + (double)sc2 * m.L2) - cy;
            const double bz = z[2 * N + j] - cz;
            const double g1 = gam[j], g2 = gam[N + j], g3 = gam[2 * N + j];
            const float bxf = (float)bx, byf = (float)by, bzf = (float)bz;
            st0 = make_float4(bxf, byf, bzf, (float)g1);
            st1 = make_float4((float)g2, (float)g3, (float)(by * g3 - bz * g2),
                              (float)(bz * g1 - bx * g3));
            // |b|^2 + eps^2 of the staged (rounded) offsets, rounded once
            const double bbd = (double)bxf * bxf + (double)byf * byf + (double)bzf * bzf + (double)eps2f;
            st2 = make_float2((float)(bx * g2 - by * g1), (float)bbd);
        } else {
            st0 = make_float4(0.f, 0.f, 0.f, 0.f);
            st1 = make_float4(0.f, 0.f, 0.f, 0.f);
            st2 = make_float2(0.f, 1.f);
        }
    };
    auto store_tile = [&](int buf) {
        T.a[buf][tid] = st0;
        T.b[buf][tid] = st1;
        T.c[buf][tid] = st2;
    };

    load_tile(0);
    store_tile(0);
    __syncthreads();

    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) load_tile(t + 1);
        const int img = t / ntiles;
        const int tile = t - img * ntiles;
        const int m1 = img % side - m.K;
        const int m2 = img / side - m.K;
        // extra image layers shift every source by (m1 L1, m2 L2)
        const float dm1 = (float)((double)m1 * m.L1);
        const bool layer0 = m1 == 0 && m2 == 0;

        const int j0 = src_begin + tile * kThreads;
        const int cnt = min(kThreads, src_end - j0);
        int j2 = j0 / n1;
        int j1 = j0 - j2 * n1;
        int k = 0;
        while (k < cnt) {
            const int seg = min(cnt - k, n1 - j1);
            const int sc2 = (j2 < cimg2.b) ? cimg2.s_lo : cimg2.s_lo - 1;
            float ayr[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int s2 = (j2 < b2[r]) ? s2lo[r] : s2lo[r] - 1;
                ayr[r] = (float)(ayd[r] - (double)(s2 - sc2 + m2) * m.L2);
            }
            bool near_row;
            interval_run(j2, near2_lo, near2_len, n2, near_row);
            const bool fact_row = ZM_F32_FACTORED && layer0 && far_ok;
            float G[R][3], C[R][3];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                G[r][0] = G[r][1] = G[r][2] = 0.f;
                C[r][0] = C[r][1] = C[r][2] = 0.f;
            }

            int a = j1;
            const int e = j1 + seg;
            while (a < e) {
                bool in_band, in_near = false;
                int run = interval_run(a, band_lo, band_len, n1, in_band);
                if (near_row) {
                    const int rn = interval_run(a, near1_lo, near1_len, n1, in_near);
                    run = min(run, rn);
                }
                const int stop = min(e, a + run);
                const int kk = k + (a - j1);
                if (in_band || m1 != 0) {
                    pair_segment_f32<R, 1>(T, buf, kk, stop - a, a, ax1.b, ax1.s_lo, cimg1.b,
                                           cimg1.s_lo, L1f, dm1, ax, ayr, az, eps2f, G, C);
                } else if (in_near || !fact_row) {
                    pair_segment_f32<R, 0>(T, buf, kk, stop - a, a, ax1.b, ax1.s_lo, cimg1.b,
                                           cimg1.s_lo, L1f, dm1, ax, ayr, az, eps2f, G, C);
                } else {
                    pair_segment_f32<R, 2>(T, buf, kk, stop - a, a, ax1.b, ax1.s_lo, cimg1.b,
                                           cimg1.s_lo, L1f, dm1, ax, ayr, az, eps2f, G, C);
                }
                a = stop;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // a x G - C, combined in FP64
                const double gx = G[r][0], gy = G[r][1], gz = G[r][2];
                acc[r][0] += ((double)ayr[r] * gz - (double)az[r] * gy) - (double)C[r][0];
                acc[r][1] += ((double)az[r] * gx - (double)ax[r] * gz) - (double)C[r][1];
                acc[r][2] += ((double)ax[r] * gy - (double)ayr[r] * gx) - (double)C[r][2];
            }
            k += seg;
            j1 += seg;
            if (j1 == n1) { j1 = 0; ++j2; }
        }
        if (t + 1 < total) store_tile(buf ^ 1);
        __syncthreads();
    }

    double* out = part + (size_t)split * 3 * N;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (valid[r]) {
            out[pidx[r]] = acc[r][0];
            out[N + pidx[r]] = acc[r][1];
            out[2 * N + pidx[r]] = acc[r][2];
        }
    }
}

// ---------------------------------------------------------------------------
// all-pairs BR sweep, FP64, factored form on patch-relative coordinates
// ---------------------------------------------------------------------------
//
// With a = target - centre and b = source image - centre (the centre is a
// target near the middle of a compact patch, source images taken as seen
// from it), sum_j w_j (a - b_j) x g_j = a x (sum_j w_j g_j) - sum_j w_j c_j
// with c_j = b_j x g_j computed once per source while staging.  Per pair
// that leaves the distance, the weight and two 3-vector accumulations (17
// VALU operations instead of 21).  The cancellation between the two terms is
// bounded by |a| / |r| ~ the patch extent over the spacing for near pairs.
// In the antipodal band a lane's image of a source differs from the
// centre's by d = 0 or +-L1 along x.  Outside the near box the lane shifts
// the staged record to its own image (b_x + d: -2b_x, |b|^2 + eps^2 and the
// two components of c that involve b_x; a select and five FP64 operations
// per source and lane, shared by its R targets) and takes the factored far
// form; inside the near box the direct form is used with the same
// per-source correction.  On meshes where a
// patch is wide compared with the finest spacing (strongly anisotropic
// spacings, or a patch that spans a short axis), that cancellation could
// reach the FP64 tolerance, so there every source takes the direct form.

// Largest patch half-extent, in units of the finest mesh spacing, for which
// the factored form is used.
constexpr double kFactoredMaxExtent = 32.0;

__host__ __device__ inline bool factored_ok(const Mesh& m, int PX, int PY)
{
    const double ex = 0.5 * (double)(PX < m.n1 ? PX : m.n1) * m.h1;
    const double ey = 0.5 * (double)(PY < m.n2 ? PY : m.n2) * m.h2;
    const double h = m.h1 < m.h2 ? m.h1 : m.h2;
    const double lim = kFactoredMaxExtent * h;
    return ex * ex + ey * ey <= lim * lim;
}

enum { kF64Direct = 0, kF64FactNear = 1, kF64FactFar = 2, kF64BandFar = 3 };

// Antipodal-band sources outside the near box take the factored far form on
// the lane's own image (1) or the direct form (0).
#ifndef ZM_BAND_FACTORED
#define ZM_BAND_FACTORED 1
#endif


// Near box half-width beyond the patch, in patch half-extents, for the
// expanded |r|^2 of the FP64 factored form.  A source outside it lies at
// least one half-extent beyond the patch, so |r| >= ext >= |a| and the
// expansion's rounding, ulp * (|a| + |b|)^2 / |r|^2 with |b| <= |r| + |a|,
// stays below 9 ulp (1 + 2 |a| / |r|)^2.
#ifndef ZM_F64_NEAR_EXTENTS
#define ZM_F64_NEAR_EXTENTS 1.0
#endif
constexpr double kF64NearExtents = ZM_F64_NEAR_EXTENTS;

// MODE: kF64Direct (direct form, antipodal band), kF64FactNear (factored,
// |r|^2 from r = a - b), kF64FactFar (factored, |r|^2 expanded as
// |a|^2 + |b|^2 + eps^2 - 2 a.b: only for sources outside the near box,
// where |r| >= |a| bounds its rounding by a few ulp), kF64BandFar (the far
// form on the lane's own image of an antipodal-band source outside the near
// box; the segment must not cross the centre's breakpoint bc1).
template <int R, int MODE>
__device__ __forceinline__ void pair_segment_f64f(const double2 (*__restrict__ buf)[kThreads],
                                                  int k0, int cnt, int j1s, int b1, int s1lo,
                                                  int bc1, int sc1lo, double L1, const double* ax, const double* ay,
                                                  const double* az, const double* aa, double eps2,
                                                  double (*A)[3], double (*B)[3])
{
    // kF64BandFar: the lane's image shift d = (s_lane - s_centre) L1 is dA
    // before the lane's breakpoint b1 and dA - L1 from it on (the centre's
    // image is constant over the segment); both are exact
    const int scb = (j1s < bc1) ? sc1lo : sc1lo - 1;
    const double dA = (double)(s1lo - scb) * L1, dB = dA - L1;
#pragma unroll ZM_PAIR_UNROLL
    for (int c = 0; c < cnt; ++c) {
        const double2 v0 = buf[0][k0 + c];
        const double2 v1 = buf[1][k0 + c];
        const double2 v2 = buf[2][k0 + c];
        double mx = v0.x;   // m = -2 b (exact)
        const double my = v0.y, mz = v1.x;
        const double g1 = v1.y, g2 = v2.x, g3 = v2.y;
        if (MODE == kF64BandFar) {
            const double d = (j1s + c < b1) ? dA : dB;   // 0 or +-L1
            const double2 v3 = buf[3][k0 + c];
            const double2 v4 = buf[4][k0 + c];
            // the record of b + d e1: m_x = -2 (b_x + d) rounded once,
            // |b + d e1|^2 + eps^2 = bb + d (d + 2 b_x), c_2 - d g_3, c_3 + d g_2
            const double mxs = fma(-2.0, d, mx);
            const double bbs = fma(d, d - mx, v4.y);
            const double c1 = v3.x, c2 = fma(-d, g3, v3.y), c3 = fma(d, g2, v4.x);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double s = fma(az[r], mz, fma(ay[r], my, fma(ax[r], mxs, bbs))) + aa[r];
                const double wgt = inv_cube_sqrt(s);
                A[r][0] = fma(wgt, g1, A[r][0]);
                A[r][1] = fma(wgt, g2, A[r][1]);
                A[r][2] = fma(wgt, g3, A[r][2]);
                B[r][0] = fma(wgt, c1, B[r][0]);
                B[r][1] = fma(wgt, c2, B[r][1]);
                B[r][2] = fma(wgt, c3, B[r][2]);
            }
        } else if (MODE == kF64Direct) {
            const int jj = j1s + c;
            const int si = (jj < b1) ? s1lo : s1lo - 1;
            const int sc = (jj < bc1) ? sc1lo : sc1lo - 1;
            // -2 (b_x + d L1) rounded once: exactly -2 times the rounded b_x + d L1
            mx = fma(-2.0 * (double)(si - sc), L1, mx);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double r1 = fma(0.5, mx, ax[r]);   // a - b, rounded as the subtraction is
                const double r2 = fma(0.5, my, ay[r]);
                const double r3 = fma(0.5, mz, az[r]);
                const double s = fma(r1, r1, fma(r2, r2, fma(r3, r3, eps2)));
                const double wgt = inv_cube_sqrt(s);
                const double a1 = wgt * g1, a2 = wgt * g2, a3 = wgt * g3;
                A[r][0] = fma(r2, a3, A[r][0]);
                A[r][0] = fma(-r3, a2, A[r][0]);
                A[r][1] = fma(r3, a1, A[r][1]);
                A[r][1] = fma(-r1, a3, A[r][1]);
                A[r][2] = fma(r1, a2, A[r][2]);
                A[r][2] = fma(-r2, a1, A[r][2]);
            }
        } else {
            const double2 v3 = buf[3][k0 + c];
            const double2 v4 = buf[4][k0 + c];
            const double c1 = v3.x, c2 = v3.y, c3 = v4.x, bb = v4.y;   // bb = |b|^2 + eps^2
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double s;
                if (MODE == kF64FactFar) {
                    // |a - b|^2 + eps^2 = |a|^2 + (|b|^2 + eps^2 - 2 a.b): 4 operations instead of 6
                    s = fma(az[r], mz, fma(ay[r], my, fma(ax[r], mx, bb))) + aa[r];
                } else {
                    const double r1 = fma(0.5, mx, ax[r]);
                    const double r2 = fma(0.5, my, ay[r]);
                    const double r3 = fma(0.5, mz, az[r]);
                    s = fma(r1, r1, fma(r2, r2, fma(r3, r3, eps2)));
                }
                // A pair with r = 0 (the self pair, or a coincident point)
                // contributes exactly 0.  In the factored sum its two terms
                // a x w g and w (b x g) cancel only to rounding, and w =
                // eps^-3 would blow that residue up for small eps; r = 0 is
                // exactly s == eps^2 here (r is formed exactly above).
                const double wgt = (MODE == kF64FactNear && s == eps2) ? 0.0 : inv_cube_sqrt(s);
                A[r][0] = fma(wgt, g1, A[r][0]);
                A[r][1] = fma(wgt, g2, A[r][1]);
                A[r][2] = fma(wgt, g3, A[r][2]);
                B[r][0] = fma(wgt, c1, B[r][0]);
                B[r][1] = fma(wgt, c2, B[r][1]);
                B[r][2] = fma(wgt, c3, B[r][2]);
            }
        }
    }
}

// Staged FP64 sources, double buffered: v[buffer][(bx,by) (bz,g1) (g2,g3)
// (c1,c2) (c3, |b|^2 + eps^2)][source].
struct F64Tile {
    double2 v[2][5][kThreads];
};

// Workgroup = target patch of PX columns x (256/PX)*R rows (lane = one
// column, R rows 256/PX apart) x one range of source rows.
template <int R, int PX>
__device__ __forceinline__ void pairs_f64f_block(const Mesh& m, const PairShape& sh,
                                                 const double* __restrict__ z,
                                                 const double* __restrict__ gam,
                                                 double* __restrict__ part, int patch, int split,
                                                 const int* __restrict__ fold, F64Tile& T)
{
    constexpr int RY = kThreads / PX;
    constexpr int PY = RY * R;

    const int N = m.N, n1 = m.n1, n2 = m.n2;
    const int tid = threadIdx.x;
    const int ptx = patch % sh.px;
    const int pty = patch / sh.px;
    const int row_begin = split * sh.rows_per_split;
    const int row_end = min(n2, row_begin + sh.rows_per_split);
    if (row_begin >= row_end) return;  // uniform over the workgroup

    // ---- patch centre ----------------------------------------------------
    const int c0 = ptx * PX, r0 = pty * PY;
    const int ci1 = min(c0 + PX / 2, n1 - 1), ci2 = min(r0 + PY / 2, n2 - 1);
    const int pc = ci2 * n1 + ci1;
    const double cx = z[pc], cy = z[N + pc], cz = z[2 * N + pc];
    const AxisImg cimg1 = axis_img_m(m, ci1, n1), cimg2 = axis_img_m(m, ci2, n2);
    const int band_lo = axis_img_m(m, c0, n1).b;   // n1 (no band) on a free sheet
    const bool band_all = PX >= n1 || !factored_ok(m, PX, PY);
    const bool band_wraps = m.periodic && band_lo + PX > n1;
    // near box: the patch widened by kF64NearExtents patch half-extents
    const double ext = 0.5 * sqrt((double)(PX * PX) * m.h1 * m.h1 + (double)(PY * PY) * m.h2 * m.h2);
    const int d1 = (int)ceil(kF64NearExtents * ext / m.h1);
    const int d2 = (int)ceil(kF64NearExtents * ext / m.h2);
    const int near1_len = PX + 2 * d1 >= n1 ? n1 : PX + 2 * d1;
    const int near1_lo = ((c0 - d1) % n1 + n1) % n1;
    const int near2_len = PY + 2 * d2 >= n2 ? n2 : PY + 2 * d2;
    const int near2_lo = ((r0 - d2) % n2 + n2) % n2;

    // ---- targets of this lane --------------------------------------------
    const int col = c0 + (tid % PX);
    const int rowg = tid / PX;
    const bool col_ok = col < n1;
    const int i1 = col_ok ? col : ci1;
    const AxisImg ax1 = axis_img_m(m, i1, n1);
    double ax0[R], ay0[R], az[R], ax[R], ay[R], aa[R];
    int b2[R], s2lo[R], pidx[R];
    bool valid[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int r = r0 + rowg + RY * k;
        valid[k] = col_ok && (r < n2);
        const int i2 = (r < n2) ? r : ci2;
        pidx[k] = i2 * n1 + i1;
        ax0[k] = z[pidx[k]] - cx;
        ay0[k] = z[N + pidx[k]] - cy;
        az[k] = z[2 * N + pidx[k]] - cz;
        const AxisImg a2 = axis_img_m(m, i2, n2);
        b2[k] = a2.b;
        s2lo[k] = a2.s_lo;
    }
    double U[R][3];
#pragma unroll
    for (int k = 0; k < R; ++k) U[k][0] = U[k][1] = U[k][2] = 0.0;

    const int src_begin = row_begin * n1;
    const int src_end = row_end * n1;
    const int ntiles = (src_end - src_begin + kThreads - 1) / kThreads;
    const int side = 2 * m.K + 1;
    const int total = ntiles * side * side;
    // the sheet's tangent map keeps index distance a bound on distance (see
    // the fold statistics above): the expanded far forms may be used this evaluation
    const bool far_ok = fold == nullptr || fold[4] == 0;

    double2 st[5];
    auto load_tile = [&](int t) {
        const int tile = t % ntiles;
        const int j = src_begin + tile * kThreads + tid;
        if (j < src_end) {
            const int j2 = j / n1, j1 = j - j2 * n1;
            const int sc1 = (j1 < cimg1.b) ? cimg1.s_lo : cimg1.s_lo - 1;
            const int sc2 = (j2 < cimg2.b) ? cimg2.s_lo : cimg2.s_lo - 1;
            const double bx = (z[j] + (double)sc1 * m.L1) - cx;
            const double by = (z[N + j] + (double)sc2 * m.L2) - cy;
            const double bz = z[2 * N + j] - cz;
            const double g1 = gam[j], g2 = gam[N + j], g3 = gam[2 * N + j];
            st[0] = make_double2(-2.0 * bx, -2.0 * by);
            st[1] = make_double2(-2.0 * bz, g1);
            st[2] = make_double2(g2, g3);
            st[3] = make_double2(by * g3 - bz * g2, bz * g1 - bx * g3);
            st[4] = make_double2(bx * g2 - by * g1, fma(bx, bx, fma(by, by, fma(bz, bz, m.eps2))));
        } else {
#pragma unroll
            for (int q = 0; q < 5; ++q) st[q] = make_double2(0.0, 0.0);
            st[4].y = 1.0;   // never read (segments stop at the last source); keeps s > 0 anyway
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 5; ++q) T.v[buf][q][tid] = st[q];
    };

    load_tile(0);
    store_tile(0);
    __syncthreads();

    for (int t = 0; t < total; ++t) {
        const int buf = t & 1;
        if (t + 1 < total) load_tile(t + 1);
        const int img = t / ntiles;
        const int tile = t - img * ntiles;
        const int m1 = img % side - m.K;
        const int m2 = img / side - m.K;
        const double dm1 = (double)m1 * m.L1;
#pragma unroll
        for (int r = 0; r < R; ++r) ax[r] = ax0[r] - dm1;

        const int j0 = src_begin + tile * kThreads;
        const int cnt = min(kThreads, src_end - j0);
        int j2 = j0 / n1;
        int j1 = j0 - j2 * n1;
        int k = 0;
        while (k < cnt) {
            const int seg = min(cnt - k, n1 - j1);
            const int sc2 = (j2 < cimg2.b) ? cimg2.s_lo : cimg2.s_lo - 1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int s2 = (j2 < b2[r]) ? s2lo[r] : s2lo[r] - 1;
                ay[r] = ay0[r] - (double)(s2 - sc2 + m2) * m.L2;
                aa[r] = fma(ax[r], ax[r], fma(ay[r], ay[r], az[r] * az[r]));
            }
            bool near_row;
            interval_run(j2, near2_lo, near2_len, n2, near_row);
            int a = j1;
            const int e = j1 + seg;
            while (a < e) {
                bool in_band;
                int stop;
                if (band_all) {
                    in_band = true; stop = e;
                } else if (!band_wraps) {
                    if (a < band_lo) { in_band = false; stop = min(e, band_lo); }
                    else if (a < band_lo + PX) { in_band = true; stop = min(e, band_lo + PX); }
                    else { in_band = false; stop = e; }
                } else {
                    const int hi_end = band_lo + PX - n1;
                    if (a < hi_end) { in_band = true; stop = min(e, hi_end); }
                    else if (a < band_lo) { in_band = false; stop = min(e, band_lo); }
                    else { in_band = true; stop = e; }
                }
                bool in_near = true;
                if (near_row && !(in_band && (band_all || !ZM_BAND_FACTORED))) {
                    const int rn = interval_run(a, near1_lo, near1_len, n1, in_near);
                    stop = min(stop, a + rn);
                } else if (!in_band) {
                    in_near = false;
                } else if (!band_all && ZM_BAND_FACTORED) {
                    in_near = false;
                }
                // a folded or strongly stretched sheet: exact r everywhere
                if (!far_ok) in_near = true;
                // a band segment of the far form keeps the centre's image fixed
                if (in_band && !in_near && a < cimg1.b && stop > cimg1.b) stop = cimg1.b;
                const int kk = k + (a - j1);
                double A[R][3], B[R][3];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    A[r][0] = A[r][1] = A[r][2] = 0.0;
                    B[r][0] = B[r][1] = B[r][2] = 0.0;
                }
                if (in_band && in_near) {
                    pair_segment_f64f<R, kF64Direct>(T.v[buf], kk, stop - a, a, ax1.b, ax1.s_lo,
                                                     cimg1.b, cimg1.s_lo, m.L1, ax, ay, az, aa,
                                                     m.eps2, A, B);
                    // direct contributions
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        U[r][0] += A[r][0];
                        U[r][1] += A[r][1];
                        U[r][2] += A[r][2];
                    }
                } else {
                    if (in_band)
                        pair_segment_f64f<R, kF64BandFar>(T.v[buf], kk, stop - a, a, ax1.b, ax1.s_lo,
                                                          cimg1.b, cimg1.s_lo, m.L1, ax, ay, az, aa,
                                                          m.eps2, A, B);
                    else if (in_near)
                        pair_segment_f64f<R, kF64FactNear>(T.v[buf], kk, stop - a, a, ax1.b, ax1.s_lo,
                                                           cimg1.b, cimg1.s_lo, m.L1, ax, ay, az, aa,
                                                           m.eps2, A, B);
                    else
                        pair_segment_f64f<R, kF64FactFar>(T.v[buf], kk, stop - a, a, ax1.b, ax1.s_lo,
                                                          cimg1.b, cimg1.s_lo, m.L1, ax, ay, az, aa,
                                                          m.eps2, A, B);
                    // a x A - B
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        U[r][0] += (ay[r] * A[r][2] - az[r] * A[r][1]) - B[r][0];
                        U[r][1] += (az[r] * A[r][0] - ax[r] * A[r][2]) - B[r][1];
                        U[r][2] += (ax[r] * A[r][1] - ay[r] * A[r][0]) - B[r][2];
                    }
                }
                a = stop;
            }
            k += seg;
            j1 += seg;
            if (j1 == n1) { j1 = 0; ++j2; }
        }
        if (t + 1 < total) store_tile(buf ^ 1);
        __syncthreads();
    }

    double* out = part + (size_t)split * 3 * N;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (valid[r]) {
            out[pidx[r]] = U[r][0];
            out[N + pidx[r]] = U[r][1];
            out[2 * N + pidx[r]] = U[r][2];
        }
    }
}

// ---------------------------------------------------------------------------
// split-tie correction
// ---------------------------------------------------------------------------

// Tie-kernel shape.  Pass 0 (n1 even) corrects the tie column, pass 1 (n2
// even) the tie row.  All targets of one mesh column share their tie column,
// all targets of one mesh row their tie row, so a workgroup takes a segment
// of one such line of targets and stages the line's tie sources through LDS.
// A line of len targets gets L lanes per target (a power of two, at most 32,
// at least the smallest with 256 / L <= len); the lanes of a target split its
// sources and are combined by a fixed butterfly, so the result does not
// depend on scheduling.
struct TieShape {
    int lanes[2];      // L per pass
    int segs[2];       // workgroups per line per pass
    int blocks[2];     // workgroups per pass (0 if the pass is not needed)
};

__host__ __device__ inline int tie_lanes_for(int len)
{
    int L = 1;
    while (L < 32 && kThreads / L > len) L *= 2;
    return L;
}

// On meshes of >= 16384 points more lanes per target are used until both
// passes together have this many threads (enough waves to hide latency);
// small meshes keep few lanes, which is faster there.
#ifndef ZM_TIE_MIN_THREADS
#define ZM_TIE_MIN_THREADS 524288
#endif

__host__ __device__ inline TieShape tie_shape(int n1, int n2)
{
    TieShape t;
    const int len[2] = {n2, n1}, lines[2] = {n1, n2};
    const bool need[2] = {(n1 & 1) == 0, (n2 & 1) == 0};
    for (int P = 0; P < 2; ++P) {
        t.lanes[P] = tie_lanes_for(len[P]);
        while (n1 * n2 >= 16384 && t.lanes[P] < 32 &&
               2L * n1 * n2 * t.lanes[P] < (long)ZM_TIE_MIN_THREADS)
            t.lanes[P] *= 2;
        const int per = kThreads / t.lanes[P];
        t.segs[P] = (len[P] + per - 1) / per;
        t.blocks[P] = need[P] ? lines[P] * t.segs[P] : 0;
    }
    return t;
}

// Workgroups of one tie launch (grid.y = 2 passes).
__host__ __device__ inline int tie_blocks(int n1, int n2)
{
    const TieShape t = tie_shape(n1, n2);
    return t.blocks[0] > t.blocks[1] ? t.blocks[0] : t.blocks[1];
}

// Adds c * (r x g) / (|r|^2 + eps^2)^(3/2) with r = (dx - S1 L1, dy - S2 L2, dz),
// where (dx, dy, dz) = target - source.
__device__ __forceinline__ void tie_term(const Mesh& m, double dx, double dy, double dz,
                                         double g1, double g2, double g3, double S1, double S2,
                                         double c, double acc[3])
{
    const double r1 = dx - S1 * m.L1;
    const double r2 = dy - S2 * m.L2;
    const double r3 = dz;
    const double s = r1 * r1 + r2 * r2 + r3 * r3 + m.eps2;
    const double wgt = c * inv_cube_sqrt(s);
    acc[0] += wgt * (r2 * g3 - r3 * g2);
    acc[1] += wgt * (r3 * g1 - r1 * g3);
    acc[2] += wgt * (r1 * g2 - r2 * g1);
}

// One workgroup of the tie kernel: block blk of pass `pass` (see TieShape).
// The pair kernels counted each tied source once at the image s_hi; the
// correct weight is 1/2 at s_hi and 1/2 at s_lo on each tied axis, 1/4 at
// each of the four images of the corner (tied on both axes, handled by pass
// 0).  Writes tie[pass][3][N] for the block's targets.  lds: 3 x kThreads
// (x, y) (z, g1) (g2, g3) of the staged tie sources.
template <int PASS>
__device__ __forceinline__ void ties_block(const Mesh& m, int blk,
                                           const double* __restrict__ z,
                                           const double* __restrict__ gam,
                                           double* __restrict__ tie,
                                           double2 (*__restrict__ lds)[kThreads])
{
    constexpr int pass = PASS;
    const TieShape ts = tie_shape(m.n1, m.n2);
    if (blk >= ts.blocks[pass]) return;   // uniform over the workgroup
    const int N = m.N, n1 = m.n1, n2 = m.n2;
    const bool even1 = (n1 & 1) == 0, even2 = (n2 & 1) == 0;
    const int L = ts.lanes[pass];
    const int per = kThreads / L;
    const int line = blk / ts.segs[pass];
    const int seg = blk - line * ts.segs[pass];
    const int slot = threadIdx.x / L, lane = threadIdx.x % L;
    const int len = pass == 0 ? n2 : n1;          // targets of the line = tie sources
    const int k_t = seg * per + slot;             // target's place along the line
    const bool active = k_t < len;
    const int i1 = pass == 0 ? line : k_t;
    const int i2 = pass == 0 ? k_t : line;
    const int p = active ? i2 * n1 + i1 : 0;
    const AxisImg a1 = axis_img(i1, n1);
    const AxisImg a2 = axis_img(i2, n2);
    const double xi = z[p], yi = z[N + p], zi = z[2 * N + p];
    // tie line: column a1.b (pass 0) or row a2.b (pass 1); a1.b and a2.b are
    // the same for every target of the workgroup on the line's axis
    const int tie_line = pass == 0 ? a1.b : a2.b;
    double acc[3] = {0.0, 0.0, 0.0};

    for (int c0 = 0; c0 < len; c0 += kThreads) {
        const int cn = len - c0 < kThreads ? len - c0 : kThreads;
        __syncthreads();   // previous chunk fully read
        if ((int)threadIdx.x < cn) {
            const int k = c0 + threadIdx.x;
            const int pj = pass == 0 ? k * n1 + tie_line : tie_line * n1 + k;
            lds[0][threadIdx.x] = make_double2(z[pj], z[N + pj]);
            lds[1][threadIdx.x] = make_double2(z[2 * N + pj], gam[pj]);
            lds[2][threadIdx.x] = make_double2(gam[N + pj], gam[2 * N + pj]);
        }
        __syncthreads();
        if (!active) continue;
        for (int m2 = -m.K; m2 <= m.K; ++m2) {
            for (int m1 = -m.K; m1 <= m.K; ++m1) {
                const double lo1 = a1.s_lo + m1, hi1 = a1.s_lo - 1 + m1;
                const double lo2 = a2.s_lo + m2, hi2 = a2.s_lo - 1 + m2;
                // Every source of the line takes +1/2 at one end image and -1/2
                // at the other; the corner (pass 0) is completed below, the
                // corner's place in the tie row (pass 1) gets weight 0.
#pragma unroll 4
                for (int kk = lane; kk < cn; kk += L) {
                    const int k = c0 + kk;   // source index along the tie line
                    const double2 v0 = lds[0][kk], v1 = lds[1][kk], v2 = lds[2][kk];
                    const double dx = xi - v0.x, dy = yi - v0.y, dz = zi - v1.x;
                    const double g1 = v1.y, g2 = v2.x, g3 = v2.y;
                    if (PASS == 0) {
                        // end images differ along axis 1: r = (r1a | r1b, r2, r3)
                        const double r2 = dy - ((k < a2.b) ? lo2 : hi2) * m.L2;
                        const double t = fma(r2, r2, fma(dz, dz, m.eps2));
                        const double r1a = dx - lo1 * m.L1, r1b = dx - hi1 * m.L1;
                        const double wa = 0.5 * inv_cube_sqrt(fma(r1a, r1a, t));
                        const double wb = -0.5 * inv_cube_sqrt(fma(r1b, r1b, t));
                        const double W = wa + wb, M = fma(wa, r1a, wb * r1b);
                        acc[0] = fma(W, r2 * g3 - dz * g2, acc[0]);
                        acc[1] = fma(W * dz, g1, fma(-M, g3, acc[1]));
                        acc[2] = fma(M, g2, fma(-W * r2, g1, acc[2]));
                    } else {
                        // end images differ along axis 2: r = (r1, r2a | r2b, r3);
                        // the corner's place in the row has weight 0
                        const double c = (even1 && k == a1.b) ? 0.0 : 0.5;
                        const double r1 = dx - ((k < a1.b) ? lo1 : hi1) * m.L1;
                        const double t = fma(r1, r1, fma(dz, dz, m.eps2));
                        const double r2a = dy - lo2 * m.L2, r2b = dy - hi2 * m.L2;
                        const double wa = c * inv_cube_sqrt(fma(r2a, r2a, t));
                        const double wb = -c * inv_cube_sqrt(fma(r2b, r2b, t));
                        const double W = wa + wb, M = fma(wa, r2a, wb * r2b);
                        acc[0] = fma(M, g3, fma(-W * dz, g2, acc[0]));
                        acc[1] = fma(W, dz * g1 - r1 * g3, acc[1]);
                        acc[2] = fma(W * r1, g2, fma(-M, g1, acc[2]));
                    }
                }
            }
        }
    }
    if (pass == 0 && even2 && active && lane == 0) {
        // corner (tied on both axes): the loop gave +1/2 at (lo1, hi2) and -1/2
        // at (hi1, hi2); the weights are 1/4, 1/4, 1/4 at (lo1, lo2), (lo1, hi2),
        // (hi1, lo2) and -3/4 at (hi1, hi2)
        const int pj = a2.b * n1 + a1.b;
        const double dx = xi - z[pj], dy = yi - z[N + pj], dz = zi - z[2 * N + pj];
        const double g1 = gam[pj], g2 = gam[N + pj], g3 = gam[2 * N + pj];
        for (int m2 = -m.K; m2 <= m.K; ++m2) {
            for (int m1 = -m.K; m1 <= m.K; ++m1) {
                const double lo1 = a1.s_lo + m1, hi1 = a1.s_lo - 1 + m1;
                const double lo2 = a2.s_lo + m2, hi2 = a2.s_lo - 1 + m2;
                tie_term(m, dx, dy, dz, g1, g2, g3, lo1, lo2, 0.25, acc);
                tie_term(m, dx, dy, dz, g1, g2, g3, lo1, hi2, -0.25, acc);
                tie_term(m, dx, dy, dz, g1, g2, g3, hi1, lo2, 0.25, acc);
                tie_term(m, dx, dy, dz, g1, g2, g3, hi1, hi2, -0.25, acc);
            }
        }
    }
    // butterfly over the target's lanes (consecutive lanes of one wave)
    for (int off = L / 2; off > 0; off >>= 1) {
        acc[0] += __shfl_xor(acc[0], off, L);
        acc[1] += __shfl_xor(acc[1], off, L);
        acc[2] += __shfl_xor(acc[2], off, L);
    }
    if (active && lane == 0) {
        double* out = tie + (size_t)pass * 3 * N;
        out[p] = acc[0];
        out[N + p] = acc[1];
        out[2 * N + p] = acc[2];
    }
}

// ---------------------------------------------------------------------------
// reduction over source splits, Bernoulli potential
// ---------------------------------------------------------------------------

// Lanes per point of the split reduction (1, 4 or 16, never more than the
// splits): small meshes have few points, so several lanes share a point's
// splits to keep enough loads in flight.
__host__ __device__ inline int reduce_lanes(int N, int splits)
{
    int L = N >= 65536 ? 1 : (N >= 16384 ? 4 : 16);
    while (L > 1 && L > splits) L >>= 2;
    return L;
}

// u = coef * (sum over splits + tie passes) at point p, and V.  Lanes
// lane = 0 .. L-1 of a group take the splits lane, lane + L, ... in order and
// are combined by a fixed butterfly; the tie passes (if ties) are added and
// lane 0 writes.
// All lanes of a group must call this together.
template <int L>
__device__ __forceinline__ void reduce_group(const Mesh& m, int p, int lane, int splits,
                                             const double* __restrict__ part,
                                             const double* __restrict__ tie,
                                             const double* __restrict__ q,
                                             const double* __restrict__ z, double* __restrict__ u,
                                             double* __restrict__ V, bool ties)
{
    if (p >= m.N) return;   // the whole lane group leaves together
    const size_t N = m.N;
    double a[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // strided sum over the splits; loads are issued 8 at a time
        double s = 0.0;
        int k = lane;
        for (; k + 7 * L < splits; k += 8 * L) {
            double v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = part[((size_t)(k + t * L) * 3 + c) * N + p];
#pragma unroll
            for (int t = 0; t < 8; ++t) s += v[t];
        }
        for (; k < splits; k += L) s += part[((size_t)k * 3 + c) * N + p];
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
        if (ties && (m.n1 & 1) == 0) s += tie[c * N + p];
        if (ties && (m.n2 & 1) == 0) s += tie[(3 + c) * N + p];
        a[c] = m.coef * s;
    }
    if (lane != 0) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c * N + p] = a[c];
    if (V) {
        const double uu = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
        V[p] = m.atwood * ((uu - 0.25 * q[p]) - (2.0 * m.gravity) * z[2 * N + p]);
    }
}

// Dispatch on the lane count for thread t of a reduction over the mesh
// (t / L is the point; L must be uniform over the wave).
__device__ __forceinline__ void reduce_thread(const Mesh& m, int t, int L, int splits,
                                              const double* __restrict__ part,
                                              const double* __restrict__ tie,
                                              const double* __restrict__ q,
                                              const double* __restrict__ z,
                                              double* __restrict__ u, double* __restrict__ V,
                                              bool ties)
{
    if (L == 1) reduce_group<1>(m, t, 0, splits, part, tie, q, z, u, V, ties);
    else if (L == 4) reduce_group<4>(m, t >> 2, t & 3, splits, part, tie, q, z, u, V, ties);
    else reduce_group<16>(m, t >> 4, t & 15, splits, part, tie, q, z, u, V, ties);
}

// ---------------------------------------------------------------------------
// vorticity right-hand side and RK3 stage combination
// ---------------------------------------------------------------------------

// y0 may alias out (the last stage writes the new state over y0 in place,
// each thread reading its own point before writing it), so neither carries
// __restrict__.
template <int PER = -1>
__device__ __forceinline__ void update_point(const Mesh& m, int p, int stage, const double* y0_z,
                                             const double* y0_w, const double* __restrict__ ys_z,
                                             const double* __restrict__ ys_w,
                                             const double* __restrict__ u,
                                             const double* __restrict__ V, double* out_z,
                                             double* out_w, int* __restrict__ nonfinite)
{
    if (p >= m.N) return;
    const int N = m.N, n1 = m.n1, n2 = m.n2;
    const int i2 = p / n1;
    const int i1 = p - i2 * n1;
    const bool per = periodic_of<PER>(m);

    double F[5];
    F[0] = u[p];
    F[1] = u[N + p];
    F[2] = u[2 * N + p];
    double va[4], vb[4];
    stencil4(per, V + (size_t)i2 * n1, 1, n1, i1, 0.0, va);
    stencil4(per, V + i1, (size_t)n1, n2, i2, 0.0, vb);
    F[3] = d1_5pt(va[0], va[1], va[2], va[3], m.h1);
    F[4] = d1_5pt(vb[0], vb[1], vb[2], vb[3], m.h2);
    if (m.nu != 0.0) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double* f = ys_w + (size_t)c * N;
            double fa[4], fb[4];
            stencil4(per, f + (size_t)i2 * n1, 1, n1, i1, 0.0, fa);
            stencil4(per, f + i1, (size_t)n1, n2, i2, 0.0, fb);
            const double lap = d2_5pt(fa[0], fa[1], f[p], fa[2], fa[3], m.h1) +
                               d2_5pt(fb[0], fb[1], f[p], fb[2], fb[3], m.h2);
            F[3 + c] = F[3 + c] + m.nu * lap;
        }
    }

    double o[5];
    if (stage == 3) {
#pragma unroll
        for (int c = 0; c < 5; ++c) o[c] = F[c];
    } else {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const size_t off = (c < 3) ? (size_t)c * N + p : (size_t)(c - 3) * N + p;
            const double yv = (c < 3) ? ys_z[off] : ys_w[off];
            const double a = yv + m.dt * F[c];
            if (stage == 0) {
                o[c] = a;
            } else {
                const double y0v = (c < 3) ? y0_z[off] : y0_w[off];
                if (stage == 1) o[c] = 0.75 * y0v + 0.25 * a;
                else o[c] = (1.0 / 3.0) * y0v + (2.0 / 3.0) * a;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) out_z[(size_t)c * N + p] = o[c];
    out_w[p] = o[3];
    out_w[N + p] = o[4];
    if (nonfinite) {
        bool bad = false;
#pragma unroll
        for (int c = 0; c < 5; ++c) bad |= !isfinite(o[c]);
        if (bad) *nonfinite = 1;
    }
}


}  // namespace dev
}  // namespace zm
