// Low-order Z-Model velocity: the BR integral replaced by its flat-sheet
// approximation u = 1/2 (R1 w1 + R2 w2) n^, R_a the Riesz transform over
// the periodic parameter mesh (symbol i k_a / |k|), evaluated with FFTs
// (the paper's low-order solver, sec. 2).
//
// Both real vorticity components ride in one complex field c = w1 + i w2.
// The symbols c_a = k_a / |k| are odd in k at every mode (they are set to 0
// at k = 0 and, along axis a, at the unpaired mode m_a = n_a / 2), so
// i c_a maps real fields to real fields, and
//   S = 1/2 (R1 w1 + R2 w2) = Re IFFT[ (c2 + i c1) / 2 * FFT(c) ]
// (the real part keeps R1 w1 + R2 w2 and drops R1 w2 - R2 w1): no partner
// mode -m is needed, so the symbol is applied between the forward and the
// inverse transform of the same row.  Five kernels:
//
//   k_lo_pack_rows   row i2: c = w1 + i w2, forward FFT over i1 -> A[i2][m1]
//   k_transpose      32 x 32 tiles through LDS -> B[m1][i2]
//   k_lo_symbol_rows row m1: forward FFT over i2, times (c2 + i c1) / (2N),
//                    inverse FFT over m2 -> B[m1][i2]
//   k_transpose      -> A[i2][m1]
//   k_lo_inv_rows    row i2: inverse FFT over m1 -> S(i1, i2) = Re (one
//                    double plane, in the spent second complex buffer)
//   k_lo_point       per point: u = S n^ (unit normal from the 5-point
//                    tangents), q from w and the tangents,
//                    V = A (|u|^2 - q/4 - 2 g z3) (a plain point kernel: the
//                    stencil loads want the occupancy the FFT rows lack)
//
// Row FFTs: one row of n = 2^L <= 4096 complex doubles per 256-thread
// workgroup, held in LDS (at most 64 KiB); Stockham auto-sort passes of
// radix 16 (and one of radix 2, 4 or 8 for the remaining bits), each thread
// owning one radix-R butterfly per pass in registers: load R inputs at
// stride n / R, twiddle input r by w_{Ns R}^{r k} (k = j mod Ns; w^r by
// repeated multiplication from one table entry), radix-R DFT (radix-2
// decimation-in-frequency network, constant twiddles), store at
// (j - k) R + k + r Ns.  The LDS index is XOR-swizzled within groups of 16
// (e ^ ((e >> 4) & 15)) so that the stride-R stores of the first pass do not
// fall into one bank.  Twiddle tables exp(-2 pi i t / n), t < n, are built by
// k_twiddle in each evaluation.  For n = 4096 the symbol rows keep the row in
// registers between the forward and the inverse transform (fft4096_regs):
// two LDS exchanges per transform instead of four.
#include "zm_device.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace zm {
namespace {

using dev::kThreads;
constexpr int kFftThreads = 256;   // n / R <= 256 for every pass when n <= 4096

__global__ __launch_bounds__(kThreads) void k_twiddle(int n1, double2* __restrict__ tw1, int n2,
                                                      double2* __restrict__ tw2)
{
    const int t = blockIdx.x * kThreads + threadIdx.x;
    double s, c;
    if (t < n1) {
        sincospi(-2.0 * (double)t / (double)n1, &s, &c);
        tw1[t] = make_double2(c, s);
    }
    if (t < n2) {
        sincospi(-2.0 * (double)t / (double)n2, &s, &c);
        tw2[t] = make_double2(c, s);
    }
}

__device__ __forceinline__ int sw(int e) { return e ^ ((e >> 4) & 15); }

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// cos(2 pi m / 16), 0 <= m < 8
__device__ __forceinline__ double cos16(int m)
{
    switch (m) {
    case 0: return 1.0;
    case 1: return 0.92387953251128674;
    case 2: return 0.70710678118654752;
    case 3: return 0.38268343236508977;
    case 4: return 0.0;
    case 5: return -0.38268343236508977;
    case 6: return -0.70710678118654752;
    default: return -0.92387953251128674;
    }
}

// t times exp(-2 pi i m / 16) (INV: exp(+2 pi i m / 16)); m is a constant
// after unrolling, so the branches fold.
template <bool INV>
__device__ __forceinline__ double2 rot16(double2 t, int m)
{
    if (m == 0) return t;
    if (m == 4) return INV ? make_double2(-t.y, t.x) : make_double2(t.y, -t.x);
    const double c = cos16(m);
    const double sn = m < 4 ? cos16(4 - m) : cos16(m - 4);   // sin(2 pi m / 16) > 0
    const double s = INV ? sn : -sn;
    return make_double2(t.x * c - t.y * s, t.x * s + t.y * c);
}

// Radix-R DFT of v[0..R) in registers (decimation in frequency): on return
// v[r] holds X[brev_R(r)].
template <int R, bool INV>
__device__ __forceinline__ void dft(double2 (&v)[16])
{
#pragma unroll
    for (int span = R / 2; span >= 1; span >>= 1) {
#pragma unroll
        for (int s0 = 0; s0 < R; s0 += 2 * span) {
#pragma unroll
            for (int k = 0; k < span; ++k) {
                const double2 a = v[s0 + k], b = v[s0 + k + span];
                v[s0 + k] = make_double2(a.x + b.x, a.y + b.y);
                v[s0 + k + span] = rot16<INV>(make_double2(a.x - b.x, a.y - b.y), k * (8 / span));
            }
        }
    }
}

template <int R>
__device__ constexpr int brev(int r)
{
    int o = 0;
    for (int b = 1, t = R >> 1; b < R; b <<= 1, t >>= 1)
        if (r & b) o |= t;
    return o;
}

// One Stockham pass of radix R over the LDS row x (n points, Ns = product
// of the radices already applied).  Every thread reaches both barriers.
template <int R, bool INV>
__device__ __forceinline__ void fft_pass(double2* x, int n, int Ns, const double2* __restrict__ tw)
{
    const int nb = n / R;
    const int j = threadIdx.x;
    double2 v[16];
    int k = 0;
    if (j < nb) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[sw(j + r * nb)];
        k = j & (Ns - 1);
        if (k != 0) {
            double2 w1 = tw[k * (n / (Ns * R))];
            if (INV) w1.y = -w1.y;
            double2 w = w1;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                v[r] = cmul(v[r], w);
                if (r + 1 < R) w = cmul(w, w1);
            }
        }
        dft<R, INV>(v);
    }
    __syncthreads();
    if (j < nb) {
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) x[sw(base + r * Ns)] = v[brev<R>(r)];
    }
    __syncthreads();
}

// Unnormalised DFT (INV: conjugate twiddles) of the LDS row x, n = 2^logn.
template <bool INV>
__device__ __forceinline__ void fft_row(double2* x, int logn, const double2* __restrict__ tw)
{
    const int n = 1 << logn;
    int Ns = 1, rem = logn;
    while (rem >= 4) {
        fft_pass<16, INV>(x, n, Ns, tw);
        Ns <<= 4;
        rem -= 4;
    }
    if (rem == 3) fft_pass<8, INV>(x, n, Ns, tw);
    else if (rem == 2) fft_pass<4, INV>(x, n, Ns, tw);
    else if (rem == 1) fft_pass<2, INV>(x, n, Ns, tw);
}

// n = 4096 = 16^3 on 256 threads: the first radix-16 pass reads, and the last
// writes, element j + 256 r in thread j (r < 16), which is also the
// coalesced row layout.  So a row enters in registers, goes through LDS only
// for the two exchanges between the three passes, and leaves in registers in
// natural order: v[r] = X[j + 256 r].  Same operations in the same order as
// fft_row (bitwise the same result), half its LDS traffic and barriers.  The
// caller must not touch x between calls except through this function: its
// first barrier orders the previous call's last LDS reads before this call's
// first writes.
template <bool INV>
__device__ __forceinline__ void fft4096_regs(double2 (&v)[16], double2* x,
                                             const double2* __restrict__ tw)
{
    const int j = threadIdx.x;
    // pass 1 (Ns = 1, no twiddles): output 16 j + r
    dft<16, INV>(v);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) x[sw(16 * j + r)] = v[brev<16>(r)];
    __syncthreads();
    // pass 2 (Ns = 16), in place in LDS
    fft_pass<16, INV>(x, 4096, 16, tw);
    // pass 3 (Ns = 256, k = j): output j + 256 r, kept in registers
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = x[sw(j + r * 256)];
    if (j != 0) {
        double2 w1 = tw[j];
        if (INV) w1.y = -w1.y;
        double2 w = w1;
#pragma unroll
        for (int r = 1; r < 16; ++r) {
            v[r] = cmul(v[r], w);
            if (r + 1 < 16) w = cmul(w, w1);
        }
    }
    dft<16, INV>(v);
    double2 o[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) o[r] = v[brev<16>(r)];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = o[r];
}

// Persistent row kernels: workgroup b takes rows b, b + G, b + 2G, ... (G =
// the grid, sized to the workgroups that fit on the CUs at once).  Each
// thread holds its n / 256 elements of the next row in registers: their
// global loads are issued before the current row's FFT passes and land
// while those run, so a row's load no longer waits behind its own compute.
constexpr int kRowRegs = 16;   // elements per thread at n = 4096

// Row i2: c = w1 + i w2 over i1, forward FFT -> A[i2][m1].
__global__ __launch_bounds__(kFftThreads) void k_lo_pack_rows(int logn, int rows, int N,
                                                              const double* __restrict__ w,
                                                              const double2* __restrict__ tw,
                                                              double2* __restrict__ A)
{
    extern __shared__ double2 x[];
    const int n = 1 << logn;
    const int tid = threadIdx.x;
    double2 pre[kRowRegs];
#define ZM_FETCH_PACK(r)                                                                     \
    do {                                                                                     \
        const size_t fb = (size_t)(r) * n;                                                   \
        _Pragma("unroll") for (int k = 0; k < kRowRegs; ++k) {                               \
            const int e = tid + k * kFftThreads;                                             \
            if (e < n) pre[k] = make_double2(w[fb + e], w[N + fb + e]);                      \
        }                                                                                    \
    } while (0)
    int row = blockIdx.x;
    if (row < rows) ZM_FETCH_PACK(row);
    for (; row < rows; row += gridDim.x) {
#pragma unroll
        for (int k = 0; k < kRowRegs; ++k) {
            const int e = tid + k * kFftThreads;
            if (e < n) x[sw(e)] = pre[k];
        }
        __syncthreads();
        const int next = row + gridDim.x;
        if (next < rows) ZM_FETCH_PACK(next);
        fft_row<false>(x, logn, tw);
        const size_t base = (size_t)row * n;
        for (int e = tid; e < n; e += kFftThreads) A[base + e] = x[sw(e)];
        __syncthreads();   // the row is out of LDS before the next one is written
    }
#undef ZM_FETCH_PACK
}

// Row m1 of B (length n2 over i2): forward FFT over i2, times the symbol
// (c2 + i c1) / (2 N) at (m1, m2), inverse FFT over m2, in place.
__global__ __launch_bounds__(kFftThreads) void k_lo_symbol_rows(int n1, int logn2, double L1,
                                                                double L2,
                                                                const double2* __restrict__ tw,
                                                                double2* __restrict__ B)
{
    extern __shared__ double2 x[];
    const int n2 = 1 << logn2;
    const int tid = threadIdx.x;
    double2 pre[kRowRegs];
#define ZM_FETCH_ROW(src, r, len)                                                            \
    do {                                                                                     \
        const double2* fr = (src) + (size_t)(r) * (len);                                     \
        _Pragma("unroll") for (int k = 0; k < kRowRegs; ++k) {                               \
            const int e = tid + k * kFftThreads;                                             \
            if (e < (len)) pre[k] = make_double2(fr[e].x, fr[e].y);                           \
        }                                                                                    \
    } while (0)
    const double h = 0.5 / ((double)n1 * (double)n2);
    int m1 = blockIdx.x;
    if (m1 < n1) ZM_FETCH_ROW(B, m1, n2);
    if (logn2 == 12) {
        for (; m1 < n1; m1 += gridDim.x) {
            double2 v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = pre[k];
            const int next = m1 + gridDim.x;
            if (next < n1) ZM_FETCH_ROW(B, next, n2);
            fft4096_regs<false>(v, x, tw);
            const int s1 = 2 * m1 < n1 ? m1 : m1 - n1;
            const double k1 = 2.0 * M_PI * s1 / L1;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int m2 = tid + k * kFftThreads;
                const int s2 = 2 * m2 < n2 ? m2 : m2 - n2;
                const double k2 = 2.0 * M_PI * s2 / L2;
                // h / |k| from the hardware rsqrt (relative error <= 2^-24) and one
                // correction y0 (1 + e / 2), e = 1 - q y0^2: error ~ 1.5 e^2 < 1e-14
                const double q = k1 * k1 + k2 * k2;
                const double y0 = __builtin_amdgcn_rsq(q);
                const double y = fma(0.5 * y0, fma(-q, y0 * y0, 1.0), y0);
                const double ih = q > 0.0 ? h * y : 0.0;   // 1 / (2N |k|)
                const double mx = (2 * m2 == n2) ? 0.0 : k2 * ih;  // (c2 + i c1) / (2N)
                const double my = (2 * m1 == n1) ? 0.0 : k1 * ih;
                v[k] = make_double2(v[k].x * mx - v[k].y * my, v[k].x * my + v[k].y * mx);
            }
            fft4096_regs<true>(v, x, tw);
            double2* row = B + (size_t)m1 * n2;
#pragma unroll
            for (int k = 0; k < 16; ++k) row[tid + k * kFftThreads] = v[k];
        }
        return;
    }
    for (; m1 < n1; m1 += gridDim.x) {
#pragma unroll
        for (int k = 0; k < kRowRegs; ++k) {
            const int e = tid + k * kFftThreads;
            if (e < n2) x[sw(e)] = pre[k];
        }
        __syncthreads();
        const int next = m1 + gridDim.x;
        if (next < n1) ZM_FETCH_ROW(B, next, n2);
        fft_row<false>(x, logn2, tw);
        const int s1 = 2 * m1 < n1 ? m1 : m1 - n1;
        const double k1 = 2.0 * M_PI * s1 / L1;
        for (int m2 = tid; m2 < n2; m2 += kFftThreads) {
            const int s2 = 2 * m2 < n2 ? m2 : m2 - n2;
            const double k2 = 2.0 * M_PI * s2 / L2;
            const double kk = sqrt(k1 * k1 + k2 * k2);
            double c1 = 0.0, c2 = 0.0;
            if (kk > 0.0) {
                c1 = (2 * m1 == n1) ? 0.0 : k1 / kk;
                c2 = (2 * m2 == n2) ? 0.0 : k2 / kk;
            }
            const double2 v = x[sw(m2)];
            const double mx = c2 * h, my = c1 * h;   // (c2 + i c1) / (2N)
            x[sw(m2)] = make_double2(v.x * mx - v.y * my, v.x * my + v.y * mx);
        }
        __syncthreads();
        fft_row<true>(x, logn2, tw);
        double2* row = B + (size_t)m1 * n2;
        for (int e = tid; e < n2; e += kFftThreads) row[e] = x[sw(e)];
        __syncthreads();
    }
}

// Row i2 of A (over m1): inverse FFT over m1, S = Re -> S[i2][i1].
__global__ __launch_bounds__(kFftThreads) void k_lo_inv_rows(int logn, int rows,
                                                             const double2* __restrict__ tw,
                                                             const double2* __restrict__ A,
                                                             double* __restrict__ S)
{
    extern __shared__ double2 x[];
    const int n = 1 << logn;
    const int tid = threadIdx.x;
    double2 pre[kRowRegs];
    int row = blockIdx.x;
    if (row < rows) ZM_FETCH_ROW(A, row, n);
    for (; row < rows; row += gridDim.x) {
#pragma unroll
        for (int k = 0; k < kRowRegs; ++k) {
            const int e = tid + k * kFftThreads;
            if (e < n) x[sw(e)] = pre[k];
        }
        __syncthreads();
        const int next = row + gridDim.x;
        if (next < rows) ZM_FETCH_ROW(A, next, n);
        fft_row<true>(x, logn, tw);
        const size_t base = (size_t)row * n;
        for (int e = tid; e < n; e += kFftThreads) S[base + e] = x[sw(e)].x;
        __syncthreads();
    }
}
#undef ZM_FETCH_ROW

// Per point: the velocity u = S n^ (not stored when u is null) and V.  A
// 256-thread workgroup owns a tile of tx x ty points (tx = min(64, n1),
// ty = min(256 / tx, n2)); the three position planes of the tile and a
// 2-point halo are staged in LDS once, seam-corrected as they are loaded
// (z1 + w L1 across the i1 seam, z2 + w L2 across the i2 seam, exactly as the
// stencil helper adds them), so the 5-point tangents read LDS instead of
// issuing 24 global loads per point.  Periodic meshes only (the FFT models
// are periodic).
constexpr int kTileMax = (64 + 4) * (4 + 4);   // largest (tx + 4)(ty + 4) over the tile shapes

__global__ __launch_bounds__(kThreads) void k_lo_point(Mesh m, int tx, int ty,
                                                       const double* __restrict__ S,
                                                       const double* __restrict__ z,
                                                       const double* __restrict__ w,
                                                       double* __restrict__ u,
                                                       double* __restrict__ V)
{
    __shared__ double tz[3][kTileMax];
    const int n1 = m.n1, n2 = m.n2, N = m.N;
    const int W = tx + 4, H = ty + 4;
    const int x0 = blockIdx.x * tx, y0 = blockIdx.y * ty;
    for (int e = threadIdx.x; e < W * H; e += kThreads) {
        const int ly = e / W, lx = e - ly * W;
        int w1, w2;
        const int j1 = dev::nbr(x0 - 2, lx, n1, w1);
        const int j2 = dev::nbr(y0 - 2, ly, n2, w2);
        const size_t q = (size_t)j2 * n1 + j1;
        double a = z[q], b = z[N + q];
        if (w1 != 0) a = a + (double)w1 * m.L1;
        if (w2 != 0) b = b + (double)w2 * m.L2;
        tz[0][e] = a;
        tz[1][e] = b;
        tz[2][e] = z[2 * (size_t)N + q];
    }
    __syncthreads();
    const int ly = threadIdx.x / tx, lx = threadIdx.x - ly * tx;
    const int i1 = x0 + lx, i2 = y0 + ly;
    if (ly >= ty || i1 >= n1 || i2 >= n2) return;   // no barrier follows
    const int p = i2 * n1 + i1;
    const int c0 = (ly + 2) * W + (lx + 2);
    double T1[3], T2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* t = tz[c];
        T1[c] = dev::d1_5pt(t[c0 - 2], t[c0 - 1], t[c0 + 1], t[c0 + 2], m.h1);
        T2[c] = dev::d1_5pt(t[c0 - 2 * W], t[c0 - W], t[c0 + W], t[c0 + 2 * W], m.h2);
    }
    {
        const double nx = T1[1] * T2[2] - T1[2] * T2[1];
        const double ny = T1[2] * T2[0] - T1[0] * T2[2];
        const double nz = T1[0] * T2[1] - T1[1] * T2[0];
        const double nn = nx * nx + ny * ny + nz * nz;
        const double inv = 1.0 / sqrt(nn);
        const double s = S[p];
        const double u1 = s * (nx * inv), u2 = s * (ny * inv), u3 = s * (nz * inv);
        if (u) {   // null for the medium-order model, which only needs V
            u[p] = u1;
            u[N + p] = u2;
            u[2 * N + p] = u3;
        }
        if (V) {
            const double w1 = w[p], w2 = w[N + p];
            const double g1 = w1 * T2[0] - w2 * T1[0];
            const double g2 = w1 * T2[1] - w2 * T1[1];
            const double g3 = w1 * T2[2] - w2 * T1[2];
            const double q = (g1 * g1 + g2 * g2 + g3 * g3) / nn;
            const double uu = u1 * u1 + u2 * u2 + u3 * u3;
            V[p] = m.atwood * ((uu - 0.25 * q) - (2.0 * m.gravity) * z[2 * N + p]);
        }
    }
}

// out[c][r] = in[r][c] for an rows x cols array; 32 x 32 tiles, 256 threads.
__global__ __launch_bounds__(kThreads) void k_transpose(const double2* __restrict__ in,
                                                        double2* __restrict__ out, int rows,
                                                        int cols)
{
    __shared__ double2 t[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int r = r0 + k, c = c0 + tx;
        if (r < rows && c < cols) t[k][tx] = in[(size_t)r * cols + c];
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) out[(size_t)c * rows + r] = t[tx][k];
    }
}

inline unsigned grid_for(long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

int log2i(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Workgroups of the persistent row kernels for rows of n complex doubles:
// as many as the CUs hold at once (LDS-bound: 160 KiB per CU, 256 CUs),
// at most one per row.
unsigned row_grid(int n, int rows)
{
    const int per_cu = std::max(1, std::min(8, (160 * 1024) / (int)(sizeof(double2) * n)));
    return (unsigned)std::min(rows, 256 * per_cu);
}

hipError_t transpose(const double2* in, double2* out, int rows, int cols, hipStream_t s)
{
    hipLaunchKernelGGL(k_transpose, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(kThreads), 0, s,
                       in, out, rows, cols);
    return hipGetLastError();
}

}  // namespace

bool low_order_supported_side(int n) { return n >= 8 && n <= 4096 && (n & (n - 1)) == 0; }

hipError_t launch_low_velocity(const Mesh& m, const double* z, const double* w,
                               const LowBuffers& b, double* u, double* V, hipStream_t s)
{
    const int n1 = m.n1, n2 = m.n2, N = m.N;
    const int l1 = log2i(n1), l2 = log2i(n2);
    hipError_t e;
    hipLaunchKernelGGL(k_twiddle, dim3(grid_for(n1 > n2 ? n1 : n2)), dim3(kThreads), 0, s, n1,
                       b.tw1, n2, b.tw2);
    hipLaunchKernelGGL(k_lo_pack_rows, dim3(row_grid(n1, n2)), dim3(kFftThreads),
                       sizeof(double2) * n1, s, l1, n2, N, w, b.tw1, b.a);   // A[i2][m1]
    if ((e = transpose(b.a, b.b, n2, n1, s)) != hipSuccess) return e;       // B[m1][i2]
    hipLaunchKernelGGL(k_lo_symbol_rows, dim3(row_grid(n2, n1)), dim3(kFftThreads),
                       sizeof(double2) * n2, s, n1, l2, m.L1, m.L2, b.tw2, b.b);   // B[m1][i2]
    if ((e = transpose(b.b, b.a, n1, n2, s)) != hipSuccess) return e;       // A[i2][m1]
    double* S = reinterpret_cast<double*>(b.b);   // B is spent after the second transpose
    hipLaunchKernelGGL(k_lo_inv_rows, dim3(row_grid(n1, n2)), dim3(kFftThreads),
                       sizeof(double2) * n1, s, l1, n2, b.tw1, b.a, S);
    const int tx = n1 < 64 ? n1 : 64;
    const int ty = kThreads / tx < n2 ? kThreads / tx : n2;
    hipLaunchKernelGGL(k_lo_point, dim3(n1 / tx, (n2 + ty - 1) / ty), dim3(kThreads), 0, s, m, tx, ty,
                       S, z, w, u, V);
    return hipGetLastError();
}

}  // namespace zm
