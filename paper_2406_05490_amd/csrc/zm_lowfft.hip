// Low-order Z-Model velocity: the BR integral replaced by its flat-sheet
// approximation u = 1/2 (R1 w1 + R2 w2) n^, R_a the Riesz transform over
// the periodic parameter mesh (symbol i k_a / |k|), evaluated with FFTs
// (the paper's low-order solver, sec. 2).  One complex 2D FFT carries both
// real vorticity components (c = w1 + i w2), one inverse FFT returns S:
//
//   k_twiddle      exp(-2 pi i k / n), k < n/2, per axis
//   k_pack         c = w1 + i w2, rows = i2
//   k_fft_rows     radix-2 FFT of every row in LDS (bit-reversed load,
//                  in-place decimation-in-time stages)
//   k_transpose    32 x 32 tiles through LDS
//   k_riesz        S^ from c^(m) and conj(c^(-m)) (splits the two real
//                  fields), symbol, 1/N
//   k_low_velocity u = Re(S) n^ and V = A (|u|^2 - q/4 - 2 g z3) (u is not
//                  stored for the medium-order model, whose sheet moves with
//                  the BR velocity: there the FFT velocity only enters V)
//
// Layouts: forward  A[i2][i1] -> rows -> A[i2][m1] -> T -> B[m1][i2] -> rows
// -> B[m1][m2]; symbol B -> A[m1][m2]; inverse A -> rows -> A[m1][i2] -> T
// -> B[i2][m1] -> rows -> B[i2][i1] = S.  Sides are powers of two up to
// 4096 (one row of complex doubles fills at most 64 KiB of LDS).
#include "zm_device.h"
#include "zm_internal.h"

#include <hip/hip_runtime.h>

namespace zm {
namespace {

using dev::kThreads;

__global__ __launch_bounds__(kThreads) void k_twiddle(int n, double2* __restrict__ tw)
{
    const int k = blockIdx.x * kThreads + threadIdx.x;
    if (k >= n / 2) return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    tw[k] = make_double2(c, s);
}

__global__ __launch_bounds__(kThreads) void k_pack(int N, const double* __restrict__ w,
                                                   double2* __restrict__ a)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p < N) a[p] = make_double2(w[p], w[N + p]);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// One row of n = 2^logn complex values per workgroup, in place.  inv: use
// conj(twiddle) (unnormalised inverse).
template <bool INV>
__global__ __launch_bounds__(kThreads) void k_fft_rows(double2* __restrict__ a, int logn,
                                                       const double2* __restrict__ tw)
{
    extern __shared__ double2 x[];
    const int n = 1 << logn;
    double2* row = a + (size_t)blockIdx.x * n;
    for (int j = threadIdx.x; j < n; j += kThreads) {
        const int r = (int)(__brev((unsigned)j) >> (32 - logn));
        x[r] = row[j];
    }
    __syncthreads();
    for (int s = 1; s <= logn; ++s) {
        const int half = 1 << (s - 1);
        const int stride = n >> s;   // twiddle index step: exp(-2 pi i pos / 2^s)
        for (int b = threadIdx.x; b < n / 2; b += kThreads) {
            const int grp = b >> (s - 1), pos = b & (half - 1);
            const int i0 = (grp << s) + pos, i1 = i0 + half;
            double2 w = tw[pos * stride];
            if (INV) w.y = -w.y;
            const double2 u = x[i0], v = cmul(x[i1], w);
            x[i0] = make_double2(u.x + v.x, u.y + v.y);
            x[i1] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
    for (int j = threadIdx.x; j < n; j += kThreads) row[j] = x[j];
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

// b holds c^ as [m1][m2] (n1 rows of n2); writes S^ = (1/2) i (c1 w1^ +
// c2 w2^) / N into a, same layout, with w1^ = (c^(m) + conj(c^(-m))) / 2 and
// w2^ = (c^(m) - conj(c^(-m))) / (2 i); symbols c_a = k_a / |k| (zero at
// k = 0 and, along axis a, at the unpaired mode m_a = n_a / 2).
__global__ __launch_bounds__(kThreads) void k_riesz(int n1, int n2, double L1, double L2,
                                                    const double2* __restrict__ b,
                                                    double2* __restrict__ a)
{
    const int idx = blockIdx.x * kThreads + threadIdx.x;
    if (idx >= n1 * n2) return;
    const int m1 = idx / n2, m2 = idx - m1 * n2;
    const int s1 = 2 * m1 < n1 ? m1 : m1 - n1;
    const int s2 = 2 * m2 < n2 ? m2 : m2 - n2;
    const double k1 = 2.0 * M_PI * s1 / L1, k2 = 2.0 * M_PI * s2 / L2;
    const double kk = sqrt(k1 * k1 + k2 * k2);
    double c1 = 0.0, c2 = 0.0;
    if (kk > 0.0) {
        c1 = (2 * m1 == n1) ? 0.0 : k1 / kk;
        c2 = (2 * m2 == n2) ? 0.0 : k2 / kk;
    }
    const int q1 = m1 == 0 ? 0 : n1 - m1, q2 = m2 == 0 ? 0 : n2 - m2;
    const double2 c = b[idx];
    const double2 d = b[q1 * n2 + q2];
    // (i c1 (c + conj d) + c2 (c - conj d)) / (4 N)
    const double sx = c.x + d.x, sy = c.y - d.y;   // c + conj(d)
    const double tx = c.x - d.x, ty = c.y + d.y;   // c - conj(d)
    const double inv4n = 0.25 / ((double)n1 * (double)n2);
    a[idx] = make_double2((-c1 * sy + c2 * tx) * inv4n, (c1 * sx + c2 * ty) * inv4n);
}

__global__ __launch_bounds__(kThreads) void k_low_velocity(Mesh m, const double* __restrict__ z,
                                                           const double2* __restrict__ S,
                                                           const double* __restrict__ q,
                                                           double* __restrict__ u,
                                                           double* __restrict__ V)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= m.N) return;
    const int N = m.N;
    double T1[3], T2[3];
    dev::tangents_at(m, p, z, T1, T2);
    const double nx = T1[1] * T2[2] - T1[2] * T2[1];
    const double ny = T1[2] * T2[0] - T1[0] * T2[2];
    const double nz = T1[0] * T2[1] - T1[1] * T2[0];
    const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
    const double s = S[p].x;
    const double u1 = s * (nx * inv), u2 = s * (ny * inv), u3 = s * (nz * inv);
    if (u) {   // null for the medium-order model, which only needs V
        u[p] = u1;
        u[N + p] = u2;
        u[2 * N + p] = u3;
    }
    if (V) {
        const double uu = u1 * u1 + u2 * u2 + u3 * u3;
        V[p] = m.atwood * ((uu - 0.25 * q[p]) - (2.0 * m.gravity) * z[2 * N + p]);
    }
}

inline unsigned grid_for(long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

int log2i(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

hipError_t fft_rows(double2* a, int rows, int n, const double2* tw, bool inv, hipStream_t s)
{
    const int logn = log2i(n);
    const size_t lds = sizeof(double2) * (size_t)n;
    if (inv)
        hipLaunchKernelGGL(k_fft_rows<true>, dim3(rows), dim3(kThreads), lds, s, a, logn, tw);
    else
        hipLaunchKernelGGL(k_fft_rows<false>, dim3(rows), dim3(kThreads), lds, s, a, logn, tw);
    return hipGetLastError();
}

hipError_t transpose(const double2* in, double2* out, int rows, int cols, hipStream_t s)
{
    hipLaunchKernelGGL(k_transpose, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(kThreads), 0, s,
                       in, out, rows, cols);
    return hipGetLastError();
}

}  // namespace

bool low_order_supported_side(int n) { return n >= 8 && n <= 4096 && (n & (n - 1)) == 0; }

hipError_t launch_low_velocity(const Mesh& m, const double* z, const double* w, const double* q,
                               const LowBuffers& b, double* u, double* V, hipStream_t s)
{
    const int n1 = m.n1, n2 = m.n2, N = m.N;
    hipError_t e;
    hipLaunchKernelGGL(k_twiddle, dim3(grid_for(n1 / 2)), dim3(kThreads), 0, s, n1, b.tw1);
    hipLaunchKernelGGL(k_twiddle, dim3(grid_for(n2 / 2)), dim3(kThreads), 0, s, n2, b.tw2);
    hipLaunchKernelGGL(k_pack, dim3(grid_for(N)), dim3(kThreads), 0, s, N, w, b.a);
    if ((e = fft_rows(b.a, n2, n1, b.tw1, false, s)) != hipSuccess) return e;   // A[i2][m1]
    if ((e = transpose(b.a, b.b, n2, n1, s)) != hipSuccess) return e;          // B[m1][i2]
    if ((e = fft_rows(b.b, n1, n2, b.tw2, false, s)) != hipSuccess) return e;  // B[m1][m2]
    hipLaunchKernelGGL(k_riesz, dim3(grid_for(N)), dim3(kThreads), 0, s, n1, n2, m.L1, m.L2, b.b,
                       b.a);                                                    // A = S^[m1][m2]
    if ((e = fft_rows(b.a, n1, n2, b.tw2, true, s)) != hipSuccess) return e;   // A[m1][i2]
    if ((e = transpose(b.a, b.b, n1, n2, s)) != hipSuccess) return e;          // B[i2][m1]
    if ((e = fft_rows(b.b, n2, n1, b.tw1, true, s)) != hipSuccess) return e;   // B[i2][i1] = S
    hipLaunchKernelGGL(k_low_velocity, dim3(grid_for(N)), dim3(kThreads), 0, s, m, z, b.b, q, u, V);
    return hipGetLastError();
}

}  // namespace zm
