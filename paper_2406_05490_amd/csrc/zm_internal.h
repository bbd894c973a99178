// Internal interface between the host runtime (zm_api.hip) and the device
// kernels (zm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zm {

// Ints of the sheet's fold statistics (tangent-map bounds gathered by the
// surface kernel, read by the pair kernels and the cutoff solver).
constexpr int kFoldWords = 10;

// Cutoff solver counters: pairs tested, pairs accepted, and the paths that
// took the evaluations (bits, the same values as the public ZM_CUT_PATH_*).
constexpr int kCutCountWords = 3;
constexpr unsigned long long kCutPathCells = 1, kCutPathWindow = 2, kCutPathStencil = 4;

// Mesh geometry and model constants, passed by value to every kernel.
struct Mesh {
    int n1, n2;          // points per axis
    int N;               // n1 * n2
    int K;               // extra image layers
    double L1, L2;       // periods
    double h1, h2;       // spacings L_a / n_a
    double eps2;         // eps^2
    double coef;         // -(h1 h2) / (4 pi)
    double atwood, gravity, nu, dt;
    int periodic;        // 1: periodic sheet; 0: free (extrapolated ghosts, no images)
    int pad_;
};

// Launch shape of the all-pairs kernel.
struct PairShape {
    int R;               // targets per lane (register blocking)
    int cx;              // patch columns; 256 / cx thread rows
    int prow;            // patch rows = (256 / cx) * R
    int px, py;          // patches along axis 1 / axis 2
    int splits;          // source row ranges
    int rows_per_split;
};

// Shape for R targets per lane and `splits` source ranges (splits <= 0: the
// default of >= 2048 workgroups).  Supported R: 1, 2, 4.
PairShape make_pair_shape(int n1, int n2, int precision, int R, int splits);

// The untuned default shape for (n1, n2, precision).
PairShape default_pair_shape(int n1, int n2, int precision);

// Shape a new context or batch member uses: the process-wide tuning entry
// for (n1, n2, precision) if one is set, else the untuned default.
PairShape choose_pair_shape(int n1, int n2, int precision);

// Process-wide tuning table (zm_tune.hip).  Returns true and fills R and
// splits if (n1, n2, precision) has an entry.
bool lookup_tuning(int n1, int n2, int precision, int* R, int* splits);

// Each launcher enqueues one kernel on `s` and returns the launch status.

// Synthetic positions (3 planes) and source strengths (3 planes) for tuning.
hipError_t launch_tune_init(const Mesh& m, double* z, double* gam, hipStream_t s);
// fold (kFoldWords ints, zero before the first use; may be NULL): the
// sheet's tangent-map statistics, gathered by the surface kernel and turned
// by a one-thread kernel launched after it into the flag fold[4] the pair
// kernels read (1: use exact r for every pair) and the values the cutoff
// solver reads.  Two launches.
hipError_t launch_surface(const Mesh& m, const double* z, const double* w,
                          double* gam, double* q, int* fold, hipStream_t s);

// part[split][3][N] = unscaled sums over the split's sources of
// (r x gamma) / (|r|^2 + eps^2)^(3/2), images handled as described in zm.h
// with ties counted once at the image of offset -n_a/2.
// fold: the flag launch_surface left (NULL: the far forms are allowed).
hipError_t launch_pairs_f64(const Mesh& m, const PairShape& sh, const double* z,
                            const double* gam, double* part, const int* fold, hipStream_t s);

// Same contract, pair terms in FP32 with tile-relative coordinates and FP64
// per-target sums.
hipError_t launch_pairs_f32(const Mesh& m, const PairShape& sh, const double* z,
                            const double* gam, double* part, const int* fold, hipStream_t s);

// tie[pass][3][N]: pass 0 (n1 even) corrects the tie column, pass 1 (n2 even)
// the tie row, so that tied sources end with weight 1/2 per end image.
hipError_t launch_ties(const Mesh& m, const double* z, const double* gam, double* tie,
                       hipStream_t s);

// u = coef * (sum_s part[s] + ties); optionally V = A (|u|^2 - q/4 - 2 g z3).
// ties = false: no tie passes (the cutoff solver).
hipError_t launch_reduce(const Mesh& m, int splits, const double* part, const double* tie,
                         const double* q, const double* z, double* u, double* V,
                         hipStream_t s, bool ties = true);

// ---- cutoff solver (zm_cutoff.hip) ----------------------------------------

// Periodic cell grid of the cutoff solver.  Cells of side cw_a >= rc / m in
// x and y; targets are processed in blocks of B x B cells, each against the
// (B + 2m) x (B + 2m) cells around it, one row of those per workgroup, so a
// target gets B + 2m partial sums ("slots").  Sort key of cell (cx, cy):
// ((by nb1 + bx) B + ly) B + lx with (bx, lx) = divmod(cx, B), so the cells
// of a target block are contiguous.
struct CutGrid {
    int m;               // neighbour reach in cells
    int B;               // target block side in cells
    int nc1, nc2;        // cells per axis
    int nb1, nb2;        // target blocks per axis
    int nkeys;           // nb1 nb2 B^2
    int key_bits;        // bits of the sort key
    int slots;           // B + 2m (neighbour rows and columns of the cell path)
    int planes;          // partial sums per target: slots, or more for the index-window path
    int chunks;          // waves per (target block, row): ~ mean chunks of 64 tr targets per block
    int tr;              // targets per lane of the pair kernel
    int sort_blocks;     // workgroups of the radix-sort passes
    int periodic;        // 1: cells wrap with the period; 0 (free sheet): cells clamp to the box
    int pad_;
    double x0, y0;       // cell-grid origin (-L1/2, -L2/2)
    double L1, L2;
    double cw1, cw2;     // cell sides
    double rc2;          // rc * rc
    double iL1, iL2;     // 1 / L1, 1 / L2
};

CutGrid make_cut_grid(int n1, int n2, double L1, double L2, double rc, bool periodic);

// Device buffers of one cutoff evaluation (all in the caller's workspace).
struct CutBuffers {
    unsigned* keys[2];   // N each (radix-sort ping-pong)
    unsigned* vals[2];   // N each
    unsigned* hist;      // 256 * sort_blocks
    int* start;          // nkeys: first sorted index of a cell
    int* end;            // nkeys: one past the last
    int* bstart;         // nb1 nb2: first sorted index of a target block
    int* bend;
    double* src;         // 8 N: per sorted point (x, y, z, g1, g2, g3, kx, ky)
    int* kflag;          // nkeys: nonzero if a point of the cell has a wrap count != 0
    unsigned long long* counts;  // 2: pairs tested, pairs within rc
};

// Bin every point into its cell and sort the points by cell (stable), then
// gather positions, source strengths and wrap counts in sorted order.
// Returns the index of the buffer pair holding the sorted (key, point).
// fold: the sheet statistics of this evaluation (launch_surface); when they
// allow the index-window path (a periodic sheet whose horizontal map is
// one-to-one) these kernels leave at once and the records are written in
// index order instead.
hipError_t launch_cut_cells(const Mesh& m, const CutGrid& g, const double* z, const double* gam,
                            const CutBuffers& b, const int* fold, int* sorted_half, hipStream_t s);

// ---- low-order model (zm_lowfft.hip) ----------------------------------------

// Scratch of the FFT velocity: two N-point complex arrays, two twiddle tables.
struct LowBuffers {
    double2* a;
    double2* b;
    double2* tw1;        // n1: exp(-2 pi i t / n1)
    double2* tw2;        // n2
};

// Sides the FFT path handles: powers of two from 8 to 4096.
bool low_order_supported_side(int n);

// u (3 planes, if u != NULL) = 1/2 (R1 w1 + R2 w2) n^ and, if V != NULL,
// V = A (|u|^2 - q/4 - 2 g z3) with q = |w1 T2 - w2 T1|^2 / |T1 x T2|^2
// formed in place (no surface pass needed).
hipError_t launch_low_velocity(const Mesh& m, const double* z, const double* w,
                               const LowBuffers& b, double* u, double* V, hipStream_t s);

// Zero the two pair counters (a kernel, so it may sit in a captured graph).
hipError_t launch_cut_count_reset(unsigned long long* counts, hipStream_t s);

// part[slot][3][N] = unscaled cutoff sums per target and slot (neighbour row
// of the cell path, row group of the patch window, band group of the
// per-target stencil, which reads the z and gam planes directly).
// count != 0: also add the tested / accepted pair counts to b.counts.
hipError_t launch_cut_pairs(const Mesh& m, const CutGrid& g, const double* z, const double* gam,
                            const CutBuffers& b, int sorted_half, double* part, bool count,
                            const int* fold, hipStream_t s);

// F = (u, D V + nu Lap w) at state ys, then
//   stage 0: out = ys + dt F
//   stage 1: out = 3/4 y0 + 1/4 (ys + dt F)
//   stage 2: out = 1/3 y0 + 2/3 (ys + dt F)
//   stage 3: out = F (plain right-hand side; out_z / out_w are zt / wt)
// y0_z / ys_z / out_z: 3 planes, *_w: 2 planes.  out may alias y0 (read and
// written by the same thread), never ys.  nonfinite != NULL receives 1 if any
// output is not finite.
hipError_t launch_update(const Mesh& m, int stage, const double* y0_z, const double* y0_w,
                         const double* ys_z, const double* ys_w, const double* u, const double* V,
                         double* out_z, double* out_w, int* nonfinite, hipStream_t s);

}  // namespace zm
