/*
 * Z-Model high-order step: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never calls it and shares no code, header or constant
 * with it.
 *
 * What it computes (paper: Beatnik, Stewart & Bridges 2024):
 *   - SurfaceMesh state (sec. 2): per mesh point a position z = (z1,z2,z3)
 *     and two vorticity components w = (w1,w2) on a regular N1 x N2 mesh.
 *   - Two-node-deep stencils for tangents and Laplacians (sec. 3.1,
 *     SurfaceMesh) with periodic coordinate correction across the seam
 *     (sec. 3.1, BoundaryCondition), or, for a non-periodic sheet, values
 *     extrapolated into the boundary cells (same passage).
 *   - The Birkhoff-Rott velocity of every point from the position and
 *     vorticity of every other point (sec. 2, BRSolver), by brute-force
 *     all pairs (sec. 3.2.1, exact integral calculation), or restricted to
 *     the sources within a 3D cutoff distance of each target (sec. 3.2.2,
 *     cutoff-based approximate integral calculation); or, for the low-order
 *     model (sec. 2: the low-order solver approximates the BR integral with
 *     FFTs), the flat-sheet velocity 1/2 (R1 w1 + R2 w2) along the unit
 *     normal, R_a the Riesz transform over the periodic mesh.
 *   - The Z-Model derivatives of position and vorticity (sec. 2, ZModel)
 *     and a third-order Runge-Kutta step with three derivative evaluations
 *     (sec. 3.1, TimeIntegrator).
 * The paper prints no equations; the formulas below are the reading this
 * project fixes (vortex-sheet Biot-Savart law with algebraic
 * desingularisation, Bernoulli-type vorticity law, SSP-RK3).  Each function
 * states the definition it implements.
 *
 * Parity status of each function:
 *   zmo_tangents / zmo_laplacian : pinned (modified-wavenumber closed form,
 *                                  flat-grid identity, symmetry).
 *   zmo_br_velocity             : pinned (flat-sheet eigenvalue -> -|k|/2,
 *                                  linear Rayleigh-Taylor growth rate,
 *                                  mirror / translation invariants,
 *                                  high-precision brute force).
 *   zmo_rhs (linear part)       : pinned by the linear growth rate.
 *   zmo_rhs (|u|^2 and q/4 terms of the Bernoulli potential): the identity
 *                                  q = g^{ab} w_a w_b is pinned, and so is the
 *                                  formula as implemented (high-order
 *                                  flat-sheet closed form of w_t, which a
 *                                  dropped |u|^2 or a wrong q coefficient
 *                                  fails); the choice to keep |u|^2 and drop
 *                                  the mean-potential time derivative is a
 *                                  reading of the model that no value from
 *                                  the paper fixes -- parity unpinned.
 *   zmo_rk3_step                : pinned (amplification factor, order 3).
 *   cutoff BR (cutoff > 0)      : pinned (flat-sheet lattice-sum eigenvalue
 *                                  over the disc |rho| < rc, brute force,
 *                                  symmetries, convergence to the exact sum).
 *   free boundary (boundary 1)  : pinned (extrapolated stencils exact on
 *                                  cubics, free-space brute force, rigid
 *                                  translation and reflection symmetries;
 *                                  with a cutoff: the exact free sum once rc
 *                                  exceeds the sheet's diameter, brute-force
 *                                  pair counts).
 *   medium order (model 2)      : built from pinned parts (z_t is the
 *                                  high-order one, w_t the low-order one,
 *                                  bitwise); which velocity enters where is
 *                                  a reading of the paper -- parity
 *                                  unpinned for the coupling itself.
 *   low-order velocity (model 1): pinned (flat-sheet symbol -|k|/2 exactly,
 *                                  a library FFT on random fields, the
 *                                  Nyquist rule, the linear growth rate
 *                                  A g (k . k~) / |k| through RK3).
 *
 * Arithmetic: plain double, 1.0/sqrt(s), Neumaier-compensated per-target
 * sums in a fixed sequential source order, no FMA contraction (build with
 * -ffp-contract=off).  Targets are split over OpenMP threads; the result
 * does not depend on the thread count.
 *
 * Layout: structure-of-arrays planes.  Point index p = i2*n1 + i1.
 * z has 3 planes (z[c*N + p]), w has 2 planes, velocities 3 planes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct {
    int32_t n1, n2;          /* mesh points along alpha_1, alpha_2           */
    int32_t images;          /* K >= 0 extra periodic image layers           */
    int32_t model;           /* 0: high order (BR sum), 1: low order (FFT),
                                2: medium order (BR moves the sheet, the FFT
                                velocity drives the vorticity)              */
    double period1, period2; /* L1, L2 (parameter and x/y period)            */
    double atwood;           /* A                                            */
    double gravity;          /* g (gravity is -g e3)                         */
    double eps;              /* desingularisation length                     */
    double nu;               /* optional artificial viscosity on w           */
    double dt;               /* time step                                    */
    double cutoff;           /* > 0: cutoff BR solver with this 3D distance  */
    int32_t boundary;        /* 0: periodic, 1: free (non-periodic sheet)    */
    int32_t pad_;
} zmo_problem;

/* ------------------------------------------------------------------ */
/* helpers                                                             */
/* ------------------------------------------------------------------ */

static int wrap_index(int i, int n, int *wraps)
{
    int w = 0;
    while (i < 0) { i += n; w -= 1; }
    while (i >= n) { i -= n; w += 1; }
    *wraps = w;
    return i;
}

/* Free boundary: ghost value at index i (i = -2, -1 or n, n+1) of a line
 * g(0..n-1) by cubic extrapolation from the four nearest points (the fourth
 * difference across the boundary vanishes):
 *   g(-1) = 4 g0 - 6 g1 + 4 g2 - g3,  g(-2) = 10 g0 - 20 g1 + 15 g2 - 4 g3,
 * and the mirror images at the far end. */
static double ghost(const double *base, size_t stride, int n, int i)
{
    if (i < 0) {
        const double g0 = base[0], g1 = base[stride], g2 = base[2 * stride], g3 = base[3 * stride];
        return i == -1 ? 4.0 * g0 - 6.0 * g1 + 4.0 * g2 - g3
                       : 10.0 * g0 - 20.0 * g1 + 15.0 * g2 - 4.0 * g3;
    }
    const double g0 = base[(size_t)(n - 1) * stride], g1 = base[(size_t)(n - 2) * stride];
    const double g2 = base[(size_t)(n - 3) * stride], g3 = base[(size_t)(n - 4) * stride];
    return i == n ? 4.0 * g0 - 6.0 * g1 + 4.0 * g2 - g3
                  : 10.0 * g0 - 20.0 * g1 + 15.0 * g2 - 4.0 * g3;
}

/* A plane (or one position component) at a possibly out-of-range index on
 * a free-boundary mesh: in range as stored, else extrapolated along the
 * axis that is out of range (5-point stencils leave one axis at a time). */
static double free_at(const zmo_problem *P, const double *f, int i1, int i2)
{
    const int n1 = P->n1, n2 = P->n2;
    if (i1 < 0 || i1 >= n1) return ghost(f + (size_t)i2 * n1, 1, n1, i1);
    if (i2 < 0 || i2 >= n2) return ghost(f + i1, (size_t)n1, n2, i2);
    return f[(size_t)i2 * n1 + i1];
}

/* Position component c at (possibly out-of-range) mesh index (i1,i2):
 * periodic in the index; z1 gains +-L1 per wrap along alpha_1, z2 gains
 * +-L2 per wrap along alpha_2 (the periodic coordinate correction);
 * z3 is plainly periodic.  Free boundary: extrapolated ghosts. */
static double z_at(const zmo_problem *P, const double *z, int c, int i1, int i2)
{
    const int n1 = P->n1, n2 = P->n2;
    if (P->boundary == 1) return free_at(P, z + (size_t)c * n1 * n2, i1, i2);
    int w1, w2;
    int j1 = wrap_index(i1, n1, &w1);
    int j2 = wrap_index(i2, n2, &w2);
    double v = z[(size_t)c * n1 * n2 + (size_t)j2 * n1 + j1];
    if (c == 0 && w1 != 0) v = v + (double)w1 * P->period1;
    if (c == 1 && w2 != 0) v = v + (double)w2 * P->period2;
    return v;
}

/* A periodic scalar plane at a possibly out-of-range index (free boundary:
 * extrapolated ghosts). */
static double f_at(const zmo_problem *P, const double *f, int i1, int i2)
{
    if (P->boundary == 1) return free_at(P, f, i1, i2);
    int w1, w2;
    int j1 = wrap_index(i1, P->n1, &w1);
    int j2 = wrap_index(i2, P->n2, &w2);
    (void)w1; (void)w2;
    return f[(size_t)j2 * P->n1 + j1];
}

/* Fourth-order central first difference from the four neighbours:
 * D f = [8 (f(+1) - f(-1)) - (f(+2) - f(-2))] / (12 h). */
static double d1_5pt(double fm2, double fm1, double fp1, double fp2, double h)
{
    return (8.0 * (fp1 - fm1) - (fp2 - fm2)) / (12.0 * h);
}

/* Fourth-order central second difference:
 * D2 f = [-f(+2) + 16 f(+1) - 30 f(0) + 16 f(-1) - f(-2)] / (12 h^2). */
static double d2_5pt(double fm2, double fm1, double f0, double fp1, double fp2, double h)
{
    return (-fp2 + 16.0 * fp1 - 30.0 * f0 + 16.0 * fm1 - fm2) / (12.0 * h * h);
}

typedef struct { double s, c; } neumaier;

static void nm_add(neumaier *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}

static double nm_value(const neumaier *a) { return a->s + a->c; }

static int set_threads(int nthreads)
{
    if (nthreads > 0) return nthreads;
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------ */
/* surface derivatives                                                 */
/* ------------------------------------------------------------------ */

/* Tangents T_a = dz/d(alpha_a) by the 5-point fourth-order stencil with the
 * periodic coordinate correction.  t1, t2: 3 planes each. */
void zmo_tangents(const zmo_problem *P, const double *z, double *t1, double *t2)
{
    const int n1 = P->n1, n2 = P->n2;
    const size_t N = (size_t)n1 * n2;
    const double h1 = P->period1 / n1, h2 = P->period2 / n2;
    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < n1; ++i1) {
            size_t p = (size_t)i2 * n1 + i1;
            for (int c = 0; c < 3; ++c) {
                t1[c * N + p] = d1_5pt(z_at(P, z, c, i1 - 2, i2), z_at(P, z, c, i1 - 1, i2),
                                       z_at(P, z, c, i1 + 1, i2), z_at(P, z, c, i1 + 2, i2), h1);
                t2[c * N + p] = d1_5pt(z_at(P, z, c, i1, i2 - 2), z_at(P, z, c, i1, i2 - 1),
                                       z_at(P, z, c, i1, i2 + 1), z_at(P, z, c, i1, i2 + 2), h2);
            }
        }
}

/* Surface quantities: tangents, the BR source strength
 * gamma = w1 T2 - w2 T1 (3 planes), and q = |gamma|^2 / |T1 x T2|^2,
 * the squared jump of tangential velocity across the sheet. */
void zmo_surface(const zmo_problem *P, const double *z, const double *w,
                 double *t1, double *t2, double *gamma, double *q)
{
    const size_t N = (size_t)P->n1 * P->n2;
    zmo_tangents(P, z, t1, t2);
    for (size_t p = 0; p < N; ++p) {
        double a1 = t1[p], a2 = t1[N + p], a3 = t1[2 * N + p];
        double b1 = t2[p], b2 = t2[N + p], b3 = t2[2 * N + p];
        double w1 = w[p], w2 = w[N + p];
        double g1 = w1 * b1 - w2 * a1;
        double g2 = w1 * b2 - w2 * a2;
        double g3 = w1 * b3 - w2 * a3;
        gamma[p] = g1; gamma[N + p] = g2; gamma[2 * N + p] = g3;
        double n1 = a2 * b3 - a3 * b2;
        double n2 = a3 * b1 - a1 * b3;
        double n3 = a1 * b2 - a2 * b1;
        q[p] = (g1 * g1 + g2 * g2 + g3 * g3) / (n1 * n1 + n2 * n2 + n3 * n3);
    }
}

/* Laplacian in the mesh parameters, sum over both axes of the fourth-order
 * second difference; f is one periodic plane. */
void zmo_laplacian(const zmo_problem *P, const double *f, double *out)
{
    const int n1 = P->n1, n2 = P->n2;
    const double h1 = P->period1 / n1, h2 = P->period2 / n2;
    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < n1; ++i1) {
            double a = d2_5pt(f_at(P, f, i1 - 2, i2), f_at(P, f, i1 - 1, i2), f_at(P, f, i1, i2),
                              f_at(P, f, i1 + 1, i2), f_at(P, f, i1 + 2, i2), h1);
            double b = d2_5pt(f_at(P, f, i1, i2 - 2), f_at(P, f, i1, i2 - 1), f_at(P, f, i1, i2),
                              f_at(P, f, i1, i2 + 1), f_at(P, f, i1, i2 + 2), h2);
            out[(size_t)i2 * n1 + i1] = a + b;
        }
}

/* ------------------------------------------------------------------ */
/* Birkhoff-Rott velocity                                              */
/* ------------------------------------------------------------------ */

/* Images of source index j seen from target index i along one axis with n
 * points: the offset o = j - i reduced modulo n to the cell centred on the
 * target.  Writes the image shifts (in periods, source moves by +s*L) and
 * their weights; returns how many (1, or 2 when |o| = n/2 exactly, which
 * only happens for even n: the two end images share weight 1/2 -- the
 * trapezoid rule over the period cell centred on the target). */
static int axis_images(int i, int j, int n, int shift[2], double weight[2])
{
    if (n < 0) {               /* free boundary (caller passes -n): no images */
        shift[0] = 0;
        weight[0] = 1.0;
        return 1;
    }
    int d = ((j - i) % n + n) % n;   /* in [0, n) */
    if (2 * d < n) {                 /* o = d */
        shift[0] = (i + d - j) / n;
        weight[0] = 1.0;
        return 1;
    }
    if (2 * d > n) {                 /* o = d - n */
        shift[0] = (i + d - n - j) / n;
        weight[0] = 1.0;
        return 1;
    }
    shift[0] = (i + d - j) / n;      /* o = +n/2 */
    shift[1] = (i + d - n - j) / n;  /* o = -n/2 */
    weight[0] = 0.5;
    weight[1] = 0.5;
    return 2;
}

/* One target: u = -(h1 h2 / 4 pi) sum_j sum_images c * (r x gamma_j) /
 * (|r|^2 + eps^2)^(3/2), r = z_i - z_j - (S1 L1, S2 L2, 0).  Sources are
 * visited in index order p_j = j2*n1 + j1; for each source the images are
 * visited in the order (extra layer m2, m1 from -K..K) x (axis-2 image,
 * axis-1 image). */
static void br_one_target(const zmo_problem *P, const double *z, const double *gamma,
                          int i1, int i2, double coef, double out[3])
{
    const int n1 = P->n1, n2 = P->n2, K = P->images;
    const size_t N = (size_t)n1 * n2;
    const double L1 = P->period1, L2 = P->period2;
    const double eps2 = P->eps * P->eps;
    const size_t pi_ = (size_t)i2 * n1 + i1;
    const double zi1 = z[pi_], zi2 = z[N + pi_], zi3 = z[2 * N + pi_];
    neumaier a1 = {0, 0}, a2 = {0, 0}, a3 = {0, 0};

    for (int j2 = 0; j2 < n2; ++j2) {
        int s2[2]; double c2[2];
        int k2 = axis_images(i2, j2, P->boundary == 1 ? -n2 : n2, s2, c2);
        for (int j1 = 0; j1 < n1; ++j1) {
            int s1[2]; double c1[2];
            int k1 = axis_images(i1, j1, P->boundary == 1 ? -n1 : n1, s1, c1);
            const size_t pj = (size_t)j2 * n1 + j1;
            const double zj1 = z[pj], zj2 = z[N + pj], zj3 = z[2 * N + pj];
            const double g1 = gamma[pj], g2 = gamma[N + pj], g3 = gamma[2 * N + pj];
            for (int m2 = -K; m2 <= K; ++m2)
                for (int m1 = -K; m1 <= K; ++m1)
                    for (int b = 0; b < k2; ++b)
                        for (int a = 0; a < k1; ++a) {
                            double c = c1[a] * c2[b];
                            double S1 = (double)(s1[a] + m1), S2 = (double)(s2[b] + m2);
                            double r1 = zi1 - zj1 - S1 * L1;
                            double r2 = zi2 - zj2 - S2 * L2;
                            double r3 = zi3 - zj3;
                            double s = r1 * r1 + r2 * r2 + r3 * r3 + eps2;
                            double inv = 1.0 / sqrt(s);
                            double wgt = inv * inv * inv;
                            double x1 = r2 * g3 - r3 * g2;
                            double x2 = r3 * g1 - r1 * g3;
                            double x3 = r1 * g2 - r2 * g1;
                            double f = c * wgt;
                            nm_add(&a1, f * x1);
                            nm_add(&a2, f * x2);
                            nm_add(&a3, f * x3);
                        }
        }
    }
    out[0] = coef * nm_value(&a1);
    out[1] = coef * nm_value(&a2);
    out[2] = coef * nm_value(&a3);
}

/* Cutoff BR, one target: the same kernel summed only over the sources whose
 * nearest periodic image lies within the 3D distance rc of the target.  Per
 * axis a = 1, 2 the image shift is the integer S_a nearest to
 * (z_i,a - z_j,a) / L_a; with r = (z_i - z_j) - (S1 L1, S2 L2, 0), written
 * out as r_a = (z_i,a - z_j,a) - S_a L_a, the source counts (weight 1) iff
 * r1*r1 + r2*r2 + r3*r3 < rc*rc, evaluated left to right in plain double.
 * rc <= 0.45 min(L1, L2), so at most one image of a source can be that
 * close and a source (nearly) half a period away along an axis never is.  Sources in index
 * order; no extra image layers.  Free sheet (boundary 1): no images, S = 0,
 * r = z_i - z_j, and any rc > 0. */
static void br_cutoff_one_target(const zmo_problem *P, const double *z, const double *gamma,
                                 int i1, int i2, double coef, double out[3])
{
    const int n1 = P->n1, n2 = P->n2;
    const size_t N = (size_t)n1 * n2;
    const double L1 = P->period1, L2 = P->period2;
    const double eps_sq = P->eps * P->eps;
    const double rc2 = P->cutoff * P->cutoff;
    const int free_sheet = P->boundary == 1;
    const size_t pi_ = (size_t)i2 * n1 + i1;
    const double zi1 = z[pi_], zi2 = z[N + pi_], zi3 = z[2 * N + pi_];
    neumaier a1 = {0, 0}, a2 = {0, 0}, a3 = {0, 0};

    for (size_t pj = 0; pj < N; ++pj) {
        const double d1 = zi1 - z[pj], d2 = zi2 - z[N + pj];
        const double S1 = free_sheet ? 0.0 : nearbyint(d1 / L1);
        const double S2 = free_sheet ? 0.0 : nearbyint(d2 / L2);
        const double r1 = d1 - S1 * L1;
        const double r2 = d2 - S2 * L2;
        const double r3 = zi3 - z[2 * N + pj];
        const double dd = r1 * r1 + r2 * r2 + r3 * r3;
        if (!(dd < rc2)) continue;
        const double g1 = gamma[pj], g2 = gamma[N + pj], g3 = gamma[2 * N + pj];
        const double inv = 1.0 / sqrt(dd + eps_sq);
        const double kw = inv * inv * inv;
        nm_add(&a1, kw * (r2 * g3 - r3 * g2));
        nm_add(&a2, kw * (r3 * g1 - r1 * g3));
        nm_add(&a3, kw * (r1 * g2 - r2 * g1));
    }
    out[0] = coef * nm_value(&a1);
    out[1] = coef * nm_value(&a2);
    out[2] = coef * nm_value(&a3);
}

static int low_order_velocity(const zmo_problem *P, const double *z, const double *w, double *u);

/* BR velocity of the listed targets (point indices), or of all points when
 * targets == NULL.  u: 3 planes of length ntargets (or N).  gamma is the
 * source strength from zmo_surface.  Returns 0, or -1 on bad arguments. */
int zmo_br_from_gamma(const zmo_problem *P, const double *z, const double *gamma,
                      int64_t ntargets, const int64_t *targets, double *u, int nthreads)
{
    if (!P || P->n1 < 1 || P->n2 < 1 || !(P->eps > 0.0) || P->images < 0) return -1;
    if (P->cutoff < 0.0 || (P->cutoff > 0.0 && (P->images != 0 ||
                                               (P->boundary == 0 && (P->cutoff > 0.45 * P->period1 ||
                                                                     P->cutoff > 0.45 * P->period2)))))
        return -1;
    if (P->boundary != 0 && (P->boundary != 1 || P->images != 0 || P->n1 < 4 || P->n2 < 4))
        return -1;
    const size_t N = (size_t)P->n1 * P->n2;
    const int64_t nt = targets ? ntargets : (int64_t)N;
    const double h1 = P->period1 / P->n1, h2 = P->period2 / P->n2;
    const double coef = -(h1 * h2) / (4.0 * M_PI);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(set_threads(nthreads)) reduction(|:bad)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t p = targets ? targets[t] : t;
        if (p < 0 || (size_t)p >= N) { bad = 1; continue; }
        double o[3];
        if (P->cutoff > 0.0)
            br_cutoff_one_target(P, z, gamma, (int)(p % P->n1), (int)(p / P->n1), coef, o);
        else
            br_one_target(P, z, gamma, (int)(p % P->n1), (int)(p / P->n1), coef, o);
        u[t] = o[0];
        u[nt + t] = o[1];
        u[2 * nt + t] = o[2];
    }
    return bad ? -1 : 0;
}

/* The velocity that moves the sheet: the BR sum for the high- and
 * medium-order models, the flat-sheet FFT velocity for the low-order one. */
int zmo_br_velocity(const zmo_problem *P, const double *z, const double *w,
                    int64_t ntargets, const int64_t *targets, double *u, int nthreads)
{
    if (!P || P->n1 < 1 || P->n2 < 1) return -1;
    if (P->model == 1) {   /* low order: every point, no sampling */
        if (targets || P->cutoff != 0.0 || P->images != 0 || P->boundary != 0) return -1;
        (void)set_threads(nthreads);
        return low_order_velocity(P, z, w, u);
    }
    if (P->model != 0 && !(P->model == 2 && P->boundary == 0)) return -1;
    const size_t N = (size_t)P->n1 * P->n2;
    double *buf = (double *)malloc(sizeof(double) * 10 * N);
    if (!buf) return -1;
    double *t1 = buf, *t2 = buf + 3 * N, *gamma = buf + 6 * N, *q = buf + 9 * N;
    zmo_surface(P, z, w, t1, t2, gamma, q);
    int rc = zmo_br_from_gamma(P, z, gamma, ntargets, targets, u, nthreads);
    free(buf);
    return rc;
}

/* ------------------------------------------------------------------ */
/* low-order velocity                                                  */
/* ------------------------------------------------------------------ */

/* Signed mode number of DFT index m on an n-point axis: m for m < n/2,
 * m - n above; *nyq = 1 for the unpaired mode m = n/2 of an even n. */
static int signed_mode(int m, int n, int *nyq)
{
    *nyq = (2 * m == n);
    return 2 * m < n ? m : m - n;
}

/* Low-order velocity u = S n^ with S = 1/2 (R1 w1 + R2 w2): the Riesz
 * transforms R_a act on the mode exp(i k.alpha) as i k_a / |k|, with
 * k_a = 2 pi m_a / L_a (m_a signed), 0 for k = 0 and, along axis a, 0 at
 * the unpaired mode m_a = n_a/2 of an even n_a (a real field cannot carry
 * i k_a there).  n^ = (T1 x T2) / |T1 x T2|.  Plain double sums: forward
 * DFT w^_a(m) = (1/N) sum_j w_a(j) exp(-2 pi i (m1 j1/n1 + m2 j2/n2)),
 * then S(i) = Re sum_m S^(m) exp(+2 pi i (m1 i1/n1 + m2 i2/n2)). */
static int low_order_velocity(const zmo_problem *P, const double *z, const double *w, double *u)
{
    const int n1 = P->n1, n2 = P->n2;
    const size_t N = (size_t)n1 * n2;
    double *buf = (double *)malloc(sizeof(double) * (6 * N + 3 * N));
    if (!buf) return -1;
    double *t1 = buf, *t2 = buf + 3 * N, *sre = buf + 6 * N, *sim = buf + 7 * N, *S = buf + 8 * N;
    zmo_tangents(P, z, t1, t2);
    /* S^ on every mode */
#pragma omp parallel for schedule(static)
    for (size_t mm = 0; mm < N; ++mm) {
        const int m1 = (int)(mm % n1), m2 = (int)(mm / n1);
        int nyq1, nyq2;
        const int s1 = signed_mode(m1, n1, &nyq1), s2 = signed_mode(m2, n2, &nyq2);
        const double k1 = 2.0 * M_PI * s1 / P->period1, k2 = 2.0 * M_PI * s2 / P->period2;
        const double kk = sqrt(k1 * k1 + k2 * k2);
        double c1 = 0.0, c2 = 0.0;   /* symbols divided by i */
        if (kk > 0.0) {
            c1 = nyq1 ? 0.0 : k1 / kk;
            c2 = nyq2 ? 0.0 : k2 / kk;
        }
        neumaier ar = {0, 0}, ai = {0, 0};
        for (int j2 = 0; j2 < n2; ++j2)
            for (int j1 = 0; j1 < n1; ++j1) {
                const size_t pj = (size_t)j2 * n1 + j1;
                /* phase in turns, reduced exactly in integers */
                const double ph = (double)((long)m1 * j1 % n1) / n1 + (double)((long)m2 * j2 % n2) / n2;
                const double c = cos(2.0 * M_PI * ph), sn = sin(2.0 * M_PI * ph);
                /* (1/2) i (c1 w1 + c2 w2) exp(-i 2 pi ph) */
                const double f = 0.5 * (c1 * w[pj] + c2 * w[N + pj]);
                nm_add(&ar, f * sn);    /* Re(i f (c - i sn)) = f sn */
                nm_add(&ai, f * c);     /* Im(i f (c - i sn)) = f c  */
            }
        sre[mm] = nm_value(&ar) / (double)N;
        sim[mm] = nm_value(&ai) / (double)N;
    }
    /* inverse DFT, real part */
#pragma omp parallel for schedule(static)
    for (size_t pi_ = 0; pi_ < N; ++pi_) {
        const int i1 = (int)(pi_ % n1), i2 = (int)(pi_ / n1);
        neumaier a = {0, 0};
        for (int m2 = 0; m2 < n2; ++m2)
            for (int m1 = 0; m1 < n1; ++m1) {
                const size_t mm = (size_t)m2 * n1 + m1;
                const double ph = (double)((long)m1 * i1 % n1) / n1 + (double)((long)m2 * i2 % n2) / n2;
                /* Re((sre + i sim)(c + i sn)) */
                nm_add(&a, sre[mm] * cos(2.0 * M_PI * ph) - sim[mm] * sin(2.0 * M_PI * ph));
            }
        S[pi_] = nm_value(&a);
    }
    for (size_t p = 0; p < N; ++p) {
        const double a1 = t1[p], a2 = t1[N + p], a3 = t1[2 * N + p];
        const double b1 = t2[p], b2 = t2[N + p], b3 = t2[2 * N + p];
        const double nx = a2 * b3 - a3 * b2, ny = a3 * b1 - a1 * b3, nz = a1 * b2 - a2 * b1;
        const double inv = 1.0 / sqrt(nx * nx + ny * ny + nz * nz);
        u[p] = S[p] * (nx * inv);
        u[N + p] = S[p] * (ny * inv);
        u[2 * N + p] = S[p] * (nz * inv);
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Z-Model right-hand side                                             */
/* ------------------------------------------------------------------ */

/* Bernoulli-type potential V = A (|u|^2 - q/4 - 2 g z3). */
static double bernoulli(const zmo_problem *P, double u1, double u2, double u3, double q, double z3)
{
    double uu = u1 * u1 + u2 * u2 + u3 * u3;
    return P->atwood * ((uu - 0.25 * q) - (2.0 * P->gravity) * z3);
}

/* F(z, w) = (z_t, w_t) with z_t = u (BR velocity) and
 * w_t = (D1 V, D2 V) + nu * Lap(w).  zt: 3 planes, wt: 2 planes.
 * Low order: u is the flat-sheet FFT velocity throughout.  Medium order
 * (sec. 2: it couples the FFT solver with the far-field BR solver; sec. 6:
 * it uses the FFTs for the change in vorticity; periodic sheets only, as the
 * FFT is): z_t is the BR velocity (exact or cutoff) and the |u|^2 of V is
 * that of the FFT velocity. */
int zmo_rhs(const zmo_problem *P, const double *z, const double *w,
            double *zt, double *wt, int nthreads)
{
    if (!P || P->n1 < 1 || P->n2 < 1) return -1;
    const int n1 = P->n1, n2 = P->n2;
    const size_t N = (size_t)n1 * n2;
    const double h1 = P->period1 / n1, h2 = P->period2 / n2;
    double *buf = (double *)malloc(sizeof(double) * 16 * N);
    if (!buf) return -1;
    double *t1 = buf, *t2 = buf + 3 * N, *gamma = buf + 6 * N, *q = buf + 9 * N;
    double *V = buf + 10 * N, *lap = buf + 11 * N, *ulo = buf + 13 * N;
    zmo_surface(P, z, w, t1, t2, gamma, q);
    int rc;
    const double *uv = zt;   /* the velocity in V */
    if (P->model == 1) {
        if (P->cutoff != 0.0 || P->images != 0 || P->boundary != 0) { free(buf); return -1; }
        (void)set_threads(nthreads);
        rc = low_order_velocity(P, z, w, zt);
    } else if (P->model == 2) {
        if (P->boundary != 0) { free(buf); return -1; }
        rc = zmo_br_from_gamma(P, z, gamma, 0, NULL, zt, nthreads);
        if (!rc) {
            (void)set_threads(nthreads);
            rc = low_order_velocity(P, z, w, ulo);
        }
        uv = ulo;
    } else {
        rc = P->model == 0 ? zmo_br_from_gamma(P, z, gamma, 0, NULL, zt, nthreads) : -1;
    }
    if (rc) { free(buf); return rc; }
    for (size_t p = 0; p < N; ++p)
        V[p] = bernoulli(P, uv[p], uv[N + p], uv[2 * N + p], q[p], z[2 * N + p]);
    for (int i2 = 0; i2 < n2; ++i2)
        for (int i1 = 0; i1 < n1; ++i1) {
            size_t p = (size_t)i2 * n1 + i1;
            wt[p] = d1_5pt(f_at(P, V, i1 - 2, i2), f_at(P, V, i1 - 1, i2),
                           f_at(P, V, i1 + 1, i2), f_at(P, V, i1 + 2, i2), h1);
            wt[N + p] = d1_5pt(f_at(P, V, i1, i2 - 2), f_at(P, V, i1, i2 - 1),
                               f_at(P, V, i1, i2 + 1), f_at(P, V, i1, i2 + 2), h2);
        }
    if (P->nu != 0.0) {
        for (int c = 0; c < 2; ++c) {
            zmo_laplacian(P, w + c * N, lap);
            for (size_t p = 0; p < N; ++p) wt[c * N + p] = wt[c * N + p] + P->nu * lap[p];
        }
    }
    free(buf);
    return 0;
}

/* The 9 points the vorticity derivative at a target reads: 0 the centre,
 * 1..4 axis-1 offsets -2,-1,+1,+2, 5..8 the same along axis 2. */
static const int stencil_off1[9] = {0, -2, -1, 1, 2, 0, 0, 0, 0};
static const int stencil_off2[9] = {0, 0, 0, 0, 0, -2, -1, 1, 2};

/* wt[c * ntargets + t] = D_c V + nu Lap(w_c) at point index p, from V at the
 * 9 stencil points (centred fourth-order differences, as zmo_rhs takes). */
static void wt_from_stencil(const zmo_problem *P, const double *w, const double V[9],
                            int64_t p, int64_t ntargets, int64_t t, double *wt)
{
    const int n1 = P->n1;
    const size_t N = (size_t)n1 * P->n2;
    const double h1 = P->period1 / n1, h2 = P->period2 / P->n2;
    wt[t] = d1_5pt(V[1], V[2], V[3], V[4], h1);
    wt[ntargets + t] = d1_5pt(V[5], V[6], V[7], V[8], h2);
    if (P->nu != 0.0) {
        const int i1 = (int)(p % n1), i2 = (int)(p / n1);
        for (int c = 0; c < 2; ++c) {
            const double *f = w + c * N;
            double lap = d2_5pt(f_at(P, f, i1 - 2, i2), f_at(P, f, i1 - 1, i2), f_at(P, f, i1, i2),
                                f_at(P, f, i1 + 1, i2), f_at(P, f, i1 + 2, i2), h1)
                       + d2_5pt(f_at(P, f, i1, i2 - 2), f_at(P, f, i1, i2 - 1), f_at(P, f, i1, i2),
                                f_at(P, f, i1, i2 + 1), f_at(P, f, i1, i2 + 2), h2);
            wt[c * ntargets + t] = wt[c * ntargets + t] + P->nu * lap;
        }
    }
}

/* F at listed targets only.  The BR velocity is evaluated at each target and
 * at its +-1, +-2 stencil neighbours along both axes (V is needed there).
 * zt: 3 planes of length ntargets, wt: 2 planes of length ntargets. */
int zmo_rhs_sampled(const zmo_problem *P, const double *z, const double *w,
                    int64_t ntargets, const int64_t *targets,
                    double *zt, double *wt, int nthreads)
{
    if (!P || P->n1 < 1 || P->n2 < 1 || ntargets < 0 || !targets || P->model != 0 ||
        P->boundary != 0)
        return -1;
    const int n1 = P->n1, n2 = P->n2;
    const size_t N = (size_t)n1 * n2;
    for (int64_t t = 0; t < ntargets; ++t)
        if (targets[t] < 0 || (size_t)targets[t] >= N) return -1;
    const int64_t ns = 9 * ntargets;
    int64_t *pts = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    double *us = (double *)malloc(sizeof(double) * 3 * (size_t)(ns > 0 ? ns : 1));
    double *buf = (double *)malloc(sizeof(double) * 10 * N);
    if (!pts || !us || !buf) { free(pts); free(us); free(buf); return -1; }
    for (int64_t t = 0; t < ntargets; ++t) {
        int i1 = (int)(targets[t] % n1), i2 = (int)(targets[t] / n1);
        for (int k = 0; k < 9; ++k) {
            int w1, w2;
            int j1 = wrap_index(i1 + stencil_off1[k], n1, &w1);
            int j2 = wrap_index(i2 + stencil_off2[k], n2, &w2);
            pts[9 * t + k] = (int64_t)j2 * n1 + j1;
        }
    }
    double *t1 = buf, *t2 = buf + 3 * N, *gamma = buf + 6 * N, *q = buf + 9 * N;
    zmo_surface(P, z, w, t1, t2, gamma, q);
    int rc = zmo_br_from_gamma(P, z, gamma, ns, pts, us, nthreads);
    if (rc) { free(pts); free(us); free(buf); return rc; }
    for (int64_t t = 0; t < ntargets; ++t) {
        double V[9];
        for (int k = 0; k < 9; ++k) {
            int64_t s = 9 * t + k, p = pts[s];
            V[k] = bernoulli(P, us[s], us[ns + s], us[2 * ns + s], q[p], z[2 * N + p]);
        }
        int64_t s0 = 9 * t;
        zt[t] = us[s0];
        zt[ntargets + t] = us[ns + s0];
        zt[2 * ntargets + t] = us[2 * ns + s0];
        wt_from_stencil(P, w, V, targets[t], ntargets, t, wt);
    }
    free(pts); free(us); free(buf);
    return 0;
}

/* w_t = (D1 V, D2 V) + nu Lap(w) at listed targets, with the velocity in V
 * supplied as a full field uv (3 planes of length N).  The medium-order model
 * takes that velocity from the FFT solver (sec. 2; sec. 6), so a caller can
 * hand in an FFT velocity computed elsewhere where the direct DFT above is
 * too slow for the mesh.  Periodic sheets only; wt: 2 planes of length
 * ntargets. */
int zmo_wt_sampled(const zmo_problem *P, const double *z, const double *w, const double *uv,
                   int64_t ntargets, const int64_t *targets, double *wt)
{
    if (!P || P->n1 < 1 || P->n2 < 1 || ntargets < 0 || !targets || !uv || P->boundary != 0)
        return -1;
    const int n1 = P->n1, n2 = P->n2;
    const size_t N = (size_t)n1 * n2;
    for (int64_t t = 0; t < ntargets; ++t)
        if (targets[t] < 0 || (size_t)targets[t] >= N) return -1;
    double *buf = (double *)malloc(sizeof(double) * 10 * N);
    if (!buf) return -1;
    double *t1 = buf, *t2 = buf + 3 * N, *gamma = buf + 6 * N, *q = buf + 9 * N;
    zmo_surface(P, z, w, t1, t2, gamma, q);
    for (int64_t t = 0; t < ntargets; ++t) {
        const int i1 = (int)(targets[t] % n1), i2 = (int)(targets[t] / n1);
        double V[9];
        for (int k = 0; k < 9; ++k) {
            int w1, w2;
            const int j1 = wrap_index(i1 + stencil_off1[k], n1, &w1);
            const int j2 = wrap_index(i2 + stencil_off2[k], n2, &w2);
            const size_t p = (size_t)j2 * n1 + j1;
            V[k] = bernoulli(P, uv[p], uv[N + p], uv[2 * N + p], q[p], z[2 * N + p]);
        }
        wt_from_stencil(P, w, V, targets[t], ntargets, t, wt);
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------ */
/* time integration                                                    */
/* ------------------------------------------------------------------ */

/* nsteps of the Shu-Osher strong-stability-preserving RK3 on y = (z, w):
 *   y1 = y0 + dt F(y0)
 *   y2 = 3/4 y0 + 1/4 (y1 + dt F(y1))
 *   y3 = 1/3 y0 + 2/3 (y2 + dt F(y2))
 * z (3 planes) and w (2 planes) are advanced in place. */
int zmo_rk3_step(const zmo_problem *P, double *z, double *w, int nsteps, int nthreads)
{
    if (!P || P->n1 < 1 || P->n2 < 1 || nsteps < 0) return -1;
    const size_t N = (size_t)P->n1 * P->n2;
    const size_t M = 5 * N;            /* y = (z planes, w planes) */
    const double dt = P->dt;
    double *mem = (double *)malloc(sizeof(double) * 4 * M);
    if (!mem) return -1;
    double *y0 = mem, *y1 = mem + M, *y2 = mem + 2 * M, *F = mem + 3 * M;
    for (int step = 0; step < nsteps; ++step) {
        memcpy(y0, z, sizeof(double) * 3 * N);
        memcpy(y0 + 3 * N, w, sizeof(double) * 2 * N);
        int rc = zmo_rhs(P, y0, y0 + 3 * N, F, F + 3 * N, nthreads);
        if (rc) { free(mem); return rc; }
        for (size_t k = 0; k < M; ++k) y1[k] = y0[k] + dt * F[k];
        rc = zmo_rhs(P, y1, y1 + 3 * N, F, F + 3 * N, nthreads);
        if (rc) { free(mem); return rc; }
        for (size_t k = 0; k < M; ++k) y2[k] = 0.75 * y0[k] + 0.25 * (y1[k] + dt * F[k]);
        rc = zmo_rhs(P, y2, y2 + 3 * N, F, F + 3 * N, nthreads);
        if (rc) { free(mem); return rc; }
        for (size_t k = 0; k < M; ++k) {
            double y3 = (1.0 / 3.0) * y0[k] + (2.0 / 3.0) * (y2[k] + dt * F[k]);
            if (k < 3 * N) z[k] = y3; else w[k - 3 * N] = y3;
        }
    }
    free(mem);
    return 0;
}

int zmo_abi_version(void) { return 5; }
