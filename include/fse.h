/*
 * fse.h -- C ABI of libfse: free-space spectral Ewald (FSE) evaluation of
 * stokeslet, stresslet and rotlet sums on one AMD Instinct MI355X (gfx950).
 *
 * Method: af Klinteberg, Shamshirgar & Tornberg, "Fast Ewald summation for
 * free-space Stokes potentials", arXiv:1607.04808.
 *
 * Problem (Section 1, eq. usumfree; Section 2, eq. usum):
 *     u(x_m) = sum_{n != m} G(x_m - x_n) . f_n ,   m = 1..N,
 * with G the stokeslet S_jl = d_jl/r + r_j r_l/r^3 (eq. def_stokeslet), the
 * stresslet T_jlm = -6 r_j r_l r_m / r^5 acting on f_lm = n_l q_m
 * (eq. def_stresslet, Section 2) or the rotlet Omega_jl = eps_jlm r_m / r^3
 * (eq. def_rotlet).  All points lie in the cube [box_lo, box_lo + L)^3
 * (Section 5.2, Section 8).
 *
 * Conventions shared by every entry point:
 *   - Array pointers are DEVICE pointers (HIP global memory) owned by the
 *     caller, C-contiguous, in the plan's dtype (float or double).  Positions
 *     x: (n, 3).  Sources and results: (batch, n, 3) with the batch index
 *     slowest (batch = 1 means a plain (n, 3) array).
 *   - Work is enqueued on the plan's HIP stream and is asynchronous; entry
 *     points only synchronise where stated.
 *   - The plan owns all workspace.  A plan is not thread-safe; calls on one
 *     plan must not overlap.
 *   - No C++ exception crosses the ABI.  Every call returns an fse_status_t;
 *     on failure fse_last_error() gives a thread-local message.
 */
#ifndef FSE_H
#define FSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { FSE_STOKESLET = 0, FSE_STRESSLET = 1, FSE_ROTLET = 2 } fse_kernel_t;
typedef enum { FSE_F32 = 0, FSE_F64 = 1 } fse_dtype_t;

typedef enum {
    FSE_OK = 0,
    FSE_EINVAL = 1,        /* bad argument or parameter                       */
    FSE_ERANGE = 2,        /* a point outside [box_lo, box_lo+L)^3 or not finite */
    FSE_ENOMEM = 3,        /* device allocation failed                        */
    FSE_EHIP = 4,          /* a HIP runtime call failed                       */
    FSE_EUNSUPPORTED = 5,  /* combination not implemented (e.g. stresslet adjoint) */
    FSE_ESTATE = 6         /* call order violated (e.g. eval before set_points) */
} fse_status_t;

/*
 * Method parameters (Section 8.2 "Parameter selection"): the Ewald parameter
 * xi, the real-space cutoff rc (Section 6), the number of grid intervals M on
 * the box side (h = L/M) and the Gaussian support P (P^3 window, Section 5.2).
 */
typedef struct {
    double xi;           /* Ewald split parameter, > 0                          */
    double rc;           /* real-space cutoff radius, > 0                        */
    int32_t M;           /* grid intervals on the box side L, >= 1              */
    int32_t P;           /* Gaussian support in grid points, 2 <= P <= 32       */
    double box_lo[3];    /* lower corner of the cube holding all points         */
    double L;            /* side of the cube, > 0                               */
    int32_t deltaL_rule; /* 0: deltaL = d = hP (Results section);
                            1: deltaL from eq. deltaL_cond (Section 5.3)        */
    int32_t Mt;          /* 0: the smallest grid size >= M + deltaL/h whose
                            doubled size 2*Mt factors into 2,3,5,7;
                            > 0: use this size (must be >= that minimum and
                            2*Mt must factor into 2,3,5,7)                      */
    double C;            /* Gaussian shape constant of m = C sqrt(pi P);
                            0 selects 0.976 (Section 5.3)                       */
    int32_t periodic;    /* 0: the free-space sum (eq. usumfree);
                            1: the triply periodic stokeslet sum of Section 1.1
                            (eq. usumper, period L in every direction, by the
                            Hasimoto split eq. usum_SR_SF_limit with eqs.
                            SR_Hasimoto, ShatH, Slimit): no domain extension or
                            precompute, the M^3 grid is the period, 2M must
                            factor into 2,3,5,7, P <= M and rc <= L/2;
                            deltaL_rule and Mt are ignored.  Stokeslet only;
                            fse_eval and fse_eval_parts only.                   */
} fse_params_t;

/*
 * Derived geometry (Sections 4.1, 6.2, 6.3 and the Results section):
 * h = L/M, d = hP, m = C sqrt(pi P), eta = (xi d/m)^2, alpha = 2 xi^2/eta
 * (exponent of the gridding Gaussians, eq. Hx), Lt = Mt h, grid nodes
 * x0 + j h (j = 0..Mt-1) with x0 = box_lo - (Lt - L)/2, FFT size n = 2 Mt,
 * R = sqrt(3) Lt, precompute grid Mg = smallest even integer > (1+sqrt 3) Mt,
 * kinf = pi/h.  The real-space pass uses a cell list of ncell^3 cells of
 * side cell >= rc.
 */
typedef struct {
    int32_t Mt, n_fft, Mg;
    int32_t ncell;
    double h, d, m, eta, alpha, Lt, R, deltaL, kinf, cell;
    double x0[3];
    int32_t radices[8];  /* FFT factorisation of n_fft, 0-terminated */
} fse_geometry_t;

typedef struct fse_plan fse_plan_t;

/* Host only, no device work.  Validates the parameters and fills *out.
 * Returns FSE_EINVAL for out-of-range parameters or an impossible Mt. */
fse_status_t fse_geometry(fse_kernel_t kernel, const fse_params_t *params, fse_geometry_t *out);

/*
 * Create a plan for `batch` (>= 1) source vectors over shared positions and
 * at most `nmax` points.  Allocates every workspace buffer on the current HIP
 * device and runs the FP64 precompute of the mollified Green's function
 * transform (Section 4.3: the truncated biharmonic transform, eq. BhatR, for
 * the stokeslet and stresslet, or the harmonic one, eq. HhatR, for the
 * rotlet, oversampled on Mg^3, inverse-transformed, cropped to (2Mt)^3 and
 * transformed back), folded with the scaling factors of eq. gridfcnsc and
 * eqs. AS/AT/AR.  `stream` is a hipStream_t (NULL = the null stream).
 * Synchronises the stream once, at the end.  *out is NULL on failure.
 */
fse_status_t fse_plan_create(fse_kernel_t kernel, fse_dtype_t dtype, const fse_params_t *params,
                             int32_t batch, int64_t nmax, void *stream, fse_plan_t **out);

/* Geometry the plan was built with (host copy). */
fse_status_t fse_plan_geometry(const fse_plan_t *plan, fse_geometry_t *out);

/* Change the stream later calls are enqueued on. */
fse_status_t fse_plan_set_stream(fse_plan_t *plan, void *stream);

/*
 * Set the n (2 <= n <= nmax) points x (device, (n,3), plan dtype): bins them
 * by grid tile (for spreading and quadrature, Section 5.2) and by real-space
 * cell (Section 6's cell list), computes each point's Gaussian window start
 * and offset in FP64, and keeps sorted copies.  Points outside the box are
 * clamped into it on the device, so no kernel ever leaves its buffers.
 * validate != 0: also synchronises the stream and returns FSE_ERANGE if any
 * point was outside [box_lo, box_lo+L)^3 or not finite.  Coincident
 * distinct points give an undefined sum (as the direct sum does).
 */
fse_status_t fse_set_points(fse_plan_t *plan, int64_t n, const void *x, int32_t validate);

/*
 * u = u^R + u^F + u^self at the n points (Section 8): src_a is f (stokeslet,
 * rotlet) or q (stresslet), src_b is NULL or the normals n (stresslet), both
 * (batch, n, 3); u is (batch, n, 3) and is overwritten.  The scaled,
 * inverse-transformed grid of this call is kept for fse_eval_adjoint.
 */
fse_status_t fse_eval(fse_plan_t *plan, const void *src_a, const void *src_b, void *u);

/*
 * The two parts separately (for tests): u_real = u^R + u^self (the truncated
 * real-space sum of Section 6 plus the stokeslet self term, eq. Slimit) and
 * u_fourier = u^F (the five steps of Section 5.2).  Either may be NULL.
 */
fse_status_t fse_eval_parts(fse_plan_t *plan, const void *src_a, const void *src_b, void *u_real,
                            void *u_fourier);

/*
 * Separate targets (Section 2: the sums may be evaluated at the sources or at
 * any other points): bins the nt (>= 1) targets y (device, (nt, 3), plan dtype)
 * like fse_set_points does the points; they must lie in the same box.  The
 * plan keeps them until the next call, which may change nt (buffers grow on
 * demand with hipMalloc, after a stream synchronisation).  validate as in
 * fse_set_points.
 */
fse_status_t fse_set_targets(fse_plan_t *plan, int64_t nt, const void *y, int32_t validate);

/*
 * u(y_t) = sum_n G(y_t - x_n) . f_n at the targets of fse_set_targets from the
 * points of fse_set_points (sources as in fse_eval): u^F by the quadrature at
 * the targets and u^R over the sources within r_c; no self term, and a target
 * that coincides with a source skips that pair.  With u_fourier == NULL,
 * u_real receives the whole sum u (batch, nt, 3); otherwise u_real (may be
 * NULL) gets u^R and u_fourier gets u^F separately.
 */
fse_status_t fse_eval_targets(fse_plan_t *plan, const void *src_a, const void *src_b, void *u_real,
                              void *u_fourier);

/*
 * Adjoint of fse_eval for L = sum_m w_m . u(x_m) (stokeslet and rotlet, whose
 * discrete operator is symmetric): dsrc = dL/df = K w (batch, n, 3) and
 * dx = dL/dx (n, 3), summed over the batch, from the derivatives of the
 * Gaussian windows (spreading and quadrature) and of the real-space kernel.
 * src_a must be the f of the last fse_eval on this plan and set_points must
 * not have been called since; with recompute != 0 the forward grid is
 * rebuilt from src_a first.  Either output may be NULL.
 * FSE_EUNSUPPORTED for the stresslet.
 */
fse_status_t fse_eval_adjoint(fse_plan_t *plan, const void *src_a, const void *w, void *dsrc,
                              void *dx, int32_t recompute);

/*
 * Forward sum and adjoint in one call, for L = sum_m w_m . u(x_m) with w known
 * beforehand (stokeslet and rotlet plans; Sections 3 and 5 as fse_eval and
 * fse_eval_adjoint): u = the sum of fse_eval, dsrc = dL/da = K w and dx = dL/dx,
 * each laid out as there, all three required (device pointers, the plan's dtype).
 * The two source sets are spread in one pass, the forward quadrature and the first
 * gradient term share one sweep of the forward field, and (batch 1) one pass over
 * the real-space pairs adds u^R + self term, the real part of K w and its part of
 * dL/dx.  The results equal those of fse_eval followed by fse_eval_adjoint to
 * rounding.  Afterwards the forward field is kept as after fse_eval.
 * FSE_EUNSUPPORTED for stresslet and periodic plans; FSE_ESTATE before
 * fse_set_points.
 */
fse_status_t fse_eval_with_adjoint(fse_plan_t *plan, const void *src_a, const void *w, void *u, void *dsrc,
                                   void *dx);

/*
 * Adjoint of fse_eval for the stresslet (eq. def_stresslet), L = sum_m w_m .
 * u(x_m) with u_j(x_m) = sum_{n != m} T_jlm(x_m - x_n) q_l(n) n_m(n): at each
 * point b, D_lm = sum_{a != b} w_j(a) T_jlm(x_a - x_b) (T fully symmetric, so D
 * is the symmetric 2-tensor of the transposed chain: w spread as 3 components,
 * the transposed multiplier +i P_j,lm(k) of eq. AT, six output components,
 * plus the real-space pairs within r_c), and dq_l = dL/dq_l = D_lm n_m,
 * dn_m = dL/dn_m = D_lm q_l.  q, nrm, w: (batch, n, 3); dq, dn: (batch, n, 3),
 * overwritten.  The plan's field buffer then holds the adjoint field, so a
 * following fse_eval_adjoint must recompute the forward field.
 */
fse_status_t fse_eval_adjoint_stresslet(fse_plan_t *plan, const void *q, const void *nrm, const void *w,
                                        void *dq, void *dn);

/* Copy the (Mt+1)^3 FP64 octant of the scalar Fourier multiplier (the
 * precomputed mollified kernel transform times the kernel's scalar factors
 * and normalisations) to host memory `out`.  Synchronises. */
fse_status_t fse_plan_multiplier(fse_plan_t *plan, double *out);

/* Copy, for tests, the grid of the last evaluation to host memory `out` as
 * FP64, layout (batch, components, z, y, x) with x fastest, Mt^3 per
 * component: which = 0 the spread sources (step 1 of Section 5.2, without the
 * Gaussian normalisation), which = 1 the scaled inverse-transformed grid that
 * the quadrature reads (step 4).  Synchronises. */
fse_status_t fse_plan_grid(fse_plan_t *plan, int32_t which, double *out);

/* The process-wide cache of the mollified transform (Section 4.3): plans with the
 * grid side Mt and kernel family (biharmonic: stokeslet, stresslet; harmonic:
 * rotlet) of an earlier plan on the same device reuse its transform, scaled by
 * (h / h0)^4 or (h / h0)^2 for their grid spacing h (the truncated transform is
 * homogeneous in k and R = sqrt(3) Mt h), and skip the precompute's FFT
 * contractions.  Entries are device memory held until the process ends, 2 GiB in
 * all at most; the no-allocation entry point reads them but adds none.  Reports
 * the lookups that found an entry (hits) or computed it (misses), the bytes held
 * and the entries.  Any pointer may be NULL. */
fse_status_t fse_precompute_cache_stats(int64_t *hits, int64_t *misses, size_t *bytes, int32_t *entries);

/* Copy, for tests, the binning of the points last set (fse_set_points) to host
 * memory.  Any array pointer may be NULL; n is the point count, nbins the bins
 * per side of the spreading grid (written first, so a call with NULL arrays
 * gives the sizes) and ncell the geometry's cells per side:
 *   perm_s[n]     the point (index into x) at each position of the spread order:
 *                 points ordered by bin (bins of bin_side^3 grid nodes, x
 *                 fastest), in input order within a bin;
 *   bpack_s[n]    its window start b = floor(t - P/2 + 1), t = (x - x0)/h, per
 *                 direction (Section 5.1's support of eq. Hx), packed
 *                 bx | by << 10 | bz << 20;
 *   coff_s[3n]    its window-centre offset t - b - (P - 1)/2 per direction, as the
 *                 quadrature and spreading use it (the plan's dtype, widened);
 *   tile_start[nbins^3 + 1]   first spread-order position of each bin;
 *   perm_r[n], cell_start[ncell^3 + 1]   the same order and offsets for the
 *                 real-space cells (side >= r_c, Section 6).
 * FSE_ESTATE before fse_set_points.  Synchronises. */
fse_status_t fse_plan_bins(fse_plan_t *plan, int32_t *nbins, int32_t *perm_s, int32_t *bpack_s, double *coff_s,
                           int32_t *tile_start, int32_t *perm_r, int32_t *cell_start);

/*
 * Per-stage timing with HIP events recorded on the plan's stream around each
 * kernel launch group.  Stages (index: name): 0 bin, 1 permute, 2 spread,
 * 3 fft_x, 4 fft_y, 5 fft_z_scale, 6 fft_yinv, 7 fft_xinv, 8 gather, 9 real,
 * 10 gather_grad, 11 real_grad.  Timing is off by default.
 * fse_plan_timings synchronises the stream, writes the summed milliseconds
 * (ms[FSE_NSTAGES]) and launch-group counts (launches[FSE_NSTAGES], may be
 * NULL) since the last call, and resets them.
 */
#define FSE_NSTAGES 12
fse_status_t fse_plan_set_timing(fse_plan_t *plan, int32_t enable);
fse_status_t fse_plan_timings(fse_plan_t *plan, double *ms, int64_t *launches);
const char *fse_stage_name(int32_t stage);

/*
 * Free-space harmonic and biharmonic solver (Section 4: the truncated-kernel
 * method of Section 4.1 with the oversampling of Section 4.2 moved into the
 * precompute of Section 4.3): u = G * f, u(x_i) = integral of G(x_i - y) f(y)
 * dy over the box, for family 0 the biharmonic G = r (eq. BhatR's kernel) and
 * family 1 the harmonic G = 1/r (eq. HhatR's), with f sampled on the M^3 grid
 * of spacing h (nodes j h, j = 0..M-1, and f negligible at the faces) and u
 * returned at the same nodes.  Spectrally accurate for smooth f (Table 1's
 * closed forms, e.g. H * gamma_E = erf(xi r)/r).  f, u: ncomp device fields of
 * M^3 in the dtype, x fastest; 2M must factor into 2,3,5,7 (M <= 1024).
 * Allocates its workspace, runs on `stream` and synchronises it.
 */
fse_status_t fse_freespace_solve(int32_t family, fse_dtype_t dtype, int32_t M, double h, int32_t ncomp,
                                 const void *f, void *u, void *stream);

/*
 * Truncation-error estimates for a parameter set (host only): the RMS over
 * targets of the real-space truncation error, Table est_real (Section 7.2),
 * and of the Fourier-space truncation error, Table est_fourier (Section 7.1,
 * with kinf = pi/h and R = sqrt(3) Lt), both absolute.  Q = sum_n |f_n|^2
 * (stokeslet, rotlet; eq. Q_stokeslet) or sum_n |q_n|^2 |n_n|^2 (stresslet,
 * eq. Q_stresslet).  Either output may be NULL.
 */
fse_status_t fse_error_estimates(fse_kernel_t kernel, const fse_params_t *params, double Q,
                                 double *est_real, double *est_fourier);

/*
 * Parameter selection (host only; Section 8.2).  For n points in the cube
 * [box_lo, box_lo + L)^3 and a target relative max-norm error rel_tol, picks
 * P = 2 points per digit of rel_tol (even, in [8, 32]; Section 8.2's 16 for 8
 * digits and 24 for 12), and for each xi of a geometric sweep the r_c and M
 * that hold the estimates of Tables est_real and est_fourier at an absolute
 * RMS target eps = rel_tol * share * u_rms / sqrt 2 (share = 0.6 in FP64, a
 * margin for the adjoint's gradient, 0.4 in FP32 to leave room for rounding),
 * with eta <= 0.95 (FP64) or 0.7 (FP32).  Of the
 * sweep it returns the xi (with its r_c, M, P, and Mt = the smallest size with
 * 2 Mt 7-smooth that holds the box extended by eq. deltaL_cond's deltaL, the
 * Section 5.3 rule that keeps the remainder Gaussians' support inside the
 * grid) that minimises a cost model of this library's kernels on
 * one MI355X (real-space pairs, transform nodes, window nodes; uniform
 * density assumed).  Q as in fse_error_estimates; u_rms is the RMS of |u| over
 * the targets, or <= 0 for an estimate for points uniform in the cube.
 * FSE_EINVAL for rel_tol outside (0, 1), FP32 with rel_tol < 1e-6, or when no
 * xi fits the grid limit.  deltaL_rule = 1 and C = 0 in *out.
 */
fse_status_t fse_choose_params(fse_kernel_t kernel, fse_dtype_t dtype, int64_t n, const double box_lo[3],
                               double L, double rel_tol, double Q, double u_rms, fse_params_t *out);

/*
 * Bounding-cube default of the box (Section 8 assumes a cube holding every
 * point): box_lo = the componentwise minimum of the n points x (device, (n,3),
 * dtype) and L = the largest extent times (1 + 2^-20), so that the largest
 * coordinate lies strictly inside [box_lo, box_lo + L).  Runs a reduction on
 * `stream` (a hipStream_t) and synchronises it; allocates a small temporary.
 * FSE_ERANGE if a coordinate is not finite.
 */
fse_status_t fse_bounding_box(fse_dtype_t dtype, int64_t n, const void *x, void *stream,
                              double box_lo[3], double *L);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): fse_plan_create,
 * fse_set_points and fse_eval in one call, with every workspace buffer (grids,
 * spectra, sort buffers, the precompute's temporaries) carved from a static
 * device array of FSE_NOALLOC_MAX_BYTES that each GPU the library runs on holds
 * until the process ends.  Calls no hipMalloc/hipFree or other allocating
 * routine.  Arguments as fse_plan_create (params, batch, stream), fse_set_points
 * (n points x, validate) and fse_eval (src_a, src_b, u), all device pointers in
 * the dtype; u is overwritten.  An evaluation whose workspace exceeds the
 * array returns FSE_EINVAL before any device work (fse_last_error names the
 * bytes it needs).  Every call on one GPU uses that GPU's one array and leaves
 * its contents there: calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  Each call reruns the
 * FP64 precompute, or scales a transform that an earlier plan on this GPU left in
 * the precompute cache (fse_precompute_cache_stats), and synchronises `stream`
 * (table upload and precompute).
 */
#define FSE_NOALLOC_MAX_BYTES ((size_t)64 << 20)
fse_status_t fse_eval_noalloc(fse_kernel_t kernel, fse_dtype_t dtype, const fse_params_t *params,
                              int32_t batch, int64_t n, const void *x, const void *src_a,
                              const void *src_b, void *u, int32_t validate, void *stream);

/*
 * Launch shapes of a plan (runtime knobs of this implementation, not of the
 * method): the side of the point bins, in grid nodes, that spreading and the
 * quadrature work in (tiles); the real-space hit-queue depths per thread of the
 * value and the gradient pass; the most waves (64 targets each) a real-space
 * work item takes; the most FFT lines (rows) one workgroup transforms.  Plans
 * start at the defaults; fse_plan_autotune times the candidates on the plan's
 * own workload and keeps the fastest.  No knob changes what is summed; the bin
 * side, queue depths and waves change the order of some sums, so results move by
 * rounding only (the FFT line count changes nothing: bit-identical fields).
 */
typedef struct {
    int32_t bin_side;         /* 4..8                                           */
    int32_t real_queue;       /* 16..96, a multiple of 8                        */
    int32_t real_queue_grad;  /* 16..96, a multiple of 8                        */
    int32_t real_waves;       /* 1..4                                           */
    int32_t fft_lines;        /* 0: each pass's default (16 or 8 FP32, 4 or 2   */
                              /* FP64, fewer where the lines exceed LDS);       */
                              /* 1, 2, 4, 8 or 16: at most that many per        */
                              /* workgroup, and the z-pass one column at a time */
} fse_tuning_t;

fse_status_t fse_plan_get_tuning(const fse_plan_t *plan, fse_tuning_t *out);

/* Apply a tuning (FSE_EINVAL outside the ranges above).  The points and any
 * targets must be set again afterwards (FSE_ESTATE otherwise). */
fse_status_t fse_plan_set_tuning(fse_plan_t *plan, const fse_tuning_t *tuning);

/*
 * Autotune the plan on its workload: for the n points x and sources (src_a,
 * src_b as fse_eval) and, when w != NULL (stokeslet and rotlet), the adjoint
 * weights, time `repeats` runs of fse_set_points + fse_eval (with w:
 * fse_eval_with_adjoint; periodic plans fse_eval + fse_eval_adjoint) with HIP
 * events for each candidate of each knob in turn (bin side, real-space waves,
 * the two queue depths, the FFT line cap; a queue depth whose pass the timed
 * calls never run keeps its value), keep the fastest, and leave the plan
 * with it and the points set.  *best (may be NULL) receives the tuning.  Allocates
 * temporary outputs and synchronises the stream.
 */
fse_status_t fse_plan_autotune(fse_plan_t *plan, int64_t n, const void *x, const void *src_a, const void *src_b,
                               const void *w, int32_t repeats, fse_tuning_t *best);

/* Device bytes held by the plan.  Synchronises nothing. */
fse_status_t fse_plan_workspace(const fse_plan_t *plan, size_t *bytes);

void fse_plan_destroy(fse_plan_t *plan);
const char *fse_status_string(fse_status_t status);
const char *fse_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FSE_H */
