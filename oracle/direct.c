/*
 * TEST INFRASTRUCTURE ONLY -- the CPU reference ("oracle") for the free-space
 * Stokes sums.  Only tests, the smoke check and the benchmark's CPU-baseline
 * leg may load this library.  It shares no code with the GPU library.
 *
 * Plain FP64 sums written from the definitions in
 *   af Klinteberg, Shamshirgar, Tornberg, "Fast Ewald summation for free-space
 *   Stokes potentials" (arXiv:1607.04808):
 *   - the kernels S, T, Omega: Section 2, eqs. def_stokeslet, def_stresslet,
 *     def_rotlet;  u(x_m) = sum_{n != m} G(x_m - x_n) . f_n  (eq. usumfree,
 *     eq. usum);  stresslet sources f_lm = n_l q_m (Section 2).
 *   - the real-space parts G^R: Section 3.2, eqs. SR_Op, TR_Op, RR_Op, with the
 *     readings listed below.
 *   - the Fourier parts G^F = G - G^R written in closed form with erf, and the
 *     self value G^F(0) (eq. Slimit).
 *
 * Readings of the paper taken here (each is pinned by a CPU test):
 *   - rotlet normalisation: the sum uses Omega_jl = eps_jlm r_m / r^3 as
 *     defined in eq. def_rotlet; its real-space part is therefore
 *     -eps_jlm d_m (erfc(xi r)/r) = eps_jlm rhat_m (erfc/r^2 + 2 xi e^{-xi^2 r^2}/(sqrt(pi) r)),
 *     i.e. one half of eq. RR_Op, whose factor 2 belongs to the operator form.
 *   - stresslet: the delta-term coefficient of eq. TR_Op carries a factor r,
 *     A2 = 4 xi^3 r e^{-xi^2 r^2}/sqrt(pi) (third derivative of r*erfc(xi r) -
 *     e^{-xi^2 r^2}/(sqrt(pi) xi)); eq. TR2int only holds with it.
 *
 * Kernel ids: 0 stokeslet, 1 stresslet, 2 rotlet.
 * Source layout: a = f (n x 3) for S and Omega; a = q, b = n (normal) for T.
 * Target layout: y (nt x 3) arbitrary points, skip[t] = source index whose
 * term is excluded (the target's own source), or -1.
 * Loop order: sources in ascending index, FP64 accumulation, OpenMP over
 * targets.  Coincident distinct points are undefined (asserted).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <stdio.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static const double SQRTPI = 1.77245385090551602729816748334;

static inline double dot3(const double *a, const double *b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* ---- full kernels (Section 2) -------------------------------------------- */

/* u += G(r) . src for the three kernels, r != 0. */
static void add_full(int kernel, const double r[3], const double *a,
                     const double *b, double u[3]) {
    double r2 = dot3(r, r);
    double ri = 1.0 / sqrt(r2);
    double ri3 = ri * ri * ri;
    if (kernel == 0) {
        /* S_jl f_l = f_j / r + r_j (r.f) / r^3 */
        double rf = dot3(r, a);
        for (int j = 0; j < 3; ++j) u[j] += a[j] * ri + r[j] * rf * ri3;
    } else if (kernel == 1) {
        /* T_jlm n_l q_m = -6 r_j (r.n)(r.q) / r^5 */
        double c = -6.0 * dot3(r, a) * dot3(r, b) * ri3 * ri * ri;
        for (int j = 0; j < 3; ++j) u[j] += c * r[j];
    } else {
        /* Omega_jl f_l = eps_jlm f_l r_m / r^3 = (f x r)_j / r^3 */
        u[0] += (a[1] * r[2] - a[2] * r[1]) * ri3;
        u[1] += (a[2] * r[0] - a[0] * r[2]) * ri3;
        u[2] += (a[0] * r[1] - a[1] * r[0]) * ri3;
    }
}

/* ---- real-space parts (Section 3.2) -------------------------------------- */

static void add_real(int kernel, double xi, const double r[3], const double *a,
                     const double *b, double u[3]) {
    double rr = sqrt(dot3(r, r));
    double rh[3] = {r[0] / rr, r[1] / rr, r[2] / rr};
    double ec = erfc(xi * rr);
    double ex = exp(-xi * xi * rr * rr);
    if (kernel == 0) {
        /* eq. SR_Op: 2(xi e/sqrt(pi) + erfc/(2r))(delta + rh rh) - 4 xi e/sqrt(pi) delta */
        double c1 = 2.0 * (xi * ex / SQRTPI + ec / (2.0 * rr));
        double cd = c1 - 4.0 * xi * ex / SQRTPI;
        double rf = dot3(rh, a);
        for (int j = 0; j < 3; ++j) u[j] += cd * a[j] + c1 * rh[j] * rf;
    } else if (kernel == 1) {
        /* eq. TR_Op with A2 = 4 xi^3 r e / sqrt(pi):
           T^R_jlm n_l q_m = A1 rh_j (rh.n)(rh.q) + A2 (n_j (rh.q) + rh_j (n.q) + q_j (rh.n)) */
        double A1 = -(2.0 / rr) * (3.0 * ec / rr + (2.0 * xi / SQRTPI) * (3.0 + 2.0 * xi * xi * rr * rr) * ex);
        double A2 = 4.0 * xi * xi * xi * rr * ex / SQRTPI;
        const double *q = a, *nn = b;
        double rq = dot3(rh, q), rn = dot3(rh, nn), nq = dot3(nn, q);
        for (int j = 0; j < 3; ++j)
            u[j] += A1 * rh[j] * rn * rq + A2 * (nn[j] * rq + rh[j] * nq + q[j] * rn);
    } else {
        /* half of eq. RR_Op (eq. def_rotlet normalisation) */
        double c = ec / (rr * rr) + 2.0 * xi * ex / (SQRTPI * rr);
        u[0] += c * (a[1] * rh[2] - a[2] * rh[1]);
        u[1] += c * (a[2] * rh[0] - a[0] * rh[2]);
        u[2] += c * (a[0] * rh[1] - a[1] * rh[0]);
    }
}

/* ---- Fourier parts G^F = G - G^R in closed form --------------------------- */

static void add_fourier(int kernel, double xi, const double r[3], const double *a,
                        const double *b, double u[3]) {
    double r2 = dot3(r, r);
    if (r2 == 0.0) {
        /* self value: only the stokeslet's is non-zero (eq. Slimit) */
        if (kernel == 0)
            for (int j = 0; j < 3; ++j) u[j] += 4.0 * xi / SQRTPI * a[j];
        return;
    }
    double rr = sqrt(r2);
    double rh[3] = {r[0] / rr, r[1] / rr, r[2] / rr};
    double ef = erf(xi * rr);
    double ex = exp(-xi * xi * r2);
    if (kernel == 0) {
        double cd = ef / rr + 2.0 * xi * ex / SQRTPI;
        double cr = ef / rr - 2.0 * xi * ex / SQRTPI;
        double rf = dot3(rh, a);
        for (int j = 0; j < 3; ++j) u[j] += cd * a[j] + cr * rh[j] * rf;
    } else if (kernel == 1) {
        double A1 = -6.0 * ef / r2 + (12.0 * xi / (SQRTPI * rr) + 8.0 * xi * xi * xi * rr / SQRTPI) * ex;
        double A2 = -4.0 * xi * xi * xi * rr * ex / SQRTPI;
        const double *q = a, *nn = b;
        double rq = dot3(rh, q), rn = dot3(rh, nn), nq = dot3(nn, q);
        for (int j = 0; j < 3; ++j)
            u[j] += A1 * rh[j] * rn * rq + A2 * (nn[j] * rq + rh[j] * nq + q[j] * rn);
    } else {
        double c = ef / r2 - 2.0 * xi * ex / (SQRTPI * rr);
        u[0] += c * (a[1] * rh[2] - a[2] * rh[1]);
        u[1] += c * (a[2] * rh[0] - a[0] * rh[2]);
        u[2] += c * (a[0] * rh[1] - a[1] * rh[0]);
    }
}

/* ---- public sums ----------------------------------------------------------
 * mode 0: full kernel, sources n != skip[t]
 * mode 1: real-space part, 0 < |r| <= rc and n != skip[t]
 * mode 2: Fourier part over ALL sources (n == skip[t] contributes G^F(0))
 */
static int sum_generic(int mode, int kernel, double xi, double rc, int64_t n,
                       const double *x, const double *a, const double *b,
                       int64_t nt, const double *y, const int64_t *skip, double *out) {
    if (kernel < 0 || kernel > 2) return 1;
    if (kernel == 1 && b == NULL) return 1;
    int bad = 0;
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t t = 0; t < nt; ++t) {
        double u[3] = {0.0, 0.0, 0.0};
        const double *yt = y + 3 * t;
        int64_t sk = skip ? skip[t] : -1;
        for (int64_t s = 0; s < n; ++s) {
            double r[3] = {yt[0] - x[3 * s], yt[1] - x[3 * s + 1], yt[2] - x[3 * s + 2]};
            double r2 = dot3(r, r);
            const double *as = a + 3 * s;
            const double *bs = b ? b + 3 * s : NULL;
            if (mode == 2) {
                if (s == sk) { double z[3] = {0, 0, 0}; add_fourier(kernel, xi, z, as, bs, u); continue; }
                if (r2 == 0.0) { bad = 1; continue; }
                add_fourier(kernel, xi, r, as, bs, u);
                continue;
            }
            if (s == sk) continue;
            if (r2 == 0.0) { bad = 1; continue; }
            if (mode == 0) add_full(kernel, r, as, bs, u);
            else if (r2 <= rc2) add_real(kernel, xi, r, as, bs, u);
        }
        out[3 * t] = u[0];
        out[3 * t + 1] = u[1];
        out[3 * t + 2] = u[2];
    }
    return bad ? 2 : 0;
}

int oracle_direct(int kernel, int64_t n, const double *x, const double *a, const double *b,
                  int64_t nt, const double *y, const int64_t *skip, double *out) {
    return sum_generic(0, kernel, 0.0, 0.0, n, x, a, b, nt, y, skip, out);
}

int oracle_real_trunc(int kernel, double xi, double rc, int64_t n, const double *x,
                      const double *a, const double *b, int64_t nt, const double *y,
                      const int64_t *skip, double *out) {
    return sum_generic(1, kernel, xi, rc, n, x, a, b, nt, y, skip, out);
}

int oracle_fourier_dir(int kernel, double xi, int64_t n, const double *x, const double *a,
                       const double *b, int64_t nt, const double *y, const int64_t *skip,
                       double *out) {
    return sum_generic(2, kernel, xi, 0.0, n, x, a, b, nt, y, skip, out);
}

/* ---- gradients -------------------------------------------------------------
 * L = sum_m w_m . sum_{n != m} G(x_m - x_n) . f_n  over targets = sources.
 * dL/dx_p = sum_{n != p} [ grad_r (w_p . G(r) f_n) + s * grad_r (w_n . G(r) f_p) ],
 * r = x_p - x_n, s = +1 for the even stokeslet, -1 for the odd rotlet.
 * mode 0 uses the full kernel, mode 1 the real-space part with 0 < |r| <= rc.
 */

/* grad_r (w . G(r) f) for the stokeslet (full or real-space part) */
static void grad_stokeslet(int real, double xi, const double r[3], const double *w,
                           const double *f, double g[3]) {
    double r2 = dot3(r, r), rr = sqrt(r2);
    double A, dA, Bc, dB; /* w.G f = A(r) (w.f) + Bc(r) (w.r)(f.r),  Bc = b/r^2 */
    if (!real) {
        A = 1.0 / rr; dA = -1.0 / r2;
        Bc = 1.0 / (r2 * rr); dB = -3.0 / (r2 * r2);
    } else {
        double ec = erfc(xi * rr), ex = exp(-xi * xi * r2);
        double a = ec / rr - 2.0 * xi * ex / SQRTPI;
        double b = ec / rr + 2.0 * xi * ex / SQRTPI;
        double da = -ec / r2 - 2.0 * xi * ex / (SQRTPI * rr) + 4.0 * xi * xi * xi * rr * ex / SQRTPI;
        double db = -ec / r2 - 2.0 * xi * ex / (SQRTPI * rr) - 4.0 * xi * xi * xi * rr * ex / SQRTPI;
        A = a; dA = da;
        Bc = b / r2; dB = db / r2 - 2.0 * b / (r2 * rr);
    }
    double wf = dot3(w, f), wr = dot3(w, r), fr = dot3(f, r);
    for (int k = 0; k < 3; ++k)
        g[k] += dA * r[k] / rr * wf + dB * r[k] / rr * wr * fr + Bc * (w[k] * fr + f[k] * wr);
}

/* grad_r (w . Omega(r) f) = grad_r [psi(r) r.(w x f)] */
static void grad_rotlet(int real, double xi, const double r[3], const double *w,
                        const double *f, double g[3]) {
    double r2 = dot3(r, r), rr = sqrt(r2);
    double psi, dpsi;
    if (!real) {
        psi = 1.0 / (r2 * rr); dpsi = -3.0 / (r2 * r2);
    } else {
        double ec = erfc(xi * rr), ex = exp(-xi * xi * r2);
        double rho = ec / r2 + 2.0 * xi * ex / (SQRTPI * rr);
        /* rho' = -2 erfc/r^3 - 2xi e/(sqrt(pi) r^2) - 2xi e/(sqrt(pi) r^2) - 4 xi^3 e/sqrt(pi) */
        double drho = -2.0 * ec / (r2 * rr) - 4.0 * xi * ex / (SQRTPI * r2) - 4.0 * xi * xi * xi * ex / SQRTPI;
        psi = rho / rr; dpsi = drho / rr - rho / r2;
    }
    double wxf[3] = {w[1] * f[2] - w[2] * f[1], w[2] * f[0] - w[0] * f[2], w[0] * f[1] - w[1] * f[0]};
    double rw = dot3(r, wxf);
    for (int k = 0; k < 3; ++k) g[k] += dpsi * r[k] / rr * rw + psi * wxf[k];
}

static int grad_generic(int real, int kernel, double xi, double rc, int64_t n,
                        const double *x, const double *f, const double *w, int64_t nt,
                        const int64_t *tgt, double *out) {
    if (kernel != 0 && kernel != 2) return 1;
    double sgn = kernel == 0 ? 1.0 : -1.0;
    double rc2 = rc * rc;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t t = 0; t < nt; ++t) {
        int64_t p = tgt[t];
        double g[3] = {0, 0, 0};
        const double *xp = x + 3 * p;
        for (int64_t s = 0; s < n; ++s) {
            if (s == p) continue;
            double r[3] = {xp[0] - x[3 * s], xp[1] - x[3 * s + 1], xp[2] - x[3 * s + 2]};
            double r2 = dot3(r, r);
            if (r2 == 0.0) { bad = 1; continue; }
            if (real && r2 > rc2) continue;
            double g1[3] = {0, 0, 0}, g2[3] = {0, 0, 0};
            if (kernel == 0) {
                grad_stokeslet(real, xi, r, w + 3 * p, f + 3 * s, g1);
                grad_stokeslet(real, xi, r, w + 3 * s, f + 3 * p, g2);
            } else {
                grad_rotlet(real, xi, r, w + 3 * p, f + 3 * s, g1);
                grad_rotlet(real, xi, r, w + 3 * s, f + 3 * p, g2);
            }
            for (int k = 0; k < 3; ++k) g[k] += g1[k] + sgn * g2[k];
        }
        out[3 * t] = g[0];
        out[3 * t + 1] = g[1];
        out[3 * t + 2] = g[2];
    }
    return bad ? 2 : 0;
}

int oracle_grad_direct(int kernel, int64_t n, const double *x, const double *f, const double *w,
                       int64_t nt, const int64_t *tgt, double *out) {
    return grad_generic(0, kernel, 0.0, 0.0, n, x, f, w, nt, tgt, out);
}

int oracle_grad_real_trunc(int kernel, double xi, double rc, int64_t n, const double *x,
                           const double *f, const double *w, int64_t nt, const int64_t *tgt,
                           double *out) {
    return grad_generic(1, kernel, xi, rc, n, x, f, w, nt, tgt, out);
}

/* Threads of the OpenMP loops above (t <= 0: the runtime default).  Timing only. */
void oracle_set_threads(int t) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    extern int omp_get_num_procs(void);
    omp_set_num_threads(t > 0 ? t : omp_get_num_procs());
#else
    (void)t;
#endif
}

int oracle_num_threads(void) {
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}
