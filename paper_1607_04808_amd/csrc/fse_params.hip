// Parameter selection (host) and the bounding-box default.
//
// Truncation-error estimates: Table est_real (Section 7.2: the RMS over targets
// of the neglected real-space interactions beyond r_c) and Table est_fourier
// (Section 7.1: the RMS of the wavenumbers beyond k_inf = pi/h, with the
// truncation radius R = sqrt(3) Lt of Section 4.1).  Selection follows the
// strategy of Section 8.2: for a given xi the estimates give r_c and M for an
// absolute tolerance; P follows the observed digits-per-support rule (P = 16
// for 8 digits, 24 for 12); xi, which only moves work between the real-space
// and Fourier parts, is the minimiser of a per-dtype cost model of this
// implementation's kernels over a geometric sweep with xi r_c and M / xi
// following the estimates.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fse_common.h"

namespace fse {

namespace {

constexpr double PI = 3.14159265358979323846;

// est_real, Table est_real
double est_real(int kernel, double Q, double xi, double L, double rc) {
    const double e = exp(-xi * xi * rc * rc);
    if (kernel == FSE_STOKESLET) return sqrt(4.0 * Q * rc / (L * L * L)) * e;
    if (kernel == FSE_STRESSLET) return sqrt(112.0 * Q * pow(xi, 4) * pow(rc, 3) / (9.0 * L * L * L)) * e;
    return sqrt(8.0 * Q / (3.0 * L * L * L * rc)) * e;
}

// est_fourier, Table est_fourier (kinf = pi / h, R = sqrt(3) Lt)
double est_fourier(int kernel, double Q, double xi, double L, double kinf, double R) {
    const double e = exp(-kinf * kinf / (4.0 * xi * xi));
    if (kernel == FSE_STOKESLET) return sqrt(Q) * R * pow(kinf, 3) / (xi * xi * PI * L) * e;
    if (kernel == FSE_STRESSLET) return sqrt(7.0 * Q / 6.0) * R * pow(kinf, 4) / (xi * xi * PI * L) * e;
    return sqrt(8.0 * xi * xi * Q / (3.0 * PI * L * L * L * kinf)) * e;
}

bool smooth7(int n) {
    if (n <= 0) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Cost model of one forward + adjoint evaluation (seconds), fitted to the kernel
// times of this implementation on MI355X: per real-space pair within r_c, per
// node and component of the (2 Mt)^3 transforms (two chains), and per point and
// window node (spreading twice, value and gradient quadrature).
struct CostModel { double pair, fft, node; };
constexpr CostModel COST_F32 = {7.8e-12, 6.0e-12, 2.8e-12};
constexpr CostModel COST_F64 = {2.1e-11, 2.7e-11, 5.0e-12};

// Scale of the result when the caller gives none: u_rms^2 ~ (Q / L^3) times
// the integral over the box of the component-averaged squared kernel, cut at the
// mean neighbour distance (stokeslet: 2/r^2, whose integral runs to ~0.55 L;
// rotlet (2/3)/r^4 and stresslet 4/r^4, dominated by near neighbours).
double u_rms_uniform(int kernel, int64_t n, double Q, double L) {
    const double rnn = 0.55 * L / cbrt((double)n);
    if (kernel == FSE_STOKESLET) return sqrt(8.0 * PI * 0.55 * L * Q / (L * L * L));
    if (kernel == FSE_STRESSLET) return sqrt(16.0 * PI / rnn * Q / (L * L * L));
    return sqrt(8.0 * PI / 3.0 / rnn * Q / (L * L * L));
}

// Per-block minima and maxima of the three coordinates (FP64): part[6 b + d] =
// min, part[6 b + 3 + d] = max over the block's grid-stride share of points.
template <typename T>
__global__ __launch_bounds__(256) void k_bbox(const T* __restrict__ x, int64_t n, double* part) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double v = (double)x[3 * i + d];
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], __shfl_xor(lo[d], o, 64));
            hi[d] = fmax(hi[d], __shfl_xor(hi[d], o, 64));
        }
    __shared__ double s[4][6];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int d = 0; d < 3; ++d) {
            s[w][d] = lo[d];
            s[w][3 + d] = hi[d];
        }
    __syncthreads();
    if (threadIdx.x < 6) {
        double v = s[0][threadIdx.x];
        for (int k = 1; k < 4; ++k) v = threadIdx.x < 3 ? fmin(v, s[k][threadIdx.x]) : fmax(v, s[k][threadIdx.x]);
        part[6 * blockIdx.x + threadIdx.x] = v;
    }
}

template <typename T>
fse_status_t bounding_box(const T* x, int64_t n, hipStream_t st, double* lo, double* hi) {
    const int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    double* part = nullptr;
    if (hipMalloc(&part, (size_t)nb * 6 * sizeof(double)) != hipSuccess) return FSE_ENOMEM;
    std::vector<double> h((size_t)nb * 6);
    hipLaunchKernelGGL(k_bbox<T>, dim3(nb), dim3(256), 0, st, x, n, part);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(part);
    if (e != hipSuccess) return FSE_EHIP;
    for (int d = 0; d < 3; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    for (int b = 0; b < nb; ++b)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], h[6 * b + d]);
            hi[d] = std::max(hi[d], h[6 * b + 3 + d]);
        }
    return FSE_OK;
}

}  // namespace

}  // namespace fse

using namespace fse;

extern "C" {

fse_status_t fse_error_estimates(fse_kernel_t kernel, const fse_params_t* params, double Q, double* est_r,
                                 double* est_f) {
    fse_geometry_t g;
    const fse_status_t st = fse_geometry(kernel, params, &g);
    if (st != FSE_OK) return st;
    if (!(Q >= 0)) { set_error("Q must be >= 0"); return FSE_EINVAL; }
    if (est_r) *est_r = est_real((int)kernel, Q, params->xi, params->L, params->rc);
    if (est_f) *est_f = est_fourier((int)kernel, Q, params->xi, params->L, g.kinf, g.R);
    return FSE_OK;
}

fse_status_t fse_choose_params(fse_kernel_t kernel, fse_dtype_t dtype, int64_t n, const double box_lo[3], double L,
                               double rel_tol, double Q, double u_rms, fse_params_t* out) {
    if (!out || !box_lo) { set_error("null argument"); return FSE_EINVAL; }
    if (kernel < FSE_STOKESLET || kernel > FSE_ROTLET || (dtype != FSE_F32 && dtype != FSE_F64)) {
        set_error("unknown kernel or dtype");
        return FSE_EINVAL;
    }
    if (n < 2 || !(L > 0) || !isfinite(L) || !(Q > 0) || !isfinite(Q)) {
        set_error("need n >= 2, L > 0 and Q > 0 (finite)");
        return FSE_EINVAL;
    }
    if (!(rel_tol > 0) || !(rel_tol < 1)) { set_error("rel_tol must be in (0, 1)"); return FSE_EINVAL; }
    if (dtype == FSE_F32 && rel_tol < 1e-6) {
        set_error("rel_tol %.1e is below what the FP32 form reaches (1e-6); use FSE_F64", rel_tol);
        return FSE_EINVAL;
    }
    if (!(u_rms > 0)) u_rms = u_rms_uniform((int)kernel, n, Q, L);
    // Absolute RMS target of the estimates: the relative max-norm error measured
    // here stays near the estimates' relative RMS (the estimates are pessimistic
    // by about the factor by which the max exceeds the RMS), so the total is held
    // at 0.6 tol (FP64; the margin covers the adjoint's gradient, whose error runs
    // about twice the value's) or 0.4 tol (FP32, leaving room for rounding as
    // well), split equally between the two parts.
    const double share = dtype == FSE_F32 ? 0.4 : 0.6;
    const double eps = rel_tol * share * u_rms / sqrt(2.0);
    // Gaussian support: 2 points per digit (Section 8.2: 16 for 8 digits, 24 for 12)
    int P = (int)ceil(-2.0 * log10(rel_tol) - 1e-9);
    if (P % 2) ++P;
    P = std::min(32, std::max(8, P));
    const double C = 0.976, m = C * sqrt(PI * P);
    const CostModel cm = dtype == FSE_F32 ? COST_F32 : COST_F64;
    const double rho = (double)n / (L * L * L);
    const int cin = kernel == FSE_STRESSLET ? 6 : 3;  // grid components spread
    const int mt_max = fft_max_mt((int)kernel, dtype == FSE_F32 ? 4 : 8);
    bool found = false;
    double best = 0;
    fse_params_t bp{};
    for (int it = 0; it <= 400; ++it) {
        const double xi = (1.0 / L) * pow(10.0, 3.0 * it / 400.0);  // 1/L .. 1000/L
        // r_c: est_real decreases in r_c (bisection on (0, L])
        double lo = 1e-9 * L, hi = L;
        if (est_real((int)kernel, Q, xi, L, hi) > eps) continue;
        for (int k = 0; k < 100; ++k) {
            const double mid = 0.5 * (lo + hi);
            (est_real((int)kernel, Q, xi, L, mid) > eps ? lo : hi) = mid;
        }
        const double rc = hi;
        // M: the smallest grid meeting est_fourier, with R = sqrt(3) Lt of the grid it
        // gives (Mt: the box extended by eq. deltaL_cond's deltaL, 2 Mt 7-smooth), and
        // with eta = (xi h P / m)^2 <= 0.95 (FP64) or 0.7 (FP32), so that Section 5.3's
        // scaling factor stays a decay (this also keeps k_inf / xi >= sqrt(pi P) / C,
        // where the estimate of Section 7.1 holds).  deltaL = d alone leaves the
        // remainder Gaussians of Section 5.3 cut at the box edge, an error that the
        // estimate does not see and that shows at the targets near the faces.
        const double eta_max = dtype == FSE_F32 ? 0.7 : 0.95;
        const int Meta = (int)ceil(xi * L * P / (m * sqrt(eta_max)));
        int M = 0, Mt = 0;
        for (int Mc = std::max(4, Meta); Mc <= mt_max; ++Mc) {
            const double h = L / Mc;
            const double eta = (xi * h * P / m) * (xi * h * P / m);
            const double dL = std::max(h * P, sqrt(2.0 * (1.0 - eta) * m * m) / xi);
            int Mtc = Mc + (int)ceil(dL / h - 1e-12);
            while (!smooth7(2 * Mtc)) ++Mtc;
            if (est_fourier((int)kernel, Q, xi, L, PI / h, sqrt(3.0) * Mtc * h) <= eps) {
                M = Mc;
                Mt = Mtc;
                break;
            }
        }
        if (M == 0 || Mt > mt_max) continue;
        const double pairs = (double)n * rho * 4.0 / 3.0 * PI * rc * rc * rc;
        const double nf = 2.0 * Mt;
        // transforms: cin components forward, 3 back, in each of the two chains
        const double cost = cm.pair * pairs + cm.fft * nf * nf * nf * (cin + 3) +
                            cm.node * (double)n * P * P * P;
        if (!found || cost < best) {
            found = true;
            best = cost;
            bp.xi = xi;
            bp.rc = rc;
            bp.M = M;
            bp.P = P;
            bp.Mt = Mt;
        }
    }
    if (!found) {
        set_error("no parameters meet rel_tol %.1e within the grid limit (Mt <= %d)", rel_tol, mt_max);
        return FSE_EINVAL;
    }
    for (int d = 0; d < 3; ++d) bp.box_lo[d] = box_lo[d];
    bp.L = L;
    bp.deltaL_rule = 1;
    bp.C = 0.0;
    *out = bp;
    return FSE_OK;
}

fse_status_t fse_bounding_box(fse_dtype_t dtype, int64_t n, const void* x, void* stream, double box_lo[3],
                              double* L) {
    if (!x || !box_lo || !L || n < 1 || (dtype != FSE_F32 && dtype != FSE_F64)) {
        set_error("bad argument");
        return FSE_EINVAL;
    }
    double lo[3], hi[3];
    const fse_status_t st = dtype == FSE_F32 ? bounding_box<float>((const float*)x, n, (hipStream_t)stream, lo, hi)
                                             : bounding_box<double>((const double*)x, n, (hipStream_t)stream, lo, hi);
    if (st != FSE_OK) {
        set_error("bounding box: device reduction failed");
        return st;
    }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        if (!isfinite(lo[d]) || !isfinite(hi[d])) {
            set_error("a coordinate is not finite");
            return FSE_ERANGE;
        }
        ext = std::max(ext, hi[d] - lo[d]);
        box_lo[d] = lo[d];
    }
    // the largest coordinate must lie strictly inside the half-open cube
    *L = ext > 0 ? ext * (1.0 + 1.0 / 1048576.0) : 1.0;
    return FSE_OK;
}

}  // extern "C"
