// Real-space part (Section 6): u^R(x_m) = sum_{0 < |x_m - x_n| <= rc} G^R(x_m - x_n) . f_n
// over a cell list of cells with side >= rc (27 neighbour cells), plus the
// stokeslet self term -4 xi/sqrt(pi) f_m (eq. Slimit).
//
// G^R (Section 3.2):
//   stokeslet  eq. SR_Op:  (erfc/r - 2 xi e/sqrt(pi)) d_jl + (erfc/r + 2 xi e/sqrt(pi)) rh_j rh_l
//   stresslet  eq. TR_Op:  A1 rh_j rh_l rh_m + A2 (d_jl rh_m + d_lm rh_j + d_mj rh_l),
//              A1 = -(2/r)(3 erfc/r + 2 xi/sqrt(pi) (3 + 2 xi^2 r^2) e),
//              A2 = 4 xi^3 r e / sqrt(pi)   (the factor r required by eq. TR2int)
//   rotlet     eps_jlm rh_m (erfc/r^2 + 2 xi e/(sqrt(pi) r)): eq. RR_Op under the
//              eq. def_rotlet normalisation (half of its operator-form factor 2)
// with e = exp(-xi^2 r^2), erfc = erfc(xi r).
//
// One workgroup per cell: one thread per target, source chunks of the 27
// neighbour cells staged in LDS.  Points are in cell order, so each chunk is a
// contiguous, coalesced read.
#include "fse_common.h"

namespace fse {

namespace {

constexpr double INV_SQRTPI = 0.56418958354775628695;

template <typename T> __device__ __forceinline__ T derfc(T x);
template <> __device__ __forceinline__ float derfc<float>(float x) { return erfcf(x); }
template <> __device__ __forceinline__ double derfc<double>(double x) { return erfc(x); }
template <typename T> __device__ __forceinline__ T dexpr(T x);
template <> __device__ __forceinline__ float dexpr<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double dexpr<double>(double x) { return exp(x); }

template <typename T, int KERNEL, int NB>
__global__ __launch_bounds__(256) void k_real(CellGeo cg, const int* __restrict__ cell_start,
                                             const T* __restrict__ x_r, const T* __restrict__ a_r,
                                             const T* __restrict__ b_r, int64_t n, int batch, T xi,
                                             T self_coef, const int* __restrict__ perm_r, T* u,
                                             int accumulate) {
    constexpr int CH = 256;
    constexpr int NS = (KERNEL == FSE_STRESSLET) ? 6 : 3;  // source values per point per batch
    __shared__ T xs[CH * 3];
    __shared__ T ss[NB][CH * NS];
    const int nc = cg.ncell;
    const int cell = blockIdx.x;
    const int cx = cell % nc, cy = (cell / nc) % nc, cz = cell / (nc * nc);
    const int b0 = blockIdx.y * NB;
    const int t0 = cell_start[cell], t1 = cell_start[cell + 1];
    const T rc2 = (T)cg.rc2;
    const T xi2 = xi * xi;
    const T c2x = (T)(2.0 * INV_SQRTPI) * xi;       // 2 xi / sqrt(pi)
    const T c4x3 = (T)(4.0 * INV_SQRTPI) * xi * xi2;  // 4 xi^3 / sqrt(pi)
    for (int tb = t0; tb < t1; tb += CH) {
        const int j = tb + (int)threadIdx.x;
        const bool act = j < t1;
        T xt0 = 0, xt1 = 0, xt2 = 0;
        if (act) {
            xt0 = x_r[3 * (int64_t)j];
            xt1 = x_r[3 * (int64_t)j + 1];
            xt2 = x_r[3 * (int64_t)j + 2];
        }
        T acc[NB][3];
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[b][0] = acc[b][1] = acc[b][2] = (T)0;
        for (int dz = -1; dz <= 1; ++dz) {
            const int nz = cz + dz;
            if (nz < 0 || nz >= nc) continue;
            for (int dy = -1; dy <= 1; ++dy) {
                const int ny = cy + dy;
                if (ny < 0 || ny >= nc) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int nx = cx + dx;
                    if (nx < 0 || nx >= nc) continue;
                    const int nb = (nz * nc + ny) * nc + nx;
                    const int s0 = cell_start[nb], s1 = cell_start[nb + 1];
                    for (int sb = s0; sb < s1; sb += CH) {
                        __syncthreads();
                        const int k = sb + (int)threadIdx.x;
                        if (k < s1) {
                            xs[3 * threadIdx.x] = x_r[3 * (int64_t)k];
                            xs[3 * threadIdx.x + 1] = x_r[3 * (int64_t)k + 1];
                            xs[3 * threadIdx.x + 2] = x_r[3 * (int64_t)k + 2];
#pragma unroll
                            for (int b = 0; b < NB; ++b) {
                                if (b0 + b < batch) {
                                    const T* ap = a_r + ((int64_t)(b0 + b) * n + k) * 3;
#pragma unroll
                                    for (int d = 0; d < 3; ++d) ss[b][NS * threadIdx.x + d] = ap[d];
                                    if (NS == 6) {
                                        const T* bp = b_r + ((int64_t)(b0 + b) * n + k) * 3;
#pragma unroll
                                        for (int d = 0; d < 3; ++d) ss[b][NS * threadIdx.x + 3 + d] = bp[d];
                                    }
                                }
                            }
                        }
                        __syncthreads();
                        if (!act) continue;
                        const int cnt = min(CH, s1 - sb);
                        for (int kk = 0; kk < cnt; ++kk) {
                            const T r0 = xt0 - xs[3 * kk], r1 = xt1 - xs[3 * kk + 1], r2v = xt2 - xs[3 * kk + 2];
                            const T r2 = r0 * r0 + r1 * r1 + r2v * r2v;
                            if (r2 > rc2 || sb + kk == j) continue;
                            const T r = sqrt(r2);
                            const T ir = (T)1 / r;
                            const T e = dexpr<T>(-xi2 * r2);
                            const T ec = derfc<T>(xi * r);
                            if constexpr (KERNEL == FSE_STOKESLET) {
                                const T cd = ec * ir - c2x * e;
                                const T c1 = (ec * ir + c2x * e) * ir * ir;  // on r r^T
#pragma unroll
                                for (int b = 0; b < NB; ++b) {
                                    const T* f = &ss[b][3 * kk];
                                    const T rf = (r0 * f[0] + r1 * f[1] + r2v * f[2]) * c1;
                                    acc[b][0] += cd * f[0] + rf * r0;
                                    acc[b][1] += cd * f[1] + rf * r1;
                                    acc[b][2] += cd * f[2] + rf * r2v;
                                }
                            } else if constexpr (KERNEL == FSE_ROTLET) {
                                const T c = (ec * ir * ir + c2x * e * ir) * ir;  // on f x r
#pragma unroll
                                for (int b = 0; b < NB; ++b) {
                                    const T* f = &ss[b][3 * kk];
                                    acc[b][0] += c * (f[1] * r2v - f[2] * r1);
                                    acc[b][1] += c * (f[2] * r0 - f[0] * r2v);
                                    acc[b][2] += c * (f[0] * r1 - f[1] * r0);
                                }
                            } else {
                                const T A1 = -(T)2 * ir * ((T)3 * ec * ir + c2x * ((T)3 + (T)2 * xi2 * r2) * e);
                                const T A2 = c4x3 * r * e;
                                const T h0 = r0 * ir, h1 = r1 * ir, h2 = r2v * ir;
#pragma unroll
                                for (int b = 0; b < NB; ++b) {
                                    const T* q = &ss[b][6 * kk];
                                    const T* nn = q + 3;
                                    const T hq = h0 * q[0] + h1 * q[1] + h2 * q[2];
                                    const T hn = h0 * nn[0] + h1 * nn[1] + h2 * nn[2];
                                    const T nq = nn[0] * q[0] + nn[1] * q[1] + nn[2] * q[2];
                                    const T s1c = A1 * hn * hq + A2 * nq;
                                    acc[b][0] += s1c * h0 + A2 * (nn[0] * hq + q[0] * hn);
                                    acc[b][1] += s1c * h1 + A2 * (nn[1] * hq + q[1] * hn);
                                    acc[b][2] += s1c * h2 + A2 * (nn[2] * hq + q[2] * hn);
                                }
                            }
                        }
                    }
                }
            }
        }
        if (act) {
            const int64_t i = perm_r[j];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b0 + b >= batch) break;
                T* o = u + ((int64_t)(b0 + b) * n + i) * 3;
                const T* a = a_r + ((int64_t)(b0 + b) * n + j) * 3;
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const T prev = accumulate ? o[d] : (T)0;
                    o[d] = prev + acc[b][d] + self_coef * a[d];
                }
            }
        }
    }
}

// Real-space gradient of L = sum_b sum_m w_bm . u^R_b(x_m):
//   dx_p += sum_{0<|r|<=rc} sum_b [ grad_r(w_bp . G^R(r) f_bn) + s grad_r(w_bn . G^R(r) f_bp) ],
// r = x_p - x_n, s = +1 for the even stokeslet, -1 for the odd rotlet.
template <typename T, int KERNEL>
__global__ __launch_bounds__(256) void k_real_grad(CellGeo cg, const int* __restrict__ cell_start,
                                                  const T* __restrict__ x_r, const T* __restrict__ f_r,
                                                  const T* __restrict__ w_r, int64_t n, int batch, T xi,
                                                  const int* __restrict__ perm_r, T* dx) {
    constexpr int CH = 128;
    __shared__ T xs[CH * 3];
    __shared__ T fs[CH * 3];
    __shared__ T ws[CH * 3];
    const int nc = cg.ncell;
    const int cell = blockIdx.x;
    const int cx = cell % nc, cy = (cell / nc) % nc, cz = cell / (nc * nc);
    const int t0 = cell_start[cell], t1 = cell_start[cell + 1];
    const T rc2 = (T)cg.rc2;
    const T xi2 = xi * xi;
    const T c2x = (T)(2.0 * INV_SQRTPI) * xi;
    const T c4x3 = (T)(4.0 * INV_SQRTPI) * xi * xi2;
    const T sgn = (KERNEL == FSE_STOKESLET) ? (T)1 : (T)-1;
    for (int tb = t0; tb < t1; tb += CH) {
        const int j = tb + (int)threadIdx.x;
        const bool act = (int)threadIdx.x < CH && j < t1;
        T xt0 = 0, xt1 = 0, xt2 = 0;
        if (act) {
            xt0 = x_r[3 * (int64_t)j];
            xt1 = x_r[3 * (int64_t)j + 1];
            xt2 = x_r[3 * (int64_t)j + 2];
        }
        T g0 = 0, g1 = 0, g2 = 0;
        for (int bm = 0; bm < batch; ++bm) {
            T fp[3] = {0, 0, 0}, wp[3] = {0, 0, 0};
            if (act) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    fp[d] = f_r[((int64_t)bm * n + j) * 3 + d];
                    wp[d] = w_r[((int64_t)bm * n + j) * 3 + d];
                }
            }
            for (int dz = -1; dz <= 1; ++dz) {
                const int nz = cz + dz;
                if (nz < 0 || nz >= nc) continue;
                for (int dy = -1; dy <= 1; ++dy) {
                    const int ny = cy + dy;
                    if (ny < 0 || ny >= nc) continue;
                    for (int ddx = -1; ddx <= 1; ++ddx) {
                        const int nx = cx + ddx;
                        if (nx < 0 || nx >= nc) continue;
                        const int nb = (nz * nc + ny) * nc + nx;
                        const int s0 = cell_start[nb], s1 = cell_start[nb + 1];
                        for (int sb = s0; sb < s1; sb += CH) {
                            __syncthreads();
                            const int k = sb + (int)threadIdx.x;
                            if ((int)threadIdx.x < CH && k < s1) {
#pragma unroll
                                for (int d = 0; d < 3; ++d) {
                                    xs[3 * threadIdx.x + d] = x_r[3 * (int64_t)k + d];
                                    fs[3 * threadIdx.x + d] = f_r[((int64_t)bm * n + k) * 3 + d];
                                    ws[3 * threadIdx.x + d] = w_r[((int64_t)bm * n + k) * 3 + d];
                                }
                            }
                            __syncthreads();
                            if (!act) continue;
                            const int cnt = min(CH, s1 - sb);
                            for (int kk = 0; kk < cnt; ++kk) {
                                const T r[3] = {xt0 - xs[3 * kk], xt1 - xs[3 * kk + 1], xt2 - xs[3 * kk + 2]};
                                const T r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                                if (r2 > rc2 || sb + kk == j) continue;
                                const T rr = sqrt(r2);
                                const T ir = (T)1 / rr;
                                const T e = dexpr<T>(-xi2 * r2);
                                const T ec = derfc<T>(xi * rr);
                                const T* fn = &fs[3 * kk];
                                const T* wn = &ws[3 * kk];
                                if constexpr (KERNEL == FSE_STOKESLET) {
                                    // w.S^R f = A (w.f) + Bc (w.r)(f.r), A = a(r), Bc = b(r)/r^2
                                    const T a_ = ec * ir - c2x * e;
                                    const T b_ = ec * ir + c2x * e;
                                    const T da = -ec * ir * ir - c2x * e * ir + c4x3 * rr * e;
                                    const T db = -ec * ir * ir - c2x * e * ir - c4x3 * rr * e;
                                    const T Bc = b_ * ir * ir;
                                    const T dB = db * ir * ir - (T)2 * b_ * ir * ir * ir;
                                    (void)a_;
                                    // term 1: (w_p, f_n); term 2: (w_n, f_p) with sign sgn
                                    const T wf1 = wp[0] * fn[0] + wp[1] * fn[1] + wp[2] * fn[2];
                                    const T wr1 = wp[0] * r[0] + wp[1] * r[1] + wp[2] * r[2];
                                    const T fr1 = fn[0] * r[0] + fn[1] * r[1] + fn[2] * r[2];
                                    const T wf2 = wn[0] * fp[0] + wn[1] * fp[1] + wn[2] * fp[2];
                                    const T wr2 = wn[0] * r[0] + wn[1] * r[1] + wn[2] * r[2];
                                    const T fr2 = fp[0] * r[0] + fp[1] * r[1] + fp[2] * r[2];
                                    const T rad = (da * (wf1 + sgn * wf2) + dB * (wr1 * fr1 + sgn * wr2 * fr2)) * ir;
                                    g0 += rad * r[0] + Bc * (wp[0] * fr1 + fn[0] * wr1 + sgn * (wn[0] * fr2 + fp[0] * wr2));
                                    g1 += rad * r[1] + Bc * (wp[1] * fr1 + fn[1] * wr1 + sgn * (wn[1] * fr2 + fp[1] * wr2));
                                    g2 += rad * r[2] + Bc * (wp[2] * fr1 + fn[2] * wr1 + sgn * (wn[2] * fr2 + fp[2] * wr2));
                                } else {
                                    // w.Omega^R f = psi(r) r.(w x f), psi = rho/r
                                    const T rho = ec * ir * ir + c2x * e * ir;
                                    const T drho = -(T)2 * ec * ir * ir * ir - (T)2 * c2x * e * ir * ir - c4x3 * e;
                                    const T psi = rho * ir;
                                    const T dpsi = drho * ir - rho * ir * ir;
                                    const T c1[3] = {wp[1] * fn[2] - wp[2] * fn[1], wp[2] * fn[0] - wp[0] * fn[2],
                                                     wp[0] * fn[1] - wp[1] * fn[0]};
                                    const T c2[3] = {wn[1] * fp[2] - wn[2] * fp[1], wn[2] * fp[0] - wn[0] * fp[2],
                                                     wn[0] * fp[1] - wn[1] * fp[0]};
                                    const T cc[3] = {c1[0] + sgn * c2[0], c1[1] + sgn * c2[1], c1[2] + sgn * c2[2]};
                                    const T rc = (r[0] * cc[0] + r[1] * cc[1] + r[2] * cc[2]) * dpsi * ir;
                                    g0 += rc * r[0] + psi * cc[0];
                                    g1 += rc * r[1] + psi * cc[1];
                                    g2 += rc * r[2] + psi * cc[2];
                                }
                            }
                        }
                    }
                }
            }
        }
        if (act) {
            const int64_t i = perm_r[j];
            dx[3 * i] += g0;
            dx[3 * i + 1] += g1;
            dx[3 * i + 2] += g2;
        }
    }
}

}  // namespace

template <typename T>
void launch_real(int kernel, const CellGeo& c, const PointsDev<T>& p, const T* src_a_r,
                 const T* src_b_r, int batch, double xi, double self_coef, T* u, int accumulate,
                 hipStream_t st) {
    const unsigned ncells = (unsigned)c.ncell * c.ncell * c.ncell;
    const int NBc = batch == 1 ? 1 : 4;
    dim3 grd(ncells, (batch + NBc - 1) / NBc);
#define LAUNCH(K, NB)                                                                                \
    hipLaunchKernelGGL((k_real<T, K, NB>), grd, dim3(256), 0, st, c, p.cell_start, p.x_r, src_a_r, \
                       src_b_r, p.n, batch, (T)xi, (T)self_coef, p.perm_r, u, accumulate)
    if (kernel == FSE_STOKESLET) {
        if (NBc == 1) LAUNCH(FSE_STOKESLET, 1); else LAUNCH(FSE_STOKESLET, 4);
    } else if (kernel == FSE_ROTLET) {
        if (NBc == 1) LAUNCH(FSE_ROTLET, 1); else LAUNCH(FSE_ROTLET, 4);
    } else {
        if (NBc == 1) LAUNCH(FSE_STRESSLET, 1); else LAUNCH(FSE_STRESSLET, 4);
    }
#undef LAUNCH
}

template <typename T>
void launch_real_grad(int kernel, const CellGeo& c, const PointsDev<T>& p, const T* f_r, const T* w_r,
                      int batch, double xi, T* dx, hipStream_t st) {
    const unsigned ncells = (unsigned)c.ncell * c.ncell * c.ncell;
    if (kernel == FSE_STOKESLET)
        hipLaunchKernelGGL((k_real_grad<T, FSE_STOKESLET>), dim3(ncells), dim3(128), 0, st, c,
                           p.cell_start, p.x_r, f_r, w_r, p.n, batch, (T)xi, p.perm_r, dx);
    else
        hipLaunchKernelGGL((k_real_grad<T, FSE_ROTLET>), dim3(ncells), dim3(128), 0, st, c,
                           p.cell_start, p.x_r, f_r, w_r, p.n, batch, (T)xi, p.perm_r, dx);
}

#define INST(T)                                                                                     \
    template void launch_real<T>(int, const CellGeo&, const PointsDev<T>&, const T*, const T*, int, \
                                 double, double, T*, int, hipStream_t);                             \
    template void launch_real_grad<T>(int, const CellGeo&, const PointsDev<T>&, const T*, const T*, \
                                      int, double, T*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace fse
