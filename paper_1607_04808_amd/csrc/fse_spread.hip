// Gaussian gridding (Section 5.2): step 1 "spreading" (eq. Hx) and step 5
// "quadrature" (eq. u_integr, trapezoidal rule), with Gaussians truncated to a
// P^3 cube of grid points (fast Gaussian gridding).  The weights here are the
// raw factors exp(-alpha |x_node - x|^2) = prod_d exp(-alpha h^2 (t_d - i_d)^2);
// the normalisations (alpha/pi)^{3/2} of both steps and the quadrature weight
// h^3 are folded into the precomputed Fourier multiplier.
//
// Spreading: one workgroup owns a TS^3 tile of grid nodes and accumulates in
// LDS the contributions of every point whose window overlaps the tile (points
// binned by the tile of their window start, so at most (1+ceil((P-1)/TS))^3
// source tiles are visited).  Each node is written exactly once, coalesced, by
// its owner: no global atomics and no clearing of the grid.
#include "fse_common.h"

namespace fse {

namespace {

template <typename T> __device__ __forceinline__ T dexp(T x);
template <> __device__ __forceinline__ float dexp<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double dexp<double>(double x) { return exp(x); }

template <typename T, int NC, int TS>
__global__ __launch_bounds__(256) void k_spread(GridGeo g, const int* __restrict__ tile_start,
                                               const int* __restrict__ bpack_s,
                                               const T* __restrict__ coff_s,
                                               const T* __restrict__ src_s, int64_t n, T* grid) {
    constexpr int TS3 = TS * TS * TS;
    __shared__ T acc[NC * TS3];
    const int nt = g.nt, Mt = g.Mt, P = g.P;
    const int t = blockIdx.x;
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int bm = blockIdx.y;
    const int lox = tx * TS, loy = ty * TS, loz = tz * TS;
    for (int q = threadIdx.x; q < NC * TS3; q += 256) acc[q] = (T)0;
    __syncthreads();

    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const T ahh = (T)g.ahh;
    const T half = (T)(0.5 * (P - 1));
    const int kspan = (P - 1 + TS - 1) / TS;
    for (int sz = max(0, tz - kspan); sz <= tz; ++sz)
        for (int sy = max(0, ty - kspan); sy <= ty; ++sy)
            for (int sx = max(0, tx - kspan); sx <= tx; ++sx) {
                const int s = (sz * nt + sy) * nt + sx;
                const int j0 = tile_start[s], j1 = tile_start[s + 1];
                for (int j = j0 + wid; j < j1; j += 4) {
                    const int bp = bpack_s[j];
                    const int bx = bp & 1023, by = (bp >> 10) & 1023, bz = bp >> 20;
                    const int x0 = max(bx, lox), x1 = min(bx + P, lox + TS);
                    const int y0 = max(by, loy), y1 = min(by + P, loy + TS);
                    const int z0 = max(bz, loz), z1 = min(bz + P, loz + TS);
                    if (x0 >= x1 || y0 >= y1 || z0 >= z1) continue;
                    const T cx = coff_s[3 * (int64_t)j], cy = coff_s[3 * (int64_t)j + 1],
                            cz = coff_s[3 * (int64_t)j + 2];
                    // lane l holds the weight of window offset l in each dimension
                    const T ex = cx + half - (T)lane, ey = cy + half - (T)lane, ez = cz + half - (T)lane;
                    const T wx = dexp<T>(-ahh * ex * ex);
                    const T wy = dexp<T>(-ahh * ey * ey);
                    const T wz = dexp<T>(-ahh * ez * ez);
                    T wxs[TS];
#pragma unroll
                    for (int k = 0; k < TS; ++k) wxs[k] = readlane(wx, min(x0 - bx + k, 63));
                    T v[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) v[c] = src_s[((int64_t)bm * n + j) * NC + c];
                    const int nx = x1 - x0, ny = y1 - y0, nyz = ny * (z1 - z0);
                    const int xoff = x0 - lox;
                    for (int qb = 0; qb < nyz; qb += 64) {
                        const int q = qb + lane;
                        const bool act = q < nyz;
                        const int qq = act ? q : 0;
                        const int iy = y0 + qq % ny, iz = z0 + qq / ny;
                        const T wyz = __shfl(wy, iy - by, 64) * __shfl(wz, iz - bz, 64);
                        if (act) {
                            T* a = acc + ((iz - loz) * TS + (iy - loy)) * TS + xoff;
#pragma unroll
                            for (int k = 0; k < TS; ++k) {
                                if (k < nx) {
                                    const T w = wxs[k] * wyz;
#pragma unroll
                                    for (int c = 0; c < NC; ++c) atomicAdd(a + c * TS3 + k, w * v[c]);
                                }
                            }
                        }
                    }
                }
            }
    __syncthreads();
    const int64_t M3 = (int64_t)Mt * Mt * Mt;
    for (int q = threadIdx.x; q < TS3; q += 256) {
        const int lx = q % TS, ly = (q / TS) % TS, lz = q / (TS * TS);
        const int gx = lox + lx, gy = loy + ly, gz = loz + lz;
        if (gx < Mt && gy < Mt && gz < Mt) {
            const int64_t o = ((int64_t)gz * Mt + gy) * Mt + gx;
#pragma unroll
            for (int c = 0; c < NC; ++c) grid[((int64_t)bm * NC + c) * M3 + o] = acc[c * TS3 + q];
        }
    }
}

// Quadrature: one wave per point, LPR lanes along x per window row.
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_gather(GridGeo g, const int* __restrict__ tile_start,
                                               const int* __restrict__ perm_s,
                                               const int* __restrict__ bpack_s,
                                               const T* __restrict__ coff_s,
                                               const T* __restrict__ field, int64_t n, T* u) {
    __shared__ T wsh[4][2][32];
    constexpr int NG = 64 / LPR;
    const int Mt = g.Mt, P = g.P;
    const int64_t M3 = (int64_t)Mt * Mt * Mt;
    const int s = blockIdx.x, bm = blockIdx.y;
    const int j0 = tile_start[s], j1 = tile_start[s + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int gx = lane % LPR, grp = lane / LPR;
    const T ahh = (T)g.ahh;
    const T half = (T)(0.5 * (P - 1));
    const T* fb0 = field + (int64_t)bm * 3 * M3;
    for (int j = j0 + wid; j < j1; j += 4) {
        const int bp = bpack_s[j];
        const int bx = bp & 1023, by = (bp >> 10) & 1023, bz = bp >> 20;
        const T cx = coff_s[3 * (int64_t)j], cy = coff_s[3 * (int64_t)j + 1], cz = coff_s[3 * (int64_t)j + 2];
        const T ex = cx + half - (T)gx;
        const T wx = (gx < P) ? dexp<T>(-ahh * ex * ex) : (T)0;
        if (lane < P) {
            const T ey = cy + half - (T)lane, ez = cz + half - (T)lane;
            wsh[wid][0][lane] = dexp<T>(-ahh * ey * ey);
            wsh[wid][1][lane] = dexp<T>(-ahh * ez * ez);
        }
        wave_lds_sync();
        T a0 = 0, a1 = 0, a2 = 0;
        if (gx < P) {
            const T* fb = fb0 + ((int64_t)bz * Mt + by) * Mt + bx + gx;
            for (int iz = 0; iz < P; ++iz) {
                const T wz = wx * wsh[wid][1][iz];
                const T* fz = fb + (int64_t)iz * Mt * Mt;
                for (int iy = grp; iy < P; iy += NG) {
                    const T w = wz * wsh[wid][0][iy];
                    const T* f = fz + (int64_t)iy * Mt;
                    a0 += w * f[0];
                    a1 += w * f[M3];
                    a2 += w * f[2 * M3];
                }
            }
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        if (lane == 0) {
            const int64_t i = perm_s[j];
            T* o = u + ((int64_t)bm * n + i) * 3;
            o[0] = a0;
            o[1] = a1;
            o[2] = a2;
        }
        wave_lds_sync();
    }
}

// Adjoint quadrature.  For each point s and batch member b:
//   dsrc_b(x_s) = quadrature of phi_w,b  (the value, as k_gather), and
//   dx(x_s) += sum_p grad_x g(x_s - x_p) [w_b,s . phi_f,b(x_p) + f_b,s . phi_w,b(x_p)],
// the derivative of the Gaussian windows of both the spreading and the
// quadrature step (the discrete operator is symmetric for S and Omega).
template <typename T, int LPR>
__global__ __launch_bounds__(256) void k_gather_grad(GridGeo g, const int* __restrict__ tile_start,
                                                    const int* __restrict__ perm_s,
                                                    const int* __restrict__ bpack_s,
                                                    const T* __restrict__ coff_s,
                                                    const T* __restrict__ phi_f,
                                                    const T* __restrict__ phi_w,
                                                    const T* __restrict__ f_s,
                                                    const T* __restrict__ w_s, int64_t n, int batch,
                                                    T* dsrc, T* dx) {
    __shared__ T wsh[4][4][32];
    constexpr int NG = 64 / LPR;
    const int Mt = g.Mt, P = g.P;
    const int64_t M3 = (int64_t)Mt * Mt * Mt;
    const int s = blockIdx.x;
    const int j0 = tile_start[s], j1 = tile_start[s + 1];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int gx = lane % LPR, grp = lane / LPR;
    const T ahh = (T)g.ahh;
    const T dfac = (T)(-2.0 * g.ahh / g.h);  // d/dx exp(-alpha h^2 e^2) = dfac * e * exp(...)
    const T half = (T)(0.5 * (P - 1));
    for (int j = j0 + wid; j < j1; j += 4) {
        const int bp = bpack_s[j];
        const int bx = bp & 1023, by = (bp >> 10) & 1023, bz = bp >> 20;
        const T cx = coff_s[3 * (int64_t)j], cy = coff_s[3 * (int64_t)j + 1], cz = coff_s[3 * (int64_t)j + 2];
        const T ex = cx + half - (T)gx;
        const T wx = (gx < P) ? dexp<T>(-ahh * ex * ex) : (T)0;
        const T dwx = dfac * ex * wx;
        if (lane < P) {
            const T ey = cy + half - (T)lane, ez = cz + half - (T)lane;
            const T wy = dexp<T>(-ahh * ey * ey), wz = dexp<T>(-ahh * ez * ez);
            wsh[wid][0][lane] = wy;
            wsh[wid][1][lane] = wz;
            wsh[wid][2][lane] = dfac * ey * wy;
            wsh[wid][3][lane] = dfac * ez * wz;
        }
        wave_lds_sync();
        const int64_t i = perm_s[j];
        T gxs = 0, gys = 0, gzs = 0;
        for (int bm = 0; bm < batch; ++bm) {
            const T* wv = w_s + ((int64_t)bm * n + j) * 3;
            const T* fv = f_s + ((int64_t)bm * n + j) * 3;
            const T w0 = wv[0], w1 = wv[1], w2 = wv[2], f0 = fv[0], f1 = fv[1], f2 = fv[2];
            T v0 = 0, v1 = 0, v2 = 0, g0 = 0, g1 = 0, g2 = 0;
            if (gx < P) {
                const int64_t off = (int64_t)bm * 3 * M3 + ((int64_t)bz * Mt + by) * Mt + bx + gx;
                const T* pf = phi_f + off;
                const T* pw = phi_w + off;
                for (int iz = 0; iz < P; ++iz) {
                    const T wz = wsh[wid][1][iz], dwz = wsh[wid][3][iz];
                    for (int iy = grp; iy < P; iy += NG) {
                        const T wy = wsh[wid][0][iy], dwy = wsh[wid][2][iy];
                        const int64_t o = ((int64_t)iz * Mt + iy) * Mt;
                        const T pw0 = pw[o], pw1 = pw[o + M3], pw2 = pw[o + 2 * M3];
                        const T psi = w0 * pf[o] + w1 * pf[o + M3] + w2 * pf[o + 2 * M3] +
                                      f0 * pw0 + f1 * pw1 + f2 * pw2;
                        const T wyz = wy * wz;
                        const T w = wx * wyz;
                        v0 += w * pw0;
                        v1 += w * pw1;
                        v2 += w * pw2;
                        g0 += psi * dwx * wyz;
                        g1 += psi * wx * dwy * wz;
                        g2 += psi * wx * wy * dwz;
                    }
                }
            }
            v0 = wave_sum(v0);
            v1 = wave_sum(v1);
            v2 = wave_sum(v2);
            gxs += g0;
            gys += g1;
            gzs += g2;
            if (lane == 0 && dsrc) {
                T* o = dsrc + ((int64_t)bm * n + i) * 3;
                o[0] = v0;
                o[1] = v1;
                o[2] = v2;
            }
        }
        gxs = wave_sum(gxs);
        gys = wave_sum(gys);
        gzs = wave_sum(gzs);
        if (lane == 0 && dx) {
            dx[3 * i] = gxs;
            dx[3 * i + 1] = gys;
            dx[3 * i + 2] = gzs;
        }
        wave_lds_sync();
    }
}

inline unsigned ntiles(const GridGeo& g) { return (unsigned)(g.nt * g.nt * g.nt); }

}  // namespace

template <typename T>
void launch_spread(const GridGeo& g, const PointsDev<T>& p, const T* src_s, int c_in, int batch,
                   T* grid, hipStream_t st) {
    // tile side: 16 for FP32, 12 for FP64 (NC * TS^3 accumulators must fit in LDS)
    constexpr int TS = sizeof(T) == 4 ? 16 : 12;
    dim3 grd(ntiles(g), batch);
    if (c_in == 3)
        hipLaunchKernelGGL((k_spread<T, 3, TS>), grd, dim3(256), 0, st, g, p.tile_start, p.bpack_s,
                           p.coff_s, src_s, p.n, grid);
    else
        hipLaunchKernelGGL((k_spread<T, 6, TS>), grd, dim3(256), 0, st, g, p.tile_start, p.bpack_s,
                           p.coff_s, src_s, p.n, grid);
}

template <typename T>
void launch_gather(const GridGeo& g, const PointsDev<T>& p, const T* field, int batch, T* u,
                   hipStream_t st) {
    dim3 grd(ntiles(g), batch);
    if (g.P <= 16)
        hipLaunchKernelGGL((k_gather<T, 16>), grd, dim3(256), 0, st, g, p.tile_start, p.perm_s,
                           p.bpack_s, p.coff_s, field, p.n, u);
    else
        hipLaunchKernelGGL((k_gather<T, 32>), grd, dim3(256), 0, st, g, p.tile_start, p.perm_s,
                           p.bpack_s, p.coff_s, field, p.n, u);
}

template <typename T>
void launch_gather_grad(const GridGeo& g, const PointsDev<T>& p, const T* phi_f, const T* phi_w,
                        const T* f_s, const T* w_s, int batch, T* dsrc, T* dx, hipStream_t st) {
    dim3 grd(ntiles(g));
    if (g.P <= 16)
        hipLaunchKernelGGL((k_gather_grad<T, 16>), grd, dim3(256), 0, st, g, p.tile_start, p.perm_s,
                           p.bpack_s, p.coff_s, phi_f, phi_w, f_s, w_s, p.n, batch, dsrc, dx);
    else
        hipLaunchKernelGGL((k_gather_grad<T, 32>), grd, dim3(256), 0, st, g, p.tile_start, p.perm_s,
                           p.bpack_s, p.coff_s, phi_f, phi_w, f_s, w_s, p.n, batch, dsrc, dx);
}

#define INST(T)                                                                                      \
    template void launch_spread<T>(const GridGeo&, const PointsDev<T>&, const T*, int, int, T*,      \
                                   hipStream_t);                                                     \
    template void launch_gather<T>(const GridGeo&, const PointsDev<T>&, const T*, int, T*,           \
                                   hipStream_t);                                                     \
    template void launch_gather_grad<T>(const GridGeo&, const PointsDev<T>&, const T*, const T*,     \
                                        const T*, const T*, int, T*, T*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace fse
