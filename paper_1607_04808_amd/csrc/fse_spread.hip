// Gaussian gridding (Section 5.2): step 1 "spreading" (eq. Hx) and step 5
// "quadrature" (eq. u_integr, trapezoidal rule), with Gaussians truncated to a
// P^3 cube of grid points (fast Gaussian gridding).  The weights here are the
// raw factors exp(-alpha |x_node - x|^2) = prod_d exp(-alpha h^2 (t_d - i_d)^2);
// the normalisations (alpha/pi)^{3/2} of both steps and the quadrature weight
// h^3 are folded into the precomputed Fourier multiplier.
//
// Points are binned by the bin (TB^3 nodes, TB = GridGeo::TS) holding their
// window start, x-fastest bin order, so a row of bins is one contiguous range.
//
// Spreading: output-stationary (see k_spread); every node is written exactly
// once, coalesced, by the thread that owns it: no atomics, no clearing of the
// grid, and a deterministic summation order.
//
// Quadrature: one workgroup per bin stages the (TB+P-1)^3 block of the field
// that the bin's windows cover in LDS (when it fits) and each wave reduces one
// point at a time from LDS; otherwise the field is read from global memory.
#include <mutex>
#include <utility>
#include <vector>

#include "fse_common.h"

namespace fse {

namespace {

template <typename T> __device__ __forceinline__ T dexp(T x);
template <> __device__ __forceinline__ float dexp<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double dexp<double>(double x) { return exp(x); }

// floor(a / b) for 0 <= a < 2^12 and 1 <= b <= 64 via a float reciprocal: a/b is
// never within 1/(2b) of an integer above it, far above the rounding error.
__device__ __forceinline__ int small_div(int a, int b) {
    return (int)(((float)a + 0.5f) * __builtin_amdgcn_rcpf((float)b));
}

// Output-stationary spreading.  The workgroup (256 threads) owns a 16 x 16 x TZ
// core of grid nodes; thread (tx, ty) keeps the z-column (tx, ty, 0..TZ-1) of
// the core in registers for every component, so no accumulation ever needs an
// atomic (LDS float atomics are slow on this hardware).  Candidate points,
// those of the bins whose window starts can reach the core, are staged in LDS
// in chunks of CH, compacted to the ones whose window overlaps the core, and
// their 3P one-dimensional Gaussian factors are computed cooperatively into
// LDS.  Every thread then walks the chunk's points in order (a fixed order, so
// the result is deterministic): a wave whose 16 x 4 block of columns misses a
// point's window skips it, and the point's z-range inside the core is a
// wave-uniform (scalar) loop bound.
template <typename T, int NC, int PMAX, int TZ, int CH>
__global__ __launch_bounds__(256) void k_spread(GridGeo g, const int* __restrict__ tile_start,
                                               const int* __restrict__ bpack_s,
                                               const T* __restrict__ coff_s,
                                               const T* __restrict__ src_s, int64_t n, T* grid) {
    __shared__ T s_w[CH][3][PMAX];
    __shared__ T s_c[CH][3];
    __shared__ T s_v[CH][NC];
    __shared__ int s_bp[CH];
    __shared__ int s_cnt;

    const int Mt = g.Mt, P = g.P, TB = g.TS, nb = g.nt;
    const int ncxy = (Mt + 15) / 16, ncz = (Mt + TZ - 1) / TZ;
    const int t = blockIdx.x;
    const int cx = t % ncxy, cy = (t / ncxy) % ncxy, cz = t / (ncxy * ncxy);
    const int bm = blockIdx.y;
    const int lox = cx * 16, loy = cy * 16, loz = cz * TZ;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int gx = lox + tx, gy = loy + ty;
    const T ahh = (T)g.ahh;
    const T half = (T)(0.5 * (P - 1));

    T acc[TZ][NC];
#pragma unroll
    for (int z = 0; z < TZ; ++z)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[z][c] = (T)0;

    // bins holding window starts b in [lo - P + 1, lo + ext - 1] ∩ [0, Mt - P]
    const int bx0 = max(0, lox - P + 1) / TB, bx1 = min(Mt - P, lox + 15) / TB;
    const int by0 = max(0, loy - P + 1) / TB, by1 = min(Mt - P, loy + 15) / TB;
    const int bz0 = max(0, loz - P + 1) / TB, bz1 = min(Mt - P, loz + TZ - 1) / TB;
    for (int sz = bz0; sz <= bz1; ++sz)
        for (int sy = by0; sy <= by1; ++sy) {
            const int row = (sz * nb + sy) * nb;
            const int j0 = tile_start[row + bx0], j1 = tile_start[row + bx1 + 1];
            for (int base = j0; base < j1; base += CH) {
                if (threadIdx.x == 0) s_cnt = 0;
                __syncthreads();
                if ((int)threadIdx.x < CH) {
                    const int j = base + (int)threadIdx.x;
                    if (j < j1) {
                        const int bp = bpack_s[j];
                        const int bx = bp & 1023, by = (bp >> 10) & 1023, bz = bp >> 20;
                        const bool ov = bx <= lox + 15 && bx + P > lox && by <= loy + 15 && by + P > loy &&
                                        bz <= loz + TZ - 1 && bz + P > loz;
                        if (ov) {
                            const int k = atomicAdd(&s_cnt, 1);
                            s_bp[k] = bp;
                            s_c[k][0] = coff_s[3 * (int64_t)j];
                            s_c[k][1] = coff_s[3 * (int64_t)j + 1];
                            s_c[k][2] = coff_s[3 * (int64_t)j + 2];
#pragma unroll
                            for (int c = 0; c < NC; ++c) s_v[k][c] = src_s[((int64_t)bm * n + j) * NC + c];
                        }
                    }
                }
                __syncthreads();
                const int cnt = s_cnt;
                // 1D Gaussian factors of the compacted points
                for (int q = threadIdx.x; q < cnt * 3 * P; q += 256) {
                    const int k = q / (3 * P), r = q - k * 3 * P;
                    const int d = r / P, i = r - d * P;
                    const T e = s_c[k][d] + half - (T)i;
                    s_w[k][d][i] = dexp<T>(-ahh * e * e);
                }
                __syncthreads();
                for (int k = 0; k < cnt; ++k) {
                    const int bp = __builtin_amdgcn_readfirstlane(s_bp[k]);
                    const int bx = bp & 1023, by = (bp >> 10) & 1023, bz = bp >> 20;
                    const int ix = gx - bx, iy = gy - by;
                    const bool in = (unsigned)ix < (unsigned)P && (unsigned)iy < (unsigned)P;
                    if (!__any(in)) continue;
                    const T wxy = in ? s_w[k][0][in ? ix : 0] * s_w[k][1][in ? iy : 0] : (T)0;
                    T v[NC];
#pragma unroll
                    for (int c = 0; c < NC; ++c) v[c] = s_v[k][c];
                    const int zlo = max(bz, loz) - loz, zhi = min(bz + P, loz + TZ) - loz;
                    const T* wz = &s_w[k][2][loz - bz];
#pragma unroll
                    for (int z = 0; z < TZ; ++z) {
                        if (z >= zlo && z < zhi) {
                            const T w = wxy * wz[z];
#pragma unroll
                            for (int c = 0; c < NC; ++c) acc[z][c] += w * v[c];
                        }
                    }
                }
                __syncthreads();
            }
        }
    if (gx < Mt && gy < Mt) {
        const int64_t M3 = (int64_t)Mt * Mt * Mt;
#pragma unroll
        for (int z = 0; z < TZ; ++z) {
            const int gz = loz + z;
            if (gz < Mt) {
                const int64_t o = ((int64_t)gz * Mt + gy) * Mt + gx;
#pragma unroll
                for (int c = 0; c < NC; ++c) grid[((int64_t)bm * NC + c) * M3 + o] = acc[z][c];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Quadrature with the bin's field block staged in LDS.  MODE 0: value gather
// u = sum g(x - x_p) F(p) (3 components).  MODE 1: gradient part with the
// forward field, dx = sum grad g (w . phi_f).  MODE 2: value of phi_w into
// dsrc and dx += sum grad g (f . phi_w).
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(512) void k_gather_lds(GridGeo g, const int* __restrict__ tile_start,
                                                   const int* __restrict__ perm_s,
                                                   const int* __restrict__ bpack_s,
                                                   const T* __restrict__ coff_s,
                                                   const T* __restrict__ field, const T* __restrict__ vec_s,
                                                   int64_t n, int batch, T* out, T* dx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = (T*)smem_raw;
    __shared__ T s_w[8][4][32];
    const int Mt = g.Mt, P = g.P, TB = g.TS, nb = g.nt;
    const int E = TB + P - 1;
    const int E3 = E * E * E;
    const int64_t M3 = (int64_t)Mt * Mt * Mt;
    const int s = blockIdx.x;
    const int j0 = tile_start[s], j1 = tile_start[s + 1];
    if (j0 == j1) return;
    const int tbx = s % nb, tby = (s / nb) % nb, tbz = s / (nb * nb);
    const int lox = tbx * TB, loy = tby * TB, loz = tbz * TB;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const T ahh = (T)g.ahh;
    const T dfac = (T)(-2.0 * g.ahh / g.h);
    const T half = (T)(0.5 * (P - 1));
    const int R = 64 / P;
    const int rr = small_div(lane, P);
    const int ix = lane - rr * P;
    const int bm0 = MODE == 0 ? blockIdx.y : 0;
    const int bm1 = MODE == 0 ? blockIdx.y + 1 : batch;
    for (int bm = bm0; bm < bm1; ++bm) {
        __syncthreads();
        for (int q = threadIdx.x; q < 3 * E3; q += blockDim.x) {
            const int c = q / E3, r = q - c * E3;
            const int x = r % E, y = (r / E) % E, z = r / (E * E);
            const int gx = lox + x, gy = loy + y, gz = loz + z;
            sm[q] = (gx < Mt && gy < Mt && gz < Mt)
                        ? field[((int64_t)bm * 3 + c) * M3 + ((int64_t)gz * Mt + gy) * Mt + gx]
                        : (T)0;
        }
        __syncthreads();
        for (int j = j0 + wid; j < j1; j += nw) {
            const int bp = bpack_s[j];
            const int lbx = (bp & 1023) - lox, lby = ((bp >> 10) & 1023) - loy, lbz = (bp >> 20) - loz;
            const T cx = coff_s[3 * (int64_t)j], cy = coff_s[3 * (int64_t)j + 1], cz = coff_s[3 * (int64_t)j + 2];
            const T ex = cx + half - (T)ix;
            const T wx = dexp<T>(-ahh * ex * ex);
            const T dwx = dfac * ex * wx;
            if (lane < P) {
                const T ey = cy + half - (T)lane;
                const T wy = dexp<T>(-ahh * ey * ey);
                s_w[wid][0][lane] = wy;
                s_w[wid][2][lane] = dfac * ey * wy;
            } else if (lane >= 32 && lane - 32 < P) {
                const T ez = cz + half - (T)(lane - 32);
                const T wz = dexp<T>(-ahh * ez * ez);
                s_w[wid][1][lane - 32] = wz;
                s_w[wid][3][lane - 32] = dfac * ez * wz;
            }
            wave_lds_sync();
            T v0 = 0, v1 = 0, v2 = 0;  // MODE 0/2 values
            T g0 = 0, g1 = 0, g2 = 0;  // MODE 1/2 gradient
            T p0 = 0, p1 = 0, p2 = 0;  // contraction vector
            if (MODE != 0) {
                const T* pv = vec_s + ((int64_t)bm * n + j) * 3;
                p0 = pv[0];
                p1 = pv[1];
                p2 = pv[2];
            }
            if (rr < R) {
                int iz = small_div(rr, P);
                int iy = rr - iz * P;
                const T* f0 = sm + (lbz * E + lby) * E + lbx + ix;
                for (int q = rr; q < P * P; q += R) {
                    const T* f = f0 + (iz * E + iy) * E;
                    const T a0 = f[0], a1 = f[E3], a2 = f[2 * E3];
                    const T wy = s_w[wid][0][iy], wz = s_w[wid][1][iz];
                    if (MODE == 0) {
                        const T w = wx * wy * wz;
                        v0 += w * a0;
                        v1 += w * a1;
                        v2 += w * a2;
                    } else {
                        const T psi = p0 * a0 + p1 * a1 + p2 * a2;
                        const T dwy = s_w[wid][2][iy], dwz = s_w[wid][3][iz];
                        g0 += psi * dwx * wy * wz;
                        g1 += psi * wx * dwy * wz;
                        g2 += psi * wx * wy * dwz;
                        if (MODE == 2) {
                            const T w = wx * wy * wz;
                            v0 += w * a0;
                            v1 += w * a1;
                            v2 += w * a2;
                        }
                    }
                    iy += R;
                    while (iy >= P) {
                        iy -= P;
                        ++iz;
                    }
                }
            }
            const int64_t i = perm_s[j];
            if (MODE != 1) {
                v0 = wave_sum(v0);
                v1 = wave_sum(v1);
                v2 = wave_sum(v2);
                if (lane == 0 && out) {
                    T* o = out + ((int64_t)bm * n + i) * 3;
                    o[0] = v0;
                    o[1] = v1;
                    o[2] = v2;
                }
            }
            if (MODE != 0) {
                g0 = wave_sum(g0);
                g1 = wave_sum(g1);
                g2 = wave_sum(g2);
                if (lane == 0 && dx) {
                    // the first contribution (forward field, first batch member) overwrites
                    const bool first = (MODE == 1 && bm == 0);
                    dx[3 * i] = (first ? (T)0 : dx[3 * i]) + g0;
                    dx[3 * i + 1] = (first ? (T)0 : dx[3 * i + 1]) + g1;
                    dx[3 * i + 2] = (first ? (T)0 : dx[3 * i + 2]) + g2;
                }
            }
            wave_lds_sync();
        }
    }
}

// Quadrature reading the field from global memory (large P or FP64 blocks that
// do not fit in LDS): one wave per point, LPR lanes along x per window row.
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
#pragma unroll 4
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

// Adjoint quadrature from global memory: for each point s and batch member b,
//   dsrc_b(x_s) = quadrature of phi_w,b, and
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
    const T dfac = (T)(-2.0 * g.ahh / g.h);
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

inline unsigned nbins(const GridGeo& g) { return (unsigned)(g.nt * g.nt * g.nt); }

// LDS bytes of the staged field block, or 0 if it does not fit
template <typename T> size_t gather_lds_bytes(const GridGeo& g) {
    const size_t E = (size_t)g.TS + g.P - 1;
    const size_t b = 3 * E * E * E * sizeof(T);
    return b <= 140 * 1024 ? b : 0;
}

// Raise a kernel's dynamic-LDS limit to `bytes` (static LDS comes on top and
// the sum must stay within the 160 KB of a workgroup); remembered per kernel.
template <typename K> void allow_lds(K kern, size_t bytes) {
    static std::mutex mu;
    static std::vector<std::pair<const void*, size_t>> done;
    std::lock_guard<std::mutex> lk(mu);
    for (auto& d : done)
        if (d.first == (const void*)kern && d.second >= bytes) return;
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    done.emplace_back((const void*)kern, bytes);
}

}  // namespace

template <typename T>
void launch_spread(const GridGeo& g, const PointsDev<T>& p, const T* src_s, int c_in, int batch,
                   T* grid, hipStream_t st) {
    // cores of 16 x 16 x TZ nodes: TZ = 16 (FP32) or 8 (FP64) register accumulators per component
    constexpr int TZ = sizeof(T) == 4 ? 16 : 8;
    const unsigned ncxy = (unsigned)((g.Mt + 15) / 16), ncz = (unsigned)((g.Mt + TZ - 1) / TZ);
    dim3 grd(ncxy * ncxy * ncz, batch);
#define SPREAD(NC, PM, CHK)                                                                                  \
    hipLaunchKernelGGL((k_spread<T, NC, PM, TZ, CHK>), grd, dim3(256), 0, st, g, p.tile_start, p.bpack_s, \
                       p.coff_s, src_s, p.n, grid)
    if (sizeof(T) == 4 && g.P <= 16) {
        if (c_in == 3) SPREAD(3, 16, 128); else SPREAD(6, 16, 128);
    } else {
        if (c_in == 3) SPREAD(3, 32, 64); else SPREAD(6, 32, 64);
    }
#undef SPREAD
}

template <typename T>
void launch_gather(const GridGeo& g, const PointsDev<T>& p, const T* field, int batch, T* u,
                   hipStream_t st) {
    const size_t lds = gather_lds_bytes<T>(g);
    if (lds) {
        allow_lds(k_gather_lds<T, 0>, lds);
        hipLaunchKernelGGL((k_gather_lds<T, 0>), dim3(nbins(g), batch), dim3(512), lds, st, g, p.tile_start,
                           p.perm_s, p.bpack_s, p.coff_s, field, (const T*)nullptr, p.n, batch, u, (T*)nullptr);
        return;
    }
    dim3 grd(nbins(g), batch);
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
    const size_t lds = gather_lds_bytes<T>(g);
    if (lds && dx) {
        // pass 1: forward field contracted with w; pass 2: phi_w value and contraction with f
        allow_lds(k_gather_lds<T, 1>, lds);
        allow_lds(k_gather_lds<T, 2>, lds);
        hipLaunchKernelGGL((k_gather_lds<T, 1>), dim3(nbins(g)), dim3(512), lds, st, g, p.tile_start, p.perm_s,
                           p.bpack_s, p.coff_s, phi_f, w_s, p.n, batch, (T*)nullptr, dx);
        hipLaunchKernelGGL((k_gather_lds<T, 2>), dim3(nbins(g)), dim3(512), lds, st, g, p.tile_start, p.perm_s,
                           p.bpack_s, p.coff_s, phi_w, f_s, p.n, batch, dsrc, dx);
        return;
    }
    dim3 grd(nbins(g));
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
