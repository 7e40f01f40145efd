// Zero-padded 3D FFT, scaling and inverse FFT (Section 5.2, steps 2-4).
//
// The (2Mt)^3 transform of an Mt^3 real grid is done as three pruned passes of
// 1D transforms staged in LDS, each pass writing its output transposed so the
// next pass reads contiguous lines:
//   x-pass  grid[c][z][y][x] (real)  -> A[c][kx][z][y]   R2C, two real rows per
//                                                          complex transform
//   y-pass  A[c][kx][z][y]           -> B[c][kx][ky][z]
//   z-pass  B[c][kx][ky][z]          -> B (in place): forward z transform,
//           multiplication by the Fourier multiplier of eq. gridfcnsc (scalar
//           precomputed part times the k-polynomial of eqs. AS/AT/AR), inverse z
//           transform, keep z < Mt.  The spectrum never reaches HBM.
//   y-inv   B -> A (keep y < Mt),  x-inv  A -> field[c][z][y][x] (C2R, keep x < Mt).
// Only the Mt nonzero input lines are read and only the Mt kept output lines are
// written per direction (the zero padding and the truncation of Section 5.2).
//
// 1D transforms: in-place mixed-radix (2,3,4,5,7,8) decimation in frequency,
// leaving the spectrum in digit-reversed order; the inverse is the matching
// decimation in time, which takes digit-reversed input and returns natural
// order.  Inverses are unnormalised (1/n^3 lives in the multiplier).
#include <mutex>
#include <utility>
#include <vector>

#include "fse_common.h"

namespace fse {

namespace {

// ---------------------------------------------------------------------------
// small DFTs: y_k = sum_j x_j exp(DIR * 2 pi i jk / R)   (DIR = -1 forward)
// ---------------------------------------------------------------------------
template <typename V, int DIR> __device__ __forceinline__ void dft2(V* x) {
    V a = cadd(x[0], x[1]), b = csub(x[0], x[1]);
    x[0] = a;
    x[1] = b;
}
template <typename V, int DIR> __device__ __forceinline__ void dft3(V* x) {
    using T = decltype(V::x);
    const T h3 = (T)0.86602540378443864676;
    V s = cadd(x[1], x[2]), d = csub(x[1], x[2]);
    V t = csub(x[0], cscale(s, (T)0.5));
    V e = cmuli<DIR>(cscale(d, h3));
    x[0] = cadd(x[0], s);
    x[1] = cadd(t, e);
    x[2] = csub(t, e);
}
template <typename V, int DIR> __device__ __forceinline__ void dft4(V* x) {
    V a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    V c = cadd(x[1], x[3]), d = cmuli<DIR>(csub(x[1], x[3]));
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, d);
    x[3] = csub(b, d);
}
template <typename V, int DIR> __device__ __forceinline__ void dft5(V* x) {
    using T = decltype(V::x);
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    V a1 = cadd(x[1], x[4]), b1 = csub(x[1], x[4]);
    V a2 = cadd(x[2], x[3]), b2 = csub(x[2], x[3]);
    V y0 = cadd(x[0], cadd(a1, a2));
    V t1 = cadd(x[0], cadd(cscale(a1, c1), cscale(a2, c2)));
    V t2 = cadd(x[0], cadd(cscale(a1, c2), cscale(a2, c1)));
    V u1 = cmuli<DIR>(cadd(cscale(b1, s1), cscale(b2, s2)));
    V u2 = cmuli<DIR>(csub(cscale(b1, s2), cscale(b2, s1)));
    x[0] = y0;
    x[1] = cadd(t1, u1);
    x[4] = csub(t1, u1);
    x[2] = cadd(t2, u2);
    x[3] = csub(t2, u2);
}
template <typename V, int DIR> __device__ __forceinline__ void dft7(V* x) {
    using T = decltype(V::x);
    // cos / sin (2 pi m / 7), m = 0..6
    const T C[7] = {(T)1.0, (T)0.62348980185873353053, (T)-0.22252093395631440429,
                    (T)-0.90096886790241912624, (T)-0.90096886790241912624,
                    (T)-0.22252093395631440429, (T)0.62348980185873353053};
    const T S[7] = {(T)0.0, (T)0.78183148246802980871, (T)0.97492791218182360702,
                    (T)0.43388373911755812048, (T)-0.43388373911755812048,
                    (T)-0.97492791218182360702, (T)-0.78183148246802980871};
    V a[4], b[4];
#pragma unroll
    for (int j = 1; j <= 3; ++j) {
        a[j] = cadd(x[j], x[7 - j]);
        b[j] = csub(x[j], x[7 - j]);
    }
    V y[7];
    y[0] = cadd(x[0], cadd(a[1], cadd(a[2], a[3])));
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        V t = x[0], u = cmk<V>((T)0, (T)0);
#pragma unroll
        for (int j = 1; j <= 3; ++j) {
            const int m = (j * k) % 7;
            t = cadd(t, cscale(a[j], C[m]));
            u = cadd(u, cscale(b[j], S[m]));
        }
        u = cmuli<DIR>(u);
        y[k] = cadd(t, u);
        y[7 - k] = csub(t, u);
    }
#pragma unroll
    for (int k = 0; k < 7; ++k) x[k] = y[k];
}
template <typename V, int DIR> __device__ __forceinline__ void dft8(V* x) {
    using T = decltype(V::x);
    const T r = (T)0.70710678118654752440;
    V e[4] = {x[0], x[2], x[4], x[6]};
    V o[4] = {x[1], x[3], x[5], x[7]};
    dft4<V, DIR>(e);
    dft4<V, DIR>(o);
    // W = exp(DIR 2 pi i / 8)
    V w1 = cmul(o[1], cmk<V>(r, (T)DIR * r));
    V w2 = cmuli<DIR>(o[2]);
    V w3 = cmul(o[3], cmk<V>(-r, (T)DIR * r));
    x[0] = cadd(e[0], o[0]);
    x[4] = csub(e[0], o[0]);
    x[1] = cadd(e[1], w1);
    x[5] = csub(e[1], w1);
    x[2] = cadd(e[2], w2);
    x[6] = csub(e[2], w2);
    x[3] = cadd(e[3], w3);
    x[7] = csub(e[3], w3);
}

template <typename V, int R, int DIR> __device__ __forceinline__ void dft(V* x) {
    if constexpr (R == 2) dft2<V, DIR>(x);
    else if constexpr (R == 3) dft3<V, DIR>(x);
    else if constexpr (R == 4) dft4<V, DIR>(x);
    else if constexpr (R == 5) dft5<V, DIR>(x);
    else if constexpr (R == 7) dft7<V, DIR>(x);
    else dft8<V, DIR>(x);
}

// One DIF butterfly: DFT of x[k*m], then twiddle output k by w_Ls^{n1 k}.
template <typename V, int R>
__device__ __forceinline__ void bf_dif(V* p, int m, int tstep, const V* tw) {
    V x[R];
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = p[k * m];
    dft<V, R, -1>(x);
#pragma unroll
    for (int k = 1; k < R; ++k) x[k] = cmul(x[k], tw[tstep * k]);
#pragma unroll
    for (int k = 0; k < R; ++k) p[k * m] = x[k];
}
// Matching inverse DIT butterfly: conjugate twiddle, then inverse DFT.
template <typename V, int R>
__device__ __forceinline__ void bf_dit_inv(V* p, int m, int tstep, const V* tw) {
    V x[R];
    x[0] = p[0];
#pragma unroll
    for (int k = 1; k < R; ++k) x[k] = cmulc(p[k * m], tw[tstep * k]);
    dft<V, R, 1>(x);
#pragma unroll
    for (int k = 0; k < R; ++k) p[k * m] = x[k];
}

template <typename V, bool INV>
__device__ __forceinline__ void bf(int r, V* p, int m, int tstep, const V* tw) {
    switch (r) {
        case 2: INV ? bf_dit_inv<V, 2>(p, m, tstep, tw) : bf_dif<V, 2>(p, m, tstep, tw); break;
        case 3: INV ? bf_dit_inv<V, 3>(p, m, tstep, tw) : bf_dif<V, 3>(p, m, tstep, tw); break;
        case 4: INV ? bf_dit_inv<V, 4>(p, m, tstep, tw) : bf_dif<V, 4>(p, m, tstep, tw); break;
        case 5: INV ? bf_dit_inv<V, 5>(p, m, tstep, tw) : bf_dif<V, 5>(p, m, tstep, tw); break;
        case 7: INV ? bf_dit_inv<V, 7>(p, m, tstep, tw) : bf_dif<V, 7>(p, m, tstep, tw); break;
        default: INV ? bf_dit_inv<V, 8>(p, m, tstep, tw) : bf_dif<V, 8>(p, m, tstep, tw); break;
    }
}

// Two DIF stages s, s+1 (radices R1, R2) on one element group in registers:
// x[sub][i] = p[sub m + i mp] (m = Ls/R1, mp = m/R2); stage s transforms over
// sub for each i (position n1 = n1p + i mp), stage s+1 over i for each sub.
template <typename V, int R1, int R2>
__device__ __forceinline__ void bf2_dif(V* p, int m, int mp, int n1p, int ts1, int ts2, const V* tw) {
    V x[R1][R2];
#pragma unroll
    for (int a = 0; a < R1; ++a)
#pragma unroll
        for (int i = 0; i < R2; ++i) x[a][i] = p[a * m + i * mp];
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        V y[R1];
#pragma unroll
        for (int a = 0; a < R1; ++a) y[a] = x[a][i];
        dft<V, R1, -1>(y);
        const int n1 = n1p + i * mp;
#pragma unroll
        for (int k = 1; k < R1; ++k) y[k] = cmul(y[k], tw[ts1 * n1 * k]);
#pragma unroll
        for (int a = 0; a < R1; ++a) x[a][i] = y[a];
    }
#pragma unroll
    for (int a = 0; a < R1; ++a) {
        dft<V, R2, -1>(x[a]);
#pragma unroll
        for (int k = 1; k < R2; ++k) x[a][k] = cmul(x[a][k], tw[ts2 * n1p * k]);
    }
#pragma unroll
    for (int a = 0; a < R1; ++a)
#pragma unroll
        for (int i = 0; i < R2; ++i) p[a * m + i * mp] = x[a][i];
}
// The matching inverse of stages s+1 then s (DIT, conjugate twiddles first):
// E[a][i] = p[a Ls1 + i m1] with Ls1 = Ls[s+1], m1 = Ls1/R2; stage s+1 over i
// for each a (position n1), then stage s over a for each i (position n1 + i m1).
template <typename V, int R1, int R2>
__device__ __forceinline__ void bf2_dit_inv(V* p, int Ls1, int m1, int n1, int ts1, int ts2, const V* tw) {
    V x[R1][R2];
#pragma unroll
    for (int a = 0; a < R1; ++a)
#pragma unroll
        for (int i = 0; i < R2; ++i) x[a][i] = p[a * Ls1 + i * m1];
#pragma unroll
    for (int a = 0; a < R1; ++a) {
#pragma unroll
        for (int k = 1; k < R2; ++k) x[a][k] = cmulc(x[a][k], tw[ts2 * n1 * k]);
        dft<V, R2, 1>(x[a]);
    }
#pragma unroll
    for (int i = 0; i < R2; ++i) {
        V y[R1];
        y[0] = x[0][i];
        const int n1s = n1 + i * m1;
#pragma unroll
        for (int k = 1; k < R1; ++k) y[k] = cmulc(x[k][i], tw[ts1 * n1s * k]);
        dft<V, R1, 1>(y);
#pragma unroll
        for (int a = 0; a < R1; ++a) x[a][i] = y[a];
    }
#pragma unroll
    for (int a = 0; a < R1; ++a)
#pragma unroll
        for (int i = 0; i < R2; ++i) p[a * Ls1 + i * m1] = x[a][i];
}

#define FSE_FFT_PAIRS(X) \
    X(8, 2) X(8, 3) X(8, 4) X(7, 2) X(7, 3) X(7, 4) X(5, 2) X(5, 3) X(5, 4) X(5, 5) X(4, 3) X(2, 3) X(3, 3)

template <typename V, bool INV>
__device__ __forceinline__ void bf2(int r1, int r2, V* p, int a, int b, int n1, int ts1, int ts2, const V* tw) {
    switch (r1 * 16 + r2) {
#define FSE_CASE(R1, R2)                                                          \
    case R1 * 16 + R2:                                                            \
        if constexpr (fft_pair_ok(R1, R2, (int)sizeof(V) / 2)) {                  \
            if (INV) bf2_dit_inv<V, R1, R2>(p, a, b, n1, ts1, ts2, tw);           \
            else bf2_dif<V, R1, R2>(p, a, b, n1, ts1, ts2, tw);                   \
        }                                                                         \
        break;
        FSE_FFT_PAIRS(FSE_CASE)
#undef FSE_CASE
        default: break;
    }
}

// All stages over `nl` lines of length n stored at buf + l*ld, single stages
// or fused pairs (FftGeo::pair).  Barrier after every pass (and none needed
// before the first: callers sync after loading).
template <typename V, bool INV>
__device__ void fft_lines(V* buf, int nl, int ld, const FftGeo& fg, const V* tw) {
    const int n = fg.n;
    const int tid = threadIdx.x, nthr = blockDim.x;
    int si = 0;
    while (si < fg.ns) {
        // stage s in DIF numbering; the inverse runs the stages backwards
        const int s = INV ? fg.ns - 1 - si : si;
        const bool fused = INV ? (s >= 1 && fg.pair[s - 1]) : (fg.pair[s] != 0);
        if (fused) {
            const int s0 = INV ? s - 1 : s;  // the pair is (s0, s0 + 1)
            const int r1 = fg.rad[s0], r2 = fg.rad[s0 + 1];
            const int Ls = fg.Ls[s0], m = Ls / r1, mp = m / r2;
            const int ts1 = n / Ls, ts2 = n / m;
            const int ngrp = n / (r1 * r2);
            const int tot = nl * ngrp;
            for (int q = tid; q < tot; q += nthr) {
                const int l = small_div(q, ngrp);
                const int g = q - l * ngrp;
                if (!INV) {
                    // groups: block of stage s0, position n1p < mp
                    const int blk = small_div(g, mp);
                    const int n1p = g - blk * mp;
                    bf2<V, false>(r1, r2, buf + l * ld + blk * Ls + n1p, m, mp, n1p, ts1, ts2, tw);
                } else {
                    // groups: block of stage s0, position n1 < mp within a block of stage s0 + 1
                    const int blk = small_div(g, mp);
                    const int n1 = g - blk * mp;
                    bf2<V, true>(r1, r2, buf + l * ld + blk * Ls + n1, m, mp, n1, ts1, ts2, tw);
                }
            }
            si += 2;
        } else {
            const int r = fg.rad[s], Ls = fg.Ls[s], m = Ls / r, ts = n / Ls;
            const int nbf = n / r;
            const int tot = nl * nbf;
            for (int q = tid; q < tot; q += nthr) {
                const int l = small_div(q, nbf);
                const int b = q - l * nbf;
                const int blk = small_div(b, m);
                const int n1 = b - blk * m;
                bf<V, INV>(r, buf + l * ld + blk * Ls + n1, m, n1 * ts, tw);
            }
            si += 1;
        }
        __syncthreads();
    }
}

// Stage the twiddle and index tables in LDS; the barrier makes them visible
// to every thread before any use.
template <typename V>
__device__ __forceinline__ void load_tables(V* tw, int* idx, const V* twg, const int* idxg, int n) {
    staged_copy<4>(n, [&](int q) { return twg[q]; }, [&](int q, V v) { tw[q] = v; });
    staged_copy<4>(n, [&](int q) { return idxg[q]; }, [&](int q, int v) { idx[q] = v; });
    __syncthreads();
}

// ---------------------------------------------------------------------------
// x-pass: R2C of ROWS real rows (paired into ROWS/2 complex lines)
// ---------------------------------------------------------------------------
template <typename T, int ROWS>
__global__ __launch_bounds__(256) void k_fft_x(FftGeo fg, int Mt, const T* __restrict__ grid,
                                              C2<T>* __restrict__ A, const C2<T>* __restrict__ twg,
                                              const int* __restrict__ revinvg) {
    using V = C2<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = fg.n;
    V* tw = (V*)smem;
    V* buf = tw + n;
    int* revinv = (int*)(buf + (ROWS / 2) * n);
    load_tables(tw, revinv, twg, revinvg, n);
    const int y0 = blockIdx.x * ROWS, z = blockIdx.y, bc = blockIdx.z;
    const int64_t M2 = (int64_t)Mt * Mt;
    const T* src = grid + ((int64_t)bc * Mt + z) * M2;
    staged_copy<8>(
        (ROWS / 2) * n,
        [&](int q) {
            const int l = small_div(q, n), x = q - l * n;
            const int ya = y0 + 2 * l, yb = ya + 1;
            const T re = (x < Mt && ya < Mt) ? src[(int64_t)ya * Mt + x] : (T)0;
            const T im = (x < Mt && yb < Mt) ? src[(int64_t)yb * Mt + x] : (T)0;
            return cmk<V>(re, im);
        },
        [&](int q, V v) { buf[q] = v; });
    __syncthreads();
    fft_lines<V, false>(buf, ROWS / 2, n, fg, tw);
    const int64_t MA = (int64_t)Mt * fg.sy;  // one kx slab of A
    V* dst = A + (int64_t)bc * (Mt + 1) * MA + (int64_t)z * fg.sy + y0;
    for (int q = threadIdx.x; q < (Mt + 1) * ROWS; q += blockDim.x) {
        const int kx = q / ROWS, r = q % ROWS;
        if (y0 + r >= Mt) continue;
        const int l = r >> 1;
        const V zk = buf[l * n + revinv[kx]];
        const V zn = buf[l * n + revinv[kx == 0 ? 0 : n - kx]];
        V X;
        if (r & 1) X = cmk<V>((T)0.5 * (zk.y + zn.y), (T)0.5 * (zn.x - zk.x));
        else X = cmk<V>((T)0.5 * (zk.x + zn.x), (T)0.5 * (zk.y - zn.y));
        dst[(int64_t)kx * MA + r] = X;
    }
}

// ---------------------------------------------------------------------------
// y-pass forward: LZ lines (consecutive z) at fixed (c, kx)
// ---------------------------------------------------------------------------
template <typename T, int LZ>
__global__ __launch_bounds__(256) void k_fft_y(FftGeo fg, int Mt, const C2<T>* __restrict__ A,
                                              C2<T>* __restrict__ B, const C2<T>* __restrict__ twg,
                                              const int* __restrict__ revinvg) {
    using V = C2<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = fg.n;
    V* tw = (V*)smem;
    V* buf = tw + n;
    int* revinv = (int*)(buf + LZ * n);
    load_tables(tw, revinv, twg, revinvg, n);
    const int z0 = blockIdx.x * LZ, kx = blockIdx.y, bc = blockIdx.z;
    const int SY = fg.sy, SZ = fg.sz;
    const V* src = A + ((int64_t)bc * (Mt + 1) + kx) * Mt * SY;
    staged_copy<8>(
        LZ * n,
        [&](int q) {
            const int l = small_div(q, n), y = q - l * n;
            const int z = z0 + l;
            return (y < Mt && z < Mt) ? src[(int64_t)z * SY + y] : cmk<V>((T)0, (T)0);
        },
        [&](int q, V v) { buf[q] = v; });
    __syncthreads();
    fft_lines<V, false>(buf, LZ, n, fg, tw);
    V* dst = B + ((int64_t)bc * (Mt + 1) + kx) * n * SZ;
    for (int q = threadIdx.x; q < n * LZ; q += blockDim.x) {
        const int ky = q / LZ, r = q % LZ;
        if (z0 + r < Mt) dst[(int64_t)ky * SZ + z0 + r] = buf[r * n + revinv[ky]];
    }
}

// ---------------------------------------------------------------------------
// z-pass: forward z FFT, multiplier, inverse z FFT for one (kx, ky) column
// ---------------------------------------------------------------------------
// Apply the k-polynomial of the kernel at wavevector k (physical units) to the
// c_in grid components g, giving 3 outputs (the scalar sigma is applied after).
template <typename T, int KERNEL>
__device__ __forceinline__ void kpoly(const T k[3], const C2<T>* g, C2<T>* w, int half = 0) {
    using V = C2<T>;
    const T k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if constexpr (KERNEL == FSE_STOKESLET) {
        // (k^2 d_jl - k_j k_l) g_l
        const V kg = cadd(cadd(cscale(g[0], k[0]), cscale(g[1], k[1])), cscale(g[2], k[2]));
#pragma unroll
        for (int j = 0; j < 3; ++j) w[j] = csub(cscale(g[j], k2), cscale(kg, k[j]));
    } else if constexpr (KERNEL == FSE_ROTLET) {
        // -i eps_jlm g_l k_m = -i (g x k)_j
        const V c0 = csub(cscale(g[1], k[2]), cscale(g[2], k[1]));
        const V c1 = csub(cscale(g[2], k[0]), cscale(g[0], k[2]));
        const V c2 = csub(cscale(g[0], k[1]), cscale(g[1], k[0]));
        w[0] = cmuli<-1>(c0);
        w[1] = cmuli<-1>(c1);
        w[2] = cmuli<-1>(c2);
    } else if constexpr (KERNEL == KSCALAR) {
        w[0] = g[0];
        w[1] = g[1];
        w[2] = g[2];
    } else if constexpr (KERNEL == KTADJ) {
        // The stresslet's transpose: its multiplier -i P_j,lm(k) (P fully symmetric)
        // has the adjoint +i P_j,lm(k) g_j = +i [k^2 (g_l k_m + g_m k_l + d_lm k.g)
        // - 2 k_l k_m k.g], three of the six symmetric (l, m) per half:
        // half 0: (00, 11, 22), half 1: (01, 02, 12)
        const V kg = cadd(cadd(cscale(g[0], k[0]), cscale(g[1], k[1])), cscale(g[2], k[2]));
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            const int l = half ? (o == 2 ? 1 : 0) : o;
            const int m = half ? (o == 0 ? 1 : 2) : o;
            V t = cadd(cscale(g[l], k[m]), cscale(g[m], k[l]));
            if (!half) t = cadd(t, kg);
            t = csub(cscale(t, k2), cscale(kg, (T)2 * k[l] * k[m]));
            w[o] = cmuli<1>(t);
        }
    } else {
        // -i [ k^2 (2 (G k)_j + k_j tr G) - 2 k_j (k.G.k) ],  G symmetric:
        // g = (G00, G11, G22, G01, G02, G12)
        const V Gk0 = cadd(cadd(cscale(g[0], k[0]), cscale(g[3], k[1])), cscale(g[4], k[2]));
        const V Gk1 = cadd(cadd(cscale(g[3], k[0]), cscale(g[1], k[1])), cscale(g[5], k[2]));
        const V Gk2 = cadd(cadd(cscale(g[4], k[0]), cscale(g[5], k[1])), cscale(g[2], k[2]));
        const V tr = cadd(cadd(g[0], g[1]), g[2]);
        const V kGk = cadd(cadd(cscale(Gk0, k[0]), cscale(Gk1, k[1])), cscale(Gk2, k[2]));
        const V Gk[3] = {Gk0, Gk1, Gk2};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const V t = csub(cscale(cadd(cscale(Gk[j], (T)2), cscale(tr, k[j])), k2),
                             cscale(kGk, (T)2 * k[j]));
            w[j] = cmuli<-1>(t);
        }
    }
}

// z-pass with ZB columns transformed together (three-component kernels): the
// 3 ZB lines of a group fill more lanes of the fused stages than the 3 lines of
// one column.  Workgroup: zc consecutive ky columns, in groups of ZB.
template <typename T, int KERNEL, int ZB>
__global__ __launch_bounds__(256) void k_fft_zb(FftGeo fg, int Mt, int zc, C2<T>* __restrict__ B,
                                               const T* __restrict__ sig, double kscale,
                                               const C2<T>* __restrict__ twg,
                                               const int* __restrict__ revg) {
    using V = C2<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = fg.n;
    const int Mp = Mt + 1;
    V* tw = (V*)smem;
    V* buf = tw + n;  // line 3 j + c: component c of the group's column j
    int* rev = (int*)(buf + 3 * ZB * n);
    T* ssig = (T*)(((uintptr_t)(rev + n) + 15) & ~(uintptr_t)15);  // sigma rows, Mp each
    load_tables(tw, rev, twg, revg, n);
    const int kx = blockIdx.y, bm = blockIdx.z;
    const int64_t lstride = (int64_t)(Mt + 1) * n * fg.sz;  // between components
    const bool nyx = (kx == Mt);
    const T ks = (T)kscale;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int kyb = blockIdx.x * zc, kye = min(n, (int)(blockIdx.x + 1) * zc);
    V* const colbase = B + (int64_t)bm * 3 * lstride + (int64_t)kx * n * fg.sz;
    for (int ky0 = kyb; ky0 < kye; ky0 += ZB) {
        const int nb = min(ZB, kye - ky0);
        staged_copy<8>(
            nb * 3 * n,
            [&](int q) {
                const int jc = small_div(q, n), z = q - jc * n;
                const int j = small_div(jc, 3), c = jc - 3 * j;
                return (z < Mt) ? colbase[(int64_t)(ky0 + j) * fg.sz + c * lstride + z] : cmk<V>((T)0, (T)0);
            },
            [&](int q, V v) { buf[q] = v; });
        staged_copy<4>(
            nb * Mp,
            [&](int q) {
                const int j = small_div(q, Mp), e = q - j * Mp;
                const int ky = ky0 + j;
                const int kys = (ky < Mt) ? ky : ky - n;
                return sig[((int64_t)kx * Mp + (kys < 0 ? -kys : kys)) * Mp + e];
            },
            [&](int q, T v) { ssig[q] = v; });
        __syncthreads();
        fft_lines<V, false>(buf, 3 * nb, n, fg, tw);
        for (int q = tid; q < nb * n; q += nthr) {
            const int j = small_div(q, n), p = q - j * n;
            const int ky = ky0 + j;
            const int kys = (ky < Mt) ? ky : ky - n;
            const bool nyy = (ky == Mt);
            const int kzi = rev[p];
            const int kzs = (kzi < Mt) ? kzi : kzi - n;
            const bool nyz = (kzi == Mt);
            V* bl = buf + 3 * j * n + p;
            V g[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) g[c] = bl[c * n];
            const T sv = ssig[j * Mp + (kzs < 0 ? -kzs : kzs)];
            // wavenumbers in [-Mt, Mt): the Nyquist index carries -Mt in every direction
            T k[3] = {ks * (T)(nyx ? -Mt : kx), ks * (T)kys, ks * (T)kzs};
            V w[3];
            kpoly<T, KERNEL>(k, g, w);
            if (nyx || nyy || nyz) {
                // Nyquist planes: the Hermitian part of the multiplier, the mean of its
                // values at k and at k with the Nyquist components negated
                T kr[3] = {nyx ? -k[0] : k[0], nyy ? -k[1] : k[1], nyz ? -k[2] : k[2]};
                V wr[3];
                kpoly<T, KERNEL>(kr, g, wr);
#pragma unroll
                for (int c = 0; c < 3; ++c) w[c] = cscale(cadd(w[c], wr[c]), (T)0.5);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) bl[c * n] = cscale(w[c], sv);
        }
        __syncthreads();
        fft_lines<V, true>(buf, 3 * nb, n, fg, tw);
        for (int q = tid; q < nb * 3 * Mt; q += nthr) {
            const int jc = small_div(q, Mt), z = q - jc * Mt;
            const int j = small_div(jc, 3), c = jc - 3 * j;
            colbase[(int64_t)(ky0 + j) * fg.sz + c * lstride + z] = buf[jc * n + z];
        }
        __syncthreads();
    }
}

template <typename T, int KERNEL, int CIN, int PF>
__global__ __launch_bounds__(128) void k_fft_z(FftGeo fg, int Mt, int zc, C2<T>* __restrict__ B,
                                              const T* __restrict__ sig, double kscale,
                                              const C2<T>* __restrict__ twg,
                                              const int* __restrict__ revg) {
    // PF > 0: the next column (PF elements per thread, CIN * Mt <= 128 PF) and its
    // row of sigma are fetched into registers while the current one is
    // transformed, so the loads overlap the LDS work of the column before
    using V = C2<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = fg.n;
    const int Mp = Mt + 1;
    V* tw = (V*)smem;
    V* buf = tw + n;
    int* rev = (int*)(buf + CIN * n);
    T* ssig = (T*)(((uintptr_t)(rev + n) + 15) & ~(uintptr_t)15);  // sigma row of the column
    load_tables(tw, rev, twg, revg, n);
    const int kx = blockIdx.y, bm = blockIdx.z;
    const int64_t lstride = (int64_t)(Mt + 1) * n * fg.sz;  // between components
    const bool nyx = (kx == Mt);
    const T ks = (T)kscale;
    const int tid = threadIdx.x;
    const int ky0 = blockIdx.x * zc, ky1 = min(n, (int)(blockIdx.x + 1) * zc);
    const V* colbase = B + (int64_t)bm * CIN * lstride + (int64_t)kx * n * fg.sz;
    auto sigrow = [&](int ky) {
        const int kys = (ky < Mt) ? ky : ky - n;
        return sig + ((int64_t)kx * Mp + (kys < 0 ? -kys : kys)) * Mp;
    };
    constexpr int NP = PF > 0 ? PF : 1;
    constexpr int NS = 4;  // sigma values per thread (Mp <= 512)
    V pre[NP];
    T pres[NS];
    auto fetch = [&](int ky) {
        const V* col = colbase + (int64_t)ky * fg.sz;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int e = tid + k * 128;
            pre[k] = cmk<V>((T)0, (T)0);
            if (e < CIN * Mt) {
                const int c = small_div(e, Mt);
                pre[k] = col[c * lstride + (e - c * Mt)];
            }
        }
        const T* sr = sigrow(ky);
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const int e = tid + k * 128;
            pres[k] = e < Mp ? sr[e] : (T)0;
        }
    };
    if (PF > 0 && ky0 < ky1) fetch(ky0);
    // zc consecutive ky columns per workgroup: the tables above are loaded once
    for (int ky = ky0; ky < ky1; ++ky) {
        V* col = B + (int64_t)bm * CIN * lstride + ((int64_t)kx * n + ky) * fg.sz;
        if (PF > 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const int e = tid + k * 128;
                if (e < CIN * Mt) {
                    const int c = small_div(e, Mt);
                    buf[c * n + (e - c * Mt)] = pre[k];
                }
            }
            for (int q = tid; q < CIN * (n - Mt); q += blockDim.x) {
                const int c = small_div(q, n - Mt);
                buf[c * n + Mt + (q - c * (n - Mt))] = cmk<V>((T)0, (T)0);
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const int e = tid + k * 128;
                if (e < Mp) ssig[e] = pres[k];
            }
            __syncthreads();
            if (ky + 1 < ky1) fetch(ky + 1);
        } else {
            staged_copy<8>(
                CIN * n,
                [&](int q) {
                    const int c = small_div(q, n), z = q - c * n;
                    return (z < Mt) ? col[c * lstride + z] : cmk<V>((T)0, (T)0);
                },
                [&](int q, V v) { buf[q] = v; });
            const T* sr = sigrow(ky);
            staged_copy<4>(Mp, [&](int e) { return sr[e]; }, [&](int e, T v) { ssig[e] = v; });
            __syncthreads();
        }
        fft_lines<V, false>(buf, CIN, n, fg, tw);
        // multiplier
        const int kys = (ky < Mt) ? ky : ky - n;
        const bool nyy = (ky == Mt);
        for (int p = tid; p < n; p += blockDim.x) {
            const int kzi = rev[p];
            const int kzs = (kzi < Mt) ? kzi : kzi - n;
            const bool nyz = (kzi == Mt);
            V g[CIN];
#pragma unroll
            for (int c = 0; c < CIN; ++c) g[c] = buf[c * n + p];
            const T s = ssig[kzs < 0 ? -kzs : kzs];
            // wavenumbers in [-Mt, Mt): the Nyquist index carries -Mt in every direction
            T k[3] = {ks * (T)(nyx ? -Mt : kx), ks * (T)kys, ks * (T)kzs};
            V w[3];
            kpoly<T, KERNEL>(k, g, w, bm & 1);
            if (nyx || nyy || nyz) {
                // Nyquist planes: use the Hermitian part of the multiplier, the mean
                // of its values at k and at k with the Nyquist components negated.
                T kr[3] = {nyx ? -k[0] : k[0], nyy ? -k[1] : k[1], nyz ? -k[2] : k[2]};
                V wr[3];
                kpoly<T, KERNEL>(kr, g, wr, bm & 1);
#pragma unroll
                for (int j = 0; j < 3; ++j) w[j] = cscale(cadd(w[j], wr[j]), (T)0.5);
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) buf[j * n + p] = cscale(w[j], s);
        }
        __syncthreads();
        fft_lines<V, true>(buf, 3, n, fg, tw);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            for (int z = tid; z < Mt; z += blockDim.x) col[c * lstride + z] = buf[c * n + z];
        __syncthreads();
    }
}

// XCD-grouped block order.  Workgroups go to the 8 XCDs (each with its own L2) in
// turn by linear block id, so the G neighbouring blocks that read parts of the
// same 128-byte lines (a pass that moves fewer lines per workgroup than a cache
// line holds) would each fetch those lines into a different L2.  Within every run
// of 8 G linear ids, id j * 8 + x (XCD x, j < G) takes logical block x * G + j:
// the G neighbours run on one XCD at about the same time.  Ids past the last full
// run keep their place.  Returns the logical (x, y, z) block.
template <int G> __device__ __forceinline__ void xcd_blocks(int& bx, int& by, int& bz) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int total = gx * gy * (int)gridDim.z;
    int p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    if (G > 1 && p < total / (8 * G) * (8 * G)) {
        const int o = p % (8 * G);
        p = p - o + (o % 8) * G + o / 8;
    }
    bx = p % gx;
    by = (p / gx) % gy;
    bz = p / (gx * gy);
}
// neighbouring blocks of a pass whose workgroups move L lines of V elements
template <typename V> constexpr int xcd_group(int L) {
    return (int)sizeof(V) * L >= 128 ? 1 : 128 / ((int)sizeof(V) * L);
}

// ---------------------------------------------------------------------------
// y-pass inverse: LZ lines (consecutive z) at fixed (c, kx); keep y < Mt
// ---------------------------------------------------------------------------
template <typename T, int LZ>
__global__ __launch_bounds__(256) void k_fft_yinv(FftGeo fg, int Mt, int c_in,
                                                 const C2<T>* __restrict__ B, C2<T>* __restrict__ A,
                                                 const C2<T>* __restrict__ twg,
                                                 const int* __restrict__ revinvg) {
    using V = C2<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = fg.n;
    V* tw = (V*)smem;
    V* buf = tw + n;
    int* revinv = (int*)(buf + LZ * n);
    load_tables(tw, revinv, twg, revinvg, n);
    // blocks in XCD-grouped order: FP64 (LZ = 2, four blocks per line) 4.11 -> 3.00 ms
    // per step, FP32 (two per line) 0.688 -> 0.678 ms
    int bx, by, bz;
    xcd_blocks<xcd_group<V>(LZ)>(bx, by, bz);
    const int z0 = bx * LZ, kx = by;
    const int bm = bz / 3, c = bz % 3;
    const int64_t bc = (int64_t)bm * c_in + c;
    const int SY = fg.sy, SZ = fg.sz;
    const V* src = B + (bc * (Mt + 1) + kx) * n * SZ;
    staged_copy<8>(
        n * LZ,
        [&](int q) {
            const int ky = q / LZ, r = q % LZ;
            return (z0 + r < Mt) ? src[(int64_t)ky * SZ + z0 + r] : cmk<V>((T)0, (T)0);
        },
        [&](int q, V v) {
            const int ky = q / LZ, r = q % LZ;
            buf[r * n + revinv[ky]] = v;
        });
    __syncthreads();
    fft_lines<V, true>(buf, LZ, n, fg, tw);
    V* dst = A + (bc * (Mt + 1) + kx) * Mt * SY;
    for (int l = 0; l < LZ; ++l) {
        const int z = z0 + l;
        if (z >= Mt) break;
        for (int y = threadIdx.x; y < Mt; y += blockDim.x) dst[(int64_t)z * SY + y] = buf[l * n + y];
    }
}

// ---------------------------------------------------------------------------
// x-pass inverse: C2R of ROWS half spectra (paired), keep x < Mt
// ---------------------------------------------------------------------------
template <typename T, int ROWS>
__global__ __launch_bounds__(256) void k_fft_xinv(FftGeo fg, int Mt, int c_in,
                                                 const C2<T>* __restrict__ A, T* __restrict__ field,
                                                 const C2<T>* __restrict__ twg,
                                                 const int* __restrict__ revinvg) {
    using V = C2<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n = fg.n;
    const int Mp = Mt + 1;
    V* tw = (V*)smem;
    V* buf = tw + n;
    V* H = buf + (ROWS / 2) * n;
    int* revinv = (int*)(H + ROWS * Mp);
    load_tables(tw, revinv, twg, revinvg, n);
    // (the XCD-grouped order measured 1-2 % slower here, in both precisions)
    const int y0 = blockIdx.x * ROWS, z = blockIdx.y;
    const int bm = blockIdx.z / 3, c = blockIdx.z % 3;
    const int64_t bc = (int64_t)bm * c_in + c, fc = (int64_t)bm * 3 + c;
    const int64_t M2 = (int64_t)Mt * Mt;
    const int64_t MA = (int64_t)Mt * fg.sy;  // one kx slab of A
    const V* src = A + bc * Mp * MA + (int64_t)z * fg.sy + y0;
    staged_copy<8>(
        Mp * ROWS,
        [&](int q) {
            const int kx = q / ROWS, r = q % ROWS;
            return (y0 + r < Mt) ? src[(int64_t)kx * MA + r] : cmk<V>((T)0, (T)0);
        },
        [&](int q, V v) {
            const int kx = q / ROWS, r = q % ROWS;
            H[r * Mp + kx] = v;
        });
    __syncthreads();
    for (int l = 0; l < ROWS / 2; ++l) {
        const V* Ha = H + (2 * l) * Mp;
        const V* Hb = H + (2 * l + 1) * Mp;
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const V xa = (k <= Mt) ? Ha[k] : cconj(Ha[n - k]);
            const V xb = (k <= Mt) ? Hb[k] : cconj(Hb[n - k]);
            buf[l * n + revinv[k]] = cmk<V>(xa.x - xb.y, xa.y + xb.x);
        }
    }
    __syncthreads();
    fft_lines<V, true>(buf, ROWS / 2, n, fg, tw);
    T* dst = field + (fc * Mt + z) * M2;
    for (int r = 0; r < ROWS; ++r) {
        const int y = y0 + r;
        if (y >= Mt) break;
        const V* line = buf + (r >> 1) * n;
        for (int x = threadIdx.x; x < Mt; x += blockDim.x) {
            const V v = line[x];
            dst[(int64_t)y * Mt + x] = (r & 1) ? v.y : v.x;
        }
    }
}

// Lines (rows) per workgroup of each pass.  Fewer lines mean less LDS per
// workgroup and so more resident workgroups per CU, whose loads and stores
// overlap the others' LDS transforms; more lines make wider HBM segments where
// a pass writes across lines.  The values are the measured best per pass and
// precision at the headline grids (Mt 250 FP32, 324 FP64).
#ifndef FSE_XROWS32
#define FSE_XROWS32 16
#endif
#ifndef FSE_XINVROWS32
#define FSE_XINVROWS32 8
#endif
#ifndef FSE_YLINES32
#define FSE_YLINES32 8
#endif
#ifndef FSE_XROWS64
#define FSE_XROWS64 4
#endif
#ifndef FSE_XINVROWS64
#define FSE_XINVROWS64 2
#endif
#ifndef FSE_YLINES64
#define FSE_YLINES64 4
#endif
#ifndef FSE_YINVLINES64
#define FSE_YINVLINES64 2
#endif
template <typename T> constexpr int xrows() { return sizeof(T) == 4 ? FSE_XROWS32 : FSE_XROWS64; }
template <typename T> constexpr int xinvrows() { return sizeof(T) == 4 ? FSE_XINVROWS32 : FSE_XINVROWS64; }
template <typename T> constexpr int ylines() { return sizeof(T) == 4 ? FSE_YLINES32 : FSE_YLINES64; }
template <typename T> constexpr int yinvlines() { return sizeof(T) == 4 ? FSE_YLINES32 : FSE_YINVLINES64; }

// Raise a pass's dynamic-LDS limit to `bytes`; remembered per kernel.
template <typename K> void set_lds(K kern, size_t bytes) {
    static std::mutex mu;
    static std::vector<std::pair<const void*, size_t>> done;
    std::lock_guard<std::mutex> lk(mu);
    for (auto& d : done)
        if (d.first == (const void*)kern && d.second >= bytes) return;
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    done.emplace_back((const void*)kern, bytes);
}

// LDS of each pass (bytes) for `lines` complex lines of length n: the twiddle
// table, the lines and the digit-reversal table (the z-pass adds its sigma rows,
// the x-inverse pass its ROWS half spectra).
constexpr size_t LDS_BYTES = 160 * 1024;
template <typename T> size_t lds_lines(int n, int lines) {
    return sizeof(C2<T>) * (size_t)n * (size_t)(1 + lines) + sizeof(int) * (size_t)n;
}
template <typename T> size_t lds_xinv(int n, int Mt, int rows) {
    return sizeof(C2<T>) * ((size_t)n * (size_t)(1 + rows / 2) + (size_t)rows * (Mt + 1)) + sizeof(int) * (size_t)n;
}
template <typename T> size_t lds_z(int n, int Mt, int lines, int sigrows) {
    return lds_lines<T>(n, lines) + 16 + sizeof(T) * (size_t)sigrows * (Mt + 1);
}
// The largest count, halving from dflt down to lo, that is at most cap (when
// cap > 0) and whose LDS fits (lo when none does: fft_fits has ruled that out).
template <typename F> int fit_count(int dflt, int lo, int cap, F need) {
    for (int c = dflt; c > lo; c /= 2)
        if ((cap <= 0 || c <= cap) && need(c) <= LDS_BYTES) return c;
    return lo;
}

template <typename T, int R>
void launch_x(const FftGeo& fg, int Mt, const T* grid, C2<T>* A, int ncomp, const C2<T>* tw, const int* revinv,
              hipStream_t st) {
    const size_t sh = lds_lines<T>(fg.n, R / 2);
    set_lds(k_fft_x<T, R>, sh);
    hipLaunchKernelGGL((k_fft_x<T, R>), dim3((Mt + R - 1) / R, Mt, ncomp), dim3(256), sh, st, fg, Mt, grid, A, tw,
                       revinv);
}
template <typename T, int LZ>
void launch_y(const FftGeo& fg, int Mt, const C2<T>* A, C2<T>* B, int ncomp, const C2<T>* tw, const int* revinv,
              hipStream_t st) {
    const size_t sh = lds_lines<T>(fg.n, LZ);
    set_lds(k_fft_y<T, LZ>, sh);
    hipLaunchKernelGGL((k_fft_y<T, LZ>), dim3((Mt + LZ - 1) / LZ, Mt + 1, ncomp), dim3(256), sh, st, fg, Mt, A, B,
                       tw, revinv);
}
template <typename T, int LZ>
void launch_yinv(const FftGeo& fg, int Mt, int c_in, int batch, const C2<T>* B, C2<T>* A, const C2<T>* tw,
                 const int* revinv, hipStream_t st) {
    const size_t sh = lds_lines<T>(fg.n, LZ);
    set_lds(k_fft_yinv<T, LZ>, sh);
    hipLaunchKernelGGL((k_fft_yinv<T, LZ>), dim3((Mt + LZ - 1) / LZ, Mt + 1, 3 * batch), dim3(256), sh, st, fg, Mt,
                       c_in, B, A, tw, revinv);
}
template <typename T, int R>
void launch_xinv(const FftGeo& fg, int Mt, int c_in, int batch, const C2<T>* A, T* field, const C2<T>* tw,
                 const int* revinv, hipStream_t st) {
    const size_t sh = lds_xinv<T>(fg.n, Mt, R);
    set_lds(k_fft_xinv<T, R>, sh);
    hipLaunchKernelGGL((k_fft_xinv<T, R>), dim3((Mt + R - 1) / R, Mt, 3 * batch), dim3(256), sh, st, fg, Mt, c_in,
                       A, field, tw, revinv);
}

}  // namespace

// Whether every pass of the transforms fits in LDS at grid side Mt (n = 2 Mt),
// with its smallest line count; the launchers below take the largest count that fits.
bool fft_fits(int kernel, int elem_bytes, int Mt) {
    const int n = 2 * Mt;
    const int cin = kernel == FSE_STRESSLET ? 6 : 3;
    auto ok = [&](auto tag) {
        using T = decltype(tag);
        return lds_lines<T>(n, 1) <= LDS_BYTES && lds_xinv<T>(n, Mt, 2) <= LDS_BYTES &&
               lds_z<T>(n, Mt, cin, 1) <= LDS_BYTES;
    };
    return elem_bytes == 4 ? ok(0.0f) : ok(0.0);
}

int fft_max_mt(int kernel, int elem_bytes) {
    int Mt = 1024;
    while (Mt > 1 && !fft_fits(kernel, elem_bytes, Mt)) --Mt;
    return Mt;
}

template <typename T>
void launch_fft_forward(const FftGeo& fg, const GridGeo& g, const T* grid, void* Av, void* Bv, int ncomp,
                        const T* tw, const int* rev, const int* revinv, hipStream_t st, int passes) {
    using V = C2<T>;
    (void)rev;
    const int Mt = g.Mt, n = fg.n;
    V* A = (V*)Av;
    V* B = (V*)Bv;
    const V* twv = (const V*)tw;
    if (passes & 1) {
        // rows per workgroup: the measured best where it fits, fewer on long lines
        const int R = fit_count(xrows<T>(), 2, fg.lines_cap, [&](int r) { return lds_lines<T>(n, r / 2); });
        switch (R) {
            case 16: if constexpr (xrows<T>() >= 16) launch_x<T, 16>(fg, Mt, grid, A, ncomp, twv, revinv, st); break;
            case 8: if constexpr (xrows<T>() >= 8) launch_x<T, 8>(fg, Mt, grid, A, ncomp, twv, revinv, st); break;
            case 4: if constexpr (xrows<T>() >= 4) launch_x<T, 4>(fg, Mt, grid, A, ncomp, twv, revinv, st); break;
            default: launch_x<T, 2>(fg, Mt, grid, A, ncomp, twv, revinv, st); break;
        }
    }
    if (passes & 2) {
        const int LZ = fit_count(ylines<T>(), 1, fg.lines_cap, [&](int l) { return lds_lines<T>(n, l); });
        switch (LZ) {
            case 8: if constexpr (ylines<T>() >= 8) launch_y<T, 8>(fg, Mt, A, B, ncomp, twv, revinv, st); break;
            case 4: if constexpr (ylines<T>() >= 4) launch_y<T, 4>(fg, Mt, A, B, ncomp, twv, revinv, st); break;
            case 2: if constexpr (ylines<T>() >= 2) launch_y<T, 2>(fg, Mt, A, B, ncomp, twv, revinv, st); break;
            default: launch_y<T, 1>(fg, Mt, A, B, ncomp, twv, revinv, st); break;
        }
    }
}

template <typename T>
void launch_fft_zscale(const FftGeo& fg, const GridGeo& g, int kernel, void* Bv, int c_in, int batch,
                       const T* sig, double kscale, const T* tw, const int* rev, const int* revinv,
                       hipStream_t st) {
    using V = C2<T>;
    (void)revinv;
    const int Mt = g.Mt, n = fg.n;
    V* B = (V*)Bv;
    constexpr int ZC = 4;  // ky columns per workgroup
    dim3 grd((n + ZC - 1) / ZC, Mt + 1, batch);
    // LDS: twiddles, CIN lines, index table, sigma row
    const size_t sh = lds_z<T>(n, Mt, c_in, 1);
    const int need = (c_in * Mt + 127) / 128;  // column elements per thread
    // the prefetch registers cost the FP32 kernel a third of its occupancy (the
    // LDS allows eight blocks per CU there), a net loss; FP64 is LDS-limited to
    // three blocks per CU, so the overlap is free
    const bool sig_ok = Mt + 1 <= 4 * 128;
#define ZLAUNCH(K, CI, PFV)                                                                                  \
    do {                                                                                                     \
        set_lds(k_fft_z<T, K, CI, PFV>, sh);                                                                 \
        hipLaunchKernelGGL((k_fft_z<T, K, CI, PFV>), grd, dim3(128), sh, st, fg, Mt, ZC, B, sig, kscale,  \
                           (const V*)tw, rev);                                                               \
    } while (0)
#define ZPICK(K, CI)                                                                                         \
    do {                                                                                                     \
        if constexpr (sizeof(T) == 8) {                                                                      \
            if (sig_ok && need <= 6) ZLAUNCH(K, CI, 6);                                                      \
            else if (sig_ok && need <= 8) ZLAUNCH(K, CI, 8);                                                 \
            else if (sig_ok && need <= 12) ZLAUNCH(K, CI, 12);                                               \
            else ZLAUNCH(K, CI, 0);                                                                          \
        } else {                                                                                             \
            ZLAUNCH(K, CI, 0);                                                                               \
        }                                                                                                    \
    } while (0)
    // FP32 three-component kernels: FSE_ZB32 columns (3 FSE_ZB32 lines) transformed
    // together by FSE_ZBT32 threads, FSE_ZBG32 such groups per workgroup (measured
    // at Mt = 250: 1.05 ms against 1.15 ms one column at a time), where their
    // lines fit in LDS
#ifndef FSE_ZB32
#define FSE_ZB32 3
#endif
#ifndef FSE_ZBT32
#define FSE_ZBT32 256
#endif
    if constexpr (sizeof(T) == 4 && FSE_ZB32 > 1) {
        constexpr int ZB = FSE_ZB32;
        const size_t shb = lds_z<T>(n, Mt, 3 * ZB, ZB);
        if ((kernel == FSE_STOKESLET || kernel == FSE_ROTLET) && shb <= LDS_BYTES && fg.lines_cap == 0) {
#ifndef FSE_ZBG32
#define FSE_ZBG32 2
#endif
            constexpr int ZCB = FSE_ZBG32 * FSE_ZB32;
            const dim3 grdb((n + ZCB - 1) / ZCB, Mt + 1, batch);
#define ZBLAUNCH(K)                                                                                          \
    do {                                                                                                     \
        set_lds(k_fft_zb<T, K, ZB>, shb);                                                                    \
        hipLaunchKernelGGL((k_fft_zb<T, K, ZB>), grdb, dim3(FSE_ZBT32), shb, st, fg, Mt, ZCB, B, sig,        \
                           kscale, (const V*)tw, rev);                                                       \
    } while (0)
            if (kernel == FSE_STOKESLET) ZBLAUNCH(FSE_STOKESLET);
            else ZBLAUNCH(FSE_ROTLET);
#undef ZBLAUNCH
            return;
        }
    }
    if (kernel == FSE_STOKESLET) ZPICK(FSE_STOKESLET, 3);
    else if (kernel == FSE_ROTLET) ZPICK(FSE_ROTLET, 3);
    else if (kernel == KTADJ) ZPICK(KTADJ, 3);  // batch = 2 x members: halves of the 6 outputs
    else if (kernel == KSCALAR) ZPICK(KSCALAR, 3);
    else ZPICK(FSE_STRESSLET, 6);
#undef ZPICK
#undef ZLAUNCH
}

template <typename T>
void launch_fft_inverse(const FftGeo& fg, const GridGeo& g, void* Bv, void* Av, T* field, int c_in,
                        int batch, const T* tw, const int* rev, const int* revinv, hipStream_t st,
                        int passes) {
    using V = C2<T>;
    (void)rev;
    const int Mt = g.Mt, n = fg.n;
    V* A = (V*)Av;
    V* B = (V*)Bv;
    const V* twv = (const V*)tw;
    if (passes & 1) {
        const int LZ = fit_count(yinvlines<T>(), 1, fg.lines_cap, [&](int l) { return lds_lines<T>(n, l); });
        switch (LZ) {
            case 8: if constexpr (yinvlines<T>() >= 8) launch_yinv<T, 8>(fg, Mt, c_in, batch, B, A, twv, revinv, st); break;
            case 4: if constexpr (yinvlines<T>() >= 4) launch_yinv<T, 4>(fg, Mt, c_in, batch, B, A, twv, revinv, st); break;
            case 2: if constexpr (yinvlines<T>() >= 2) launch_yinv<T, 2>(fg, Mt, c_in, batch, B, A, twv, revinv, st); break;
            default: launch_yinv<T, 1>(fg, Mt, c_in, batch, B, A, twv, revinv, st); break;
        }
    }
    if (passes & 2) {
        const int R = fit_count(xinvrows<T>(), 2, fg.lines_cap, [&](int r) { return lds_xinv<T>(n, Mt, r); });
        switch (R) {
            case 8: if constexpr (xinvrows<T>() >= 8) launch_xinv<T, 8>(fg, Mt, c_in, batch, A, field, twv, revinv, st); break;
            case 4: if constexpr (xinvrows<T>() >= 4) launch_xinv<T, 4>(fg, Mt, c_in, batch, A, field, twv, revinv, st); break;
            default: launch_xinv<T, 2>(fg, Mt, c_in, batch, A, field, twv, revinv, st); break;
        }
    }
}

#define INST(T)                                                                                      \
    template void launch_fft_forward<T>(const FftGeo&, const GridGeo&, const T*, void*, void*, int,  \
                                        const T*, const int*, const int*, hipStream_t, int);         \
    template void launch_fft_zscale<T>(const FftGeo&, const GridGeo&, int, void*, int, int, const T*, \
                                       double, const T*, const int*, const int*, hipStream_t);       \
    template void launch_fft_inverse<T>(const FftGeo&, const GridGeo&, void*, void*, T*, int, int,   \
                                        const T*, const int*, const int*, hipStream_t, int);
INST(float)
INST(double)
#undef INST

}  // namespace fse
