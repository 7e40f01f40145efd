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
// Spreading: output-stationary (k_spread_mfma in FP32, on the matrix cores;
// k_spread in FP64); every node is written exactly once, coalesced, by the lane
// that accumulated it: no floating-point atomics and no clearing of the grid.
// A node's terms are summed in the sorted point order, so repeated runs agree
// bit for bit.
//
// Quadrature: one workgroup per bin stages the (TB+P-1)^3 block of the field
// that the bin's windows cover in LDS (when it fits) and each wave reduces one
// point at a time from LDS; otherwise the field is read from global memory.
#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "fse_common.h"

namespace fse {

namespace {

// Gaussian factor exp(-alpha h^2 e^2) as gauss(gauss_coef(alpha h^2) e^2): in FP32
// the hardware base-2 exponential with log2(e) folded into the coefficient (the
// rounding of the argument then dominates, as it does for expf of a rounded
// -alpha h^2 e^2), in FP64 exp.
template <typename T> __host__ __device__ inline T gauss_coef(double ahh) {
    return sizeof(T) == 4 ? (T)(-ahh * 1.4426950408889634) : (T)(-ahh);
}
template <typename T> __device__ __forceinline__ T gauss(T y);
template <> __device__ __forceinline__ float gauss<float>(float y) { return __builtin_amdgcn_exp2f(y); }
template <> __device__ __forceinline__ double gauss<double>(double y) { return exp(y); }


// One point of a chunk, held in registers between its load and its staging.
template <typename T, int NC> struct ChunkPoint {
    int bp;       // packed window start; -1: no point
    T cc[3], vv[NC];
};

// Thread t < CH loads point base + t of the bin range ending at j1 (all of its
// loads at once: one memory latency).
// With src2 (NC = 6): components 0-2 from src_s and 3-5 from src2, both 3 per point.
template <typename T, int NC, int CH>
__device__ __forceinline__ void load_point(ChunkPoint<T, NC>& pt, int base, int j1, int bm, int64_t n,
                                           const int* __restrict__ bpack_s, const T* __restrict__ coff_s,
                                           const T* __restrict__ src_s, const T* __restrict__ src2) {
    pt.bp = -1;
    const int j = base + (int)threadIdx.x;
    if ((int)threadIdx.x < CH && j < j1) {
        pt.bp = bpack_s[j];
#pragma unroll
        for (int d = 0; d < 3; ++d) pt.cc[d] = coff_s[3 * (int64_t)j + d];
        if (NC == 6 && src2) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pt.vv[c] = src_s[((int64_t)bm * n + j) * 3 + c];
                pt.vv[3 + c] = src2[((int64_t)bm * n + j) * 3 + c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < NC; ++c) pt.vv[c] = src_s[((int64_t)bm * n + j) * NC + c];
        }
    }
}

// Stage the loaded points whose window overlaps the core (lox, loy, loz) +
// [0,16) x [0,16) x [0,TZ) into LDS, compacted in thread order (wave ballots,
// then the waves' counts in wave order), so the staged order is the sorted
// point order.  Returns the number staged, the same in every thread.  s_wc
// holds the four waves' counts; it is written before the first barrier, which
// is safe because every read of it in the previous call precedes that call's
// second barrier.
template <typename T, int NC, int TZ>
__device__ __forceinline__ int stage_points(const ChunkPoint<T, NC>& pt, int P, int lox, int loy, int loz,
                                            T (*s_c)[3], T (*s_v)[NC], int* s_bp, int* s_wc) {
    bool ov = false;
    if (pt.bp >= 0) {
        const int bx = pt.bp & 1023, by = (pt.bp >> 10) & 1023, bz = pt.bp >> 20;
        ov = bx <= lox + 15 && bx + P > lox && by <= loy + 15 && by + P > loy && bz <= loz + TZ - 1 &&
             bz + P > loz;
    }
    const unsigned long long m = __ballot(ov);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) s_wc[wid] = __popcll(m);
    __syncthreads();
    const int c0 = s_wc[0], c1 = s_wc[1], c2 = s_wc[2], c3 = s_wc[3];
    if (ov) {
        const int k = (wid > 0 ? c0 : 0) + (wid > 1 ? c1 : 0) + (wid > 2 ? c2 : 0) +
                      __popcll(m & ((1ull << lane) - 1ull));
        s_bp[k] = pt.bp;
#pragma unroll
        for (int d = 0; d < 3; ++d) s_c[k][d] = pt.cc[d];
#pragma unroll
        for (int c = 0; c < NC; ++c) s_v[k][c] = pt.vv[c];
    }
    __syncthreads();
    return c0 + c1 + c2 + c3;
}

// Gaussian factors of the cnt staged points at the core's 16 + 16 + TZ node
// offsets, zero outside the window: one work item per point and direction.
// The caller synchronises before reading them.
template <typename T, int TZ>
__device__ __forceinline__ void chunk_factors(const GridGeo& g, int cnt, int lox, int loy, int loz,
                                              T (*s_w)[32 + TZ], T (*s_c)[3], const int* s_bp) {
    const int P = g.P;
    const T gk = gauss_coef<T>(g.ahh);
    const T g2 = sizeof(T) == 8 ? gauss<T>((T)2 * gk) : (T)0;  // exp(2 gk), FP64 recurrence
    const T half = (T)(0.5 * (P - 1));
    for (int q = threadIdx.x; q < cnt * 3; q += 256) {
        const int k = small_div(q, 3), d = q - 3 * k;
        const int bp = s_bp[k];
        const int b = d == 0 ? (bp & 1023) : (d == 1 ? ((bp >> 10) & 1023) : (bp >> 20));
        const int lo = d == 0 ? lox : (d == 1 ? loy : loz);
        const int i0 = lo - b;                      // window index of core offset 0
        // window coordinate there: the offset plus an exact half-integer, so
        // the coordinate e carries one rounding (adding half first would round
        // at the magnitude of P / 2 for every node)
        const T sc = s_c[k][d], k0 = half - (T)i0;
        T* dst = &s_w[k][16 * d];
        if constexpr (sizeof(T) == 4) {
#pragma unroll
            for (int o = 0; o < 16; ++o) {
                if (o >= TZ && d == 2) break;
                const T e = sc + (k0 - (T)o);
                const T w = gauss<T>(gk * e * e);
                dst[o] = (unsigned)(i0 + o) < (unsigned)P ? w : (T)0;  // 0 <= i0 + o < P
            }
        } else {
            // FP64: two exponentials per point and direction, the rest by the
            // recurrence of fast Gaussian gridding: with e(o) = e(o - 1) - 1,
            // g(o + 1) = g(o) r(o), r(o) = exp(gk (1 - 2 e(o))), r(o + 1) = r(o) exp(2 gk),
            // started at the window's first node inside the core (inside the window
            // |e| <= P/2, so nothing underflows; 2 o + 2 roundings, ~4e-15 relative)
            const int os = i0 < 0 ? -i0 : 0;
            const T es = sc + (k0 - (T)os);
            T w = gauss<T>(gk * es * es);
            T r = gauss<T>(gk * ((T)1 - (T)2 * es));
#pragma unroll
            for (int o = 0; o < 16; ++o) {
                if (o >= TZ && d == 2) break;
                dst[o] = (unsigned)(i0 + o) < (unsigned)P ? w : (T)0;  // 0 <= i0 + o < P
                const bool adv = o >= os;
                w = adv ? w * r : w;
                r = adv ? r * g2 : r;
            }
        }
    }
}

// Output-stationary spreading.  The workgroup (256 threads) owns a 16 x 16 x TZ
// core of grid nodes; each wave covers an 8 x 8 tile of its columns and each
// thread keeps the z-column (x, y, 0..TZ-1) of the core in registers for every
// component, so no accumulation ever needs an atomic (LDS float atomics are
// slow on this hardware).  Candidate points, those of the bins whose window
// starts can reach the core, are staged in LDS in chunks of CH, compacted to
// the ones whose window overlaps the core, and their Gaussian factors at the
// core's 16 + 16 + TZ node offsets (zero outside the window) are computed
// cooperatively into LDS.  Each wave then lists the staged points whose window
// meets its 8 x 8 tile, each entry tagged with the groups of 4 core z-nodes the
// window covers, and walks its list: the entries are read 64 at a time into
// lanes and taken from there one per visit, the point's factors and values come
// in as LDS broadcasts, and only the tagged z-groups are accumulated.
template <typename T, int NC, int TZ, int CH>
__global__ __launch_bounds__(256) void k_spread(GridGeo g, const int* __restrict__ tile_start,
                                               const int* __restrict__ bpack_s,
                                               const T* __restrict__ coff_s,
                                               const T* __restrict__ src_s, int64_t n, T* grid,
                                               const T* __restrict__ src2, T* grid2) {
    constexpr int NW = 32 + TZ;  // factors per point: x (16), y (16), z (TZ)
    __shared__ __align__(16) T s_w[CH][NW];
    __shared__ T s_c[CH][3];
    __shared__ T s_v[CH][NC];
    __shared__ int s_bp[CH];
    __shared__ int s_wc[4];
    // per wave: the staged points whose window meets its tile, as k | (z-group mask << 8)
    __shared__ unsigned short s_list[4][CH];
    static_assert(CH <= 256 && TZ <= 32, "list entries: point index byte and z-group mask");

    const int Mt = g.Mt, P = g.P, TB = g.TS, nb = g.nt;
    const int ncxy = (Mt + 15) / 16;
    const int t = blockIdx.x;
    const int cx = t % ncxy, cy = (t / ncxy) % ncxy, cz = t / (ncxy * ncxy);
    const int bm = blockIdx.y;
    const int lox = cx * 16, loy = cy * 16, loz = cz * TZ;
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wx0 = (wid & 1) * 8, wy0 = (wid >> 1) * 8;  // the wave's 8 x 8 tile in the core
    const int tx = wx0 + (lane & 7), ty = wy0 + (lane >> 3);
    const int gx = lox + tx, gy = loy + ty;

    T acc[TZ][NC];
#pragma unroll
    for (int z = 0; z < TZ; ++z)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[z][c] = (T)0;

    // bins holding window starts b in [lo - P + 1, lo + ext - 1] ∩ [0, Mt - P]
    const int bx0 = max(0, lox - P + 1) / TB, bx1 = min(Mt - P, lox + 15) / TB;
    const int by0 = max(0, loy - P + 1) / TB, by1 = min(Mt - P, loy + 15) / TB;
    const int bz0 = max(0, loz - P + 1) / TB, bz1 = min(Mt - P, loz + TZ - 1) / TB;
    // The chunks run as one sequence over the bin rows (sz, sy), row r = (sz - bz0)
    // nry + sy - by0, each row's range cut into chunks of CH; the next chunk's range
    // and points are loaded while the current one is processed (as in k_spread_mfma)
    const int nry = by1 - by0 + 1, nrows = (nry > 0 && bz1 >= bz0) ? (bz1 - bz0 + 1) * nry : 0;
    auto find_row = [&](int r, int& jb, int& je) {
        for (; r < nrows; ++r) {
            const int rz = r / nry;
            const int row = ((bz0 + rz) * nb + by0 + (r - rz * nry)) * nb;
            jb = tile_start[row + bx0];
            je = tile_start[row + bx1 + 1];
            if (jb < je) break;
        }
        return r;
    };
    int r = 0, base = 0, end = 0;
    r = find_row(0, base, end);
    ChunkPoint<T, NC> pt;
    if (r < nrows) load_point<T, NC, CH>(pt, base, end, bm, n, bpack_s, coff_s, src_s, src2);
    while (r < nrows) {
        const int cnt = stage_points<T, NC, TZ>(pt, P, lox, loy, loz, s_c, s_v, s_bp, s_wc);
        int nr = r, nbase = base + CH, nend = end;
        if (nbase >= end) nr = find_row(r + 1, nbase, nend);
        if (nr < nrows) load_point<T, NC, CH>(pt, nbase, nend, bm, n, bpack_s, coff_s, src_s, src2);
        chunk_factors<T, TZ>(g, cnt, lox, loy, loz, s_w, s_c, s_bp);
        // this wave's list: the staged points whose window reaches its 8 x 8 tile
        int nl = 0;
        for (int k0 = 0; k0 < cnt; k0 += 64) {
            const int k = k0 + lane;
            bool hit = false;
            unsigned zm = 0;  // groups of 4 core z-nodes the window meets
            if (k < cnt) {
                const int bp = s_bp[k];
                const int bx = bp & 1023, by = (bp >> 10) & 1023, bz = bp >> 20;
                hit = !(bx > lox + wx0 + 7 || bx + P <= lox + wx0 || by > loy + wy0 + 7 ||
                        by + P <= loy + wy0);
                const int zlo = max(bz, loz) - loz, zhi = min(bz + P, loz + TZ) - loz;
#pragma unroll
                for (int z4 = 0; z4 < TZ; z4 += 4)
                    if (z4 < zhi && z4 + 4 > zlo) zm |= 1u << (z4 / 4);
            }
            const unsigned long long m = __ballot(hit);
            if (hit)
                s_list[wid][nl + __popcll(m & ((1ull << lane) - 1ull))] = (unsigned short)(k | (zm << 8));
            nl += __popcll(m);
        }
        __syncthreads();
        // list entries come 64 at a time, one per lane, and are read from the
        // lanes as the wave visits them (no LDS round trip per visit)
        for (int l0 = 0; l0 < nl; l0 += 64) {
          const int mine = l0 + lane < nl ? (int)s_list[wid][l0 + lane] : 0;
          const int cl = min(64, nl - l0);
          for (int li = 0; li < cl; ++li) {
            const int ent = __builtin_amdgcn_readlane(mine, li);
            const int k = ent & 255;
            const unsigned zm = (unsigned)ent >> 8;
            const T wxy = s_w[k][tx] * s_w[k][16 + ty];
            T v[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) v[c] = s_v[k][c];
            T wz[TZ];
#pragma unroll
            for (int z = 0; z < TZ; ++z) wz[z] = s_w[k][32 + z];
            // z in groups of 4 that meet the window (the factors are zero outside it)
#pragma unroll
            for (int z4 = 0; z4 < TZ; z4 += 4) {
                if (zm & (1u << (z4 / 4))) {
#pragma unroll
                    for (int z = z4; z < z4 + 4; ++z) {
                        const T w = wxy * wz[z];
#pragma unroll
                        for (int c = 0; c < NC; ++c) acc[z][c] += w * v[c];
                    }
                }
            }
          }
        }
        __syncthreads();
        r = nr;
        base = nbase;
        end = nend;
    }
    if (gx < Mt && gy < Mt) {
        const int64_t M3 = (int64_t)Mt * Mt * Mt;
#pragma unroll
        for (int z = 0; z < TZ; ++z) {
            const int gz = loz + z;
            if (gz < Mt) {
                const int64_t o = ((int64_t)gz * Mt + gy) * Mt + gx;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    // with grid2: components 0-2 to grid, 3-5 to grid2, 3 per batch member
                    T* gd = (NC == 6 && grid2) ? (c < 3 ? grid + (int64_t)bm * 3 * M3 : grid2 + ((int64_t)bm * 3 - 3) * M3)
                                               : grid + (int64_t)bm * NC * M3;
                    gd[(int64_t)c * M3 + o] = acc[z][c];
                }
            }
        }
    }
}

// FP32 spreading on the matrix cores.  Same cores and chunks as k_spread
// (TZ = 16), but a wave's contribution from four listed points k is one product
// per component c and 16-node xy block:
//   acc_c[z][xy] += sum_k (wz_k(z) v_k[c]) (wx_k(x) wy_k(y)),
// a 16 x 4 by 4 x 16 matrix product (v_mfma_f32_16x16x4f32; z rows, points
// along k, xy nodes as columns).  Lane l supplies A[z = l mod 16][k = l / 16]
// and B[k = l / 16][xy = l mod 16] and holds D[z = 4 (l / 16) + j][xy = l mod 16],
// j = 0..3.  The wave's 8 x 8 tile is four 4 x 4 blocks (xy = 4 y' + x' within
// a block), and each block keeps its own list of the staged points whose window
// meets it, so a point costs products only on the blocks it reaches (2.4 of 4
// on average at P = 11).  The four lists are walked together, one group of four
// points from each per step, so every step still issues up to 4 c independent
// products.  Every listed point costs the full 16 z-rows (no z-group skipping)
// at twice the non-packed FP32 FMA rate of the vector units.
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int NC, int CH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_spread_mfma(GridGeo g, const int* __restrict__ tile_start,
                                                    const int* __restrict__ bpack_s,
                                                    const float* __restrict__ coff_s,
                                                    const float* __restrict__ src_s, int64_t n,
                                                    float* grid, const float* __restrict__ src2,
                                                    float* grid2) {
    constexpr int TZ = 16;
    __shared__ __align__(16) float s_w[CH][32 + TZ];
    __shared__ float s_c[CH][3];
    __shared__ float s_v[CH][NC];
    __shared__ int s_bp[CH];
    __shared__ int s_wc[4];
    __shared__ unsigned char s_list[4][4][CH];  // per wave and 4 x 4 block: the staged points that meet it
    static_assert(CH <= 256, "list entries are point index bytes");
    const int Mt = g.Mt, P = g.P, TB = g.TS, nb = g.nt;
    const int ncxy = (Mt + 15) / 16;
    const int t = blockIdx.x;
    const int cx = t % ncxy, cy = (t / ncxy) % ncxy, cz = t / (ncxy * ncxy);
    const int bm = blockIdx.y;
    const int lox = cx * 16, loy = cy * 16, loz = cz * TZ;
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wx0 = (wid & 1) * 8, wy0 = (wid >> 1) * 8;  // the wave's 8 x 8 tile in the core
    const int kl = lane >> 4, cl = lane & 15;              // operand slot: point kl, row / column cl
    const int xo = wx0 + (cl & 3), yo = wy0 + (cl >> 2);   // xy node of column cl in block 0
    // block b covers x in xo + 4 (b & 1), y in yo + 4 (b >> 1)

    f32x4 acc[NC][4];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[c][b] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int bx0 = max(0, lox - P + 1) / TB, bx1 = min(Mt - P, lox + 15) / TB;
    const int by0 = max(0, loy - P + 1) / TB, by1 = min(Mt - P, loy + 15) / TB;
    const int bz0 = max(0, loz - P + 1) / TB, bz1 = min(Mt - P, loz + TZ - 1) / TB;
    // The chunks run as one sequence over the bin rows (sz, sy), row r = (sz - bz0)
    // nry + sy - by0, each row's range cut into chunks of CH.  The next chunk's
    // range and points are loaded while the current one is processed, so neither
    // memory latency waits behind the chunk's barriers.
    const int nry = by1 - by0 + 1, nrows = (nry > 0 && bz1 >= bz0) ? (bz1 - bz0 + 1) * nry : 0;
    // first non-empty row from r on: its range in [jb, je), or r = nrows
    auto find_row = [&](int r, int& jb, int& je) {
        for (; r < nrows; ++r) {
            const int rz = r / nry;
            const int row = ((bz0 + rz) * nb + by0 + (r - rz * nry)) * nb;
            jb = tile_start[row + bx0];
            je = tile_start[row + bx1 + 1];
            if (jb < je) break;
        }
        return r;
    };
    int r = 0, base = 0, end = 0;
    r = find_row(0, base, end);
    ChunkPoint<float, NC> pt;
    if (r < nrows) load_point<float, NC, CH>(pt, base, end, bm, n, bpack_s, coff_s, src_s, src2);
    while (r < nrows) {
        const int cnt = stage_points<float, NC, TZ>(pt, P, lox, loy, loz, s_c, s_v, s_bp, s_wc);
        // the next chunk: the rest of this row, else the next non-empty row
        int nr = r, nbase = base + CH, nend = end;
        if (nbase >= end) nr = find_row(r + 1, nbase, nend);
        if (nr < nrows) load_point<float, NC, CH>(pt, nbase, nend, bm, n, bpack_s, coff_s, src_s, src2);
        chunk_factors<float, TZ>(g, cnt, lox, loy, loz, s_w, s_c, s_bp);
        int nl[4] = {0, 0, 0, 0};
        for (int k0 = 0; k0 < cnt; k0 += 64) {
            const int k = k0 + lane;
            bool hx[2] = {false, false}, hy[2] = {false, false};
            if (k < cnt) {
                const int bp = s_bp[k];
                const int bx = bp & 1023, by = (bp >> 10) & 1023;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int x0 = lox + wx0 + 4 * h, y0 = loy + wy0 + 4 * h;
                    hx[h] = !(bx > x0 + 3 || bx + P <= x0);
                    hy[h] = !(by > y0 + 3 || by + P <= y0);
                }
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const bool hit = hx[b & 1] && hy[b >> 1];
                const unsigned long long m = __ballot(hit);
                if (hit) s_list[wid][b][nl[b] + __popcll(m & ((1ull << lane) - 1ull))] = (unsigned char)k;
                nl[b] += __popcll(m);
            }
        }
        __syncthreads();
        // step g takes listed points 4 g .. 4 g + 3 of every block whose list
        // reaches that far; slots past a list get zero A operands (their B
        // operands read point 0's factors, which are finite)
        const int ng = (max(max(nl[0], nl[1]), max(nl[2], nl[3])) + 3) >> 2;
        for (int l0 = 0; l0 < 4 * ng; l0 += 4) {
            // the four blocks' entries in one LDS round trip (the slot index is
            // clamped into the list row; entries past a list are not used)
            int kk[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) kk[b] = s_list[wid][b][min(l0 + kl, CH - 1)];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if (l0 < nl[b]) {
                    const bool ok = l0 + kl < nl[b];
                    const int k = ok ? kk[b] : 0;
                    const float wzk = s_w[k][32 + cl];
                    const float wz = ok ? wzk : 0.f;
                    const float bb = s_w[k][xo + 4 * (b & 1)] * s_w[k][16 + yo + 4 * (b >> 1)];
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        acc[c][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(wz * s_v[k][c], bb, acc[c][b], 0, 0, 0);
                }
            }
        }
        __syncthreads();
        r = nr;
        base = nbase;
        end = nend;
    }
    const int64_t M3 = (int64_t)Mt * Mt * Mt;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int gx = lox + xo + 4 * (b & 1), gy = loy + yo + 4 * (b >> 1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gz = loz + 4 * kl + j;
            if (gx < Mt && gy < Mt && gz < Mt) {
                const int64_t o = ((int64_t)gz * Mt + gy) * Mt + gx;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    // with grid2: components 0-2 to grid, 3-5 to grid2, 3 per batch member
                    float* gd = (NC == 6 && grid2) ? (c < 3 ? grid + (int64_t)bm * 3 * M3
                                                            : grid2 + ((int64_t)bm * 3 - 3) * M3)
                                                   : grid + (int64_t)bm * NC * M3;
                    gd[(int64_t)c * M3 + o] = acc[c][b][j];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Quadrature with the bin's field block staged in LDS, NCS of the 3 field
// components at a time (3 when the (TB+P-1)^3 block of all of them fits,
// else 1).  One wave per point; lane l owns the window rows r = l, l + 64, ...
// (r = iy + P iz) and sums along x with the x-weights broadcast from LDS, so
// every LDS read of the field feeds one or two FMAs and no index arithmetic.
//   MODE 0: u = sum g F (value).
//   MODE 1: dx  = sum grad g (p . F), p = the point's vector (the forward
//           field contracted with w; the first contribution overwrites).
//   MODE 2: out = sum g F and dx += sum grad g (p . F).
//   MODE 3 (k_gather_col only): mode 2 whose first contribution overwrites dx,
//           for the forward value and the first gradient term in one sweep.
// ---------------------------------------------------------------------------
constexpr int GW = 4;  // waves per quadrature workgroup

template <typename T, int MODE, int NCS>
__global__ __launch_bounds__(64 * GW) void k_gather_lds(GridGeo g, const int* __restrict__ tile_start,
                                                       const int* __restrict__ perm_s,
                                                       const int* __restrict__ bpack_s,
                                                       const T* __restrict__ coff_s,
                                                       const T* __restrict__ field,
                                                       const T* __restrict__ vec_s, int64_t n, int batch,
                                                       T* out, T* dx) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = (T*)smem_raw;
    // per wave: wx, wy, wz, dwx, dwy, dwz; zero beyond P
    __shared__ __align__(16) T s_w[GW][6][32];
    const int Mt = g.Mt, P = g.P, TB = g.TS, nb = g.nt;
    const int E = TB + P - 1, E2 = E * E, E3 = E2 * E;
    const int E3S = E3 + 4;  // component stride: 4 zero pads absorb the x-unroll overrun
    const int64_t M3 = (int64_t)Mt * Mt * Mt;
    const int s = blockIdx.x;
    const int j0 = tile_start[s], j1 = tile_start[s + 1];
    if (j0 == j1) return;
    const int tbx = s % nb, tby = (s / nb) % nb, tbz = s / (nb * nb);
    const int lox = tbx * TB, loy = tby * TB, loz = tbz * TB;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const T gk = gauss_coef<T>(g.ahh);
    const T dfac = (T)(-2.0 * g.ahh / g.h);
    const T half = (T)(0.5 * (P - 1));
    const int PP = P * P, P4 = (P + 3) & ~3;
    const int bm0 = MODE == 0 ? blockIdx.y : 0;
    const int bm1 = MODE == 0 ? blockIdx.y + 1 : batch;
    for (int bm = bm0; bm < bm1; ++bm) {
        for (int cs = 0; cs < 3; cs += NCS) {
            __syncthreads();
            for (int q = threadIdx.x; q < NCS * E3S; q += 64 * GW) {
                const int c = NCS == 1 ? 0 : small_div(q, E3S);
                const int r = q - c * E3S;
                T v = (T)0;
                if (r < E3) {
                    const int z = small_div(r, E2), rem = r - z * E2;
                    const int y = small_div(rem, E), x = rem - y * E;
                    const int gx = lox + x, gy = loy + y, gz = loz + z;
                    if (gx < Mt && gy < Mt && gz < Mt)
                        v = field[((int64_t)bm * 3 + cs + c) * M3 + ((int64_t)gz * Mt + gy) * Mt + gx];
                }
                sm[q] = v;
            }
            __syncthreads();
            for (int j = j0 + wid; j < j1; j += GW) {
                const int bp = bpack_s[j];
                const int lbx = (bp & 1023) - lox, lby = ((bp >> 10) & 1023) - loy, lbz = (bp >> 20) - loz;
                {
                    // 1-D weights: lanes 0-31 x, lanes 32-63 y, then lanes 0-31 z
                    const int d = lane >> 5, i = lane & 31;
                    const T c0 = coff_s[3 * (int64_t)j + d];
                    const T e = c0 + (half - (T)i);
                    const T w = i < P ? gauss<T>(gk * e * e) : (T)0;
                    s_w[wid][d][i] = w;
                    s_w[wid][3 + d][i] = dfac * e * w;
                    if (d == 0) {
                        const T ez = coff_s[3 * (int64_t)j + 2] + (half - (T)i);
                        const T wz = i < P ? gauss<T>(gk * ez * ez) : (T)0;
                        s_w[wid][2][i] = wz;
                        s_w[wid][5][i] = dfac * ez * wz;
                    }
                }
                wave_lds_sync();
                T pv[NCS];
#pragma unroll
                for (int c = 0; c < NCS; ++c) pv[c] = MODE != 0 ? vec_s[((int64_t)bm * n + j) * 3 + cs + c] : (T)0;
                T v[NCS];
#pragma unroll
                for (int c = 0; c < NCS; ++c) v[c] = (T)0;
                T g0 = 0, g1 = 0, g2 = 0;
                const T* wxr = s_w[wid][0];
                const T* dwxr = s_w[wid][3];
                for (int r = lane; r < PP; r += 64) {
                    const int iz = small_div(r, P), iy = r - iz * P;
                    const T* row = sm + ((lbz + iz) * E + lby + iy) * E + lbx;
                    T S[NCS], D[NCS];
#pragma unroll
                    for (int c = 0; c < NCS; ++c) S[c] = D[c] = (T)0;
                    for (int ix = 0; ix < P4; ix += 4) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const T wxu = wxr[ix + u];
                            const T dwxu = MODE != 0 ? dwxr[ix + u] : (T)0;
#pragma unroll
                            for (int c = 0; c < NCS; ++c) {
                                const T a = row[c * E3S + ix + u];
                                S[c] += wxu * a;
                                if (MODE != 0) D[c] += dwxu * a;
                            }
                        }
                    }
                    const T wy = s_w[wid][1][iy], wz = s_w[wid][2][iz];
                    if (MODE != 1) {
                        const T wyz = wy * wz;
#pragma unroll
                        for (int c = 0; c < NCS; ++c) v[c] += wyz * S[c];
                    }
                    if (MODE != 0) {
                        T Sp = 0, Dp = 0;
#pragma unroll
                        for (int c = 0; c < NCS; ++c) {
                            Sp += pv[c] * S[c];
                            Dp += pv[c] * D[c];
                        }
                        const T dwy = s_w[wid][4][iy], dwz = s_w[wid][5][iz];
                        g0 += wy * wz * Dp;
                        g1 += dwy * wz * Sp;
                        g2 += wy * dwz * Sp;
                    }
                }
                const int64_t i = perm_s[j];
                if (MODE != 1) {
#pragma unroll
                    for (int c = 0; c < NCS; ++c) v[c] = wave_sum(v[c]);
                    if (lane == 0 && out) {
                        T* o = out + ((int64_t)bm * n + i) * 3 + cs;
#pragma unroll
                        for (int c = 0; c < NCS; ++c) o[c] = v[c];
                    }
                }
                if (MODE != 0) {
                    g0 = wave_sum(g0);
                    g1 = wave_sum(g1);
                    g2 = wave_sum(g2);
                    if (lane == 0 && dx) {
                        // the first contribution (forward field, first batch member,
                        // first component pass) overwrites; the same lane adds the rest
                        const bool first = (MODE == 1 && bm == 0 && cs == 0);
                        dx[3 * i] = (first ? (T)0 : dx[3 * i]) + g0;
                        dx[3 * i + 1] = (first ? (T)0 : dx[3 * i + 1]) + g1;
                        dx[3 * i + 2] = (first ? (T)0 : dx[3 * i + 2]) + g2;
                    }
                }
                wave_lds_sync();
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Quadrature sweeping z: one workgroup owns an xy tile of KX x KX bins and a
// run of bins along z.  The field planes the current z-bin's windows touch
// (TB + P - 1 of them, over the (KX TB + P - 1)^2 xy footprint) sit in an LDS
// ring; moving one bin up in z replaces only TB planes, so each plane is read
// from global memory once per sweep instead of once per bin it overlaps.  Per
// point the work is that of the quadrature above (one wave per point, lanes
// over window rows).
// ---------------------------------------------------------------------------
constexpr int CW = 8;  // waves per sweeping workgroup
// FP64 value quadrature with one component per pass: its ring leaves one workgroup
// per CU and a bin step holds about ten points, so it runs 12 waves (one point each)
#ifndef FSE_CW64V
#define FSE_CW64V 12
#endif
constexpr int CW64V = FSE_CW64V;
// Window width the sweeping quadrature sums over: P padded to a multiple of 4 (the
// runtime-width x-sums run in fours), except FP64 P = 17 or 18, which run the
// unrolled width 18 (16-byte groups of two doubles; the FP64 headline's P = 18
// then sums 18 terms per row instead of 20).
template <typename T> __host__ __device__ constexpr int col_p4(int P) {
    return (sizeof(T) == 8 && (P == 17 || P == 18)) ? 18 : (P + 3) & ~3;
}
// Terms of the unrolled x sums: col_p4, except FP32 P = 11 (the FP32 headline's),
// which sums its 11 terms from rows of 12 factors.
template <typename T> __host__ __device__ constexpr int col_pt(int P) {
    return (sizeof(T) == 4 && P == 11) ? 11 : col_p4<T>(P);
}

template <typename T, int MODE, int NCS, int GP, int PT, int NW = CW>
__global__ __launch_bounds__(64 * NW) void k_gather_col(GridGeo g, int KX, int segb, int ES, int PS,
                                                       const int* __restrict__ tile_start,
                                                       const int* __restrict__ perm_s,
                                                       const int* __restrict__ bpack_s,
                                                       const T* __restrict__ coff_s,
                                                       const T* __restrict__ field,
                                                       const T* __restrict__ vec_s, int64_t n, int batch,
                                                       T* out, T* dx) {
    constexpr int GL = 64 / GP;  // lanes per point: a wave works on GP points at once
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* sm = (T*)smem_raw;
    const int Mt = g.Mt, P = g.P, TB = g.TS, nb = g.nt;
    const int X = KX * TB, E = X + P - 1, E2 = E * E, EZ = TB + P - 1;
    // PT > 0: the x sums run over PT terms, unrolled with immediate LDS offsets
    // (P <= PT; the factors beyond P are zero); PT = 0: any P.  The factor rows are
    // P4 long either way.
    const int P4 = PT > 0 ? (sizeof(T) == 8 ? (PT + 1) & ~1 : (PT + 3) & ~3) : col_p4<T>(P);
    // after the ring: per wave and point, the 1-D factors wx, wy, wz, dwx, dwy, dwz
    // (P4 each, zero beyond P)
    // LDS layout: row stride ES >= E and plane stride PS >= E ES, padded so the
    // lanes' rows fall in distinct banks; the padding is zero and absorbs the
    // x-unroll overrun, as do 4 zero elements after each component
    const int CS = EZ * PS + 4;
    const int64_t M3 = (int64_t)Mt * Mt * Mt;
    const int ncx = (nb + KX - 1) / KX;
    // work item: column (x fastest) then z-segment; surplus items return
    const int nwork = ncx * ncx * ((nb + segb - 1) / segb);
    // work items in XCD-grouped order in FP64: each run of 32 block ids puts four
    // neighbouring columns (which stage largely the same planes) on one XCD's L2
    // (FP64 value and gradient passes 2.4 % faster; FP32 1-3 % slower, so it keeps
    // the plain order)
    int w = (int)blockIdx.x;
    if constexpr (sizeof(T) == 8) {
        constexpr int G = 4;
        if (w < (int)gridDim.x / (8 * G) * (8 * G)) {
            const int o = w % (8 * G);
            w = w - o + (o % 8) * G + o / 8;
        }
    }
    if (w >= nwork) return;
    const int col = w % (ncx * ncx), seg = w / (ncx * ncx);
    const int cx = col % ncx, cy = col / ncx;
    const int lox = cx * X, loy = cy * X;
    const int tz0 = seg * segb, tz1 = min(nb, tz0 + segb);
    if (tz0 >= tz1) return;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const T gk = gauss_coef<T>(g.ahh);
    const T dfac = (T)(-2.0 * g.ahh / g.h);
    const T half = (T)(0.5 * (P - 1));
    const int PP = P * P;
    const int grp = GP == 1 ? 0 : lane / GL, gl = GP == 1 ? lane : lane % GL;
    // row advance by GL: (dq, dr) = divmod(GL, P), and the matching ring offsets
    const int dq = GL / P, dr = GL - dq * P;
    const int step_r = dq * PS + dr * ES, step_c = PS - P * ES;
    // this group's factors, 16-byte aligned (the ring is rounded up to 4 elements
    // and P4 is a multiple of 4) so the x-factors load as 128-bit broadcasts
    T* const s_w = (T*)__builtin_assume_aligned(sm + ((NCS * CS + 3) & ~3) + (wid * GP + grp) * 6 * P4, 16);
    const int bm0 = MODE == 0 ? blockIdx.y : 0;
    const int bm1 = MODE == 0 ? blockIdx.y + 1 : batch;
    const int bx0 = cx * KX, bx1 = min(nb, bx0 + KX) - 1;
    const int by0 = cy * KX, by1 = min(nb, by0 + KX) - 1;
    // stage planes [z1, z1 + npl) of the current field into their ring slots: a
    // thread owns (component, y, x) columns of the footprint, located once, and
    // walks the planes with a pointer that advances one plane per load, eight
    // loads in flight; planes beyond the grid (from nv on) and nodes outside it
    // stage zeros (the node's address is clamped into the field, its value dropped)
    auto stage_planes = [&](const T* fb, int z1, int npl) {
        const int s1 = z1 % EZ;
        const int nv = min(npl, Mt - z1);
        const int64_t MM = (int64_t)Mt * Mt;
        for (int q = tid; q < NCS * E2; q += 64 * NW) {
            const int c = NCS == 1 ? 0 : small_div(q, E2);
            const int t = q - c * E2;
            const int y = small_div(t, E), x = t - y * E;
            const int gx = lox + x, gy = loy + y;
            const bool in = gx < Mt && gy < Mt;
            const T* src = fb + (int64_t)c * M3 + (int64_t)min(gy, Mt - 1) * Mt + min(gx, Mt - 1);
            T* dst = sm + c * CS + y * ES + x;
            for (int k0 = 0; k0 < npl; k0 += 8) {
                T v[8];
                const T* pz = src + (int64_t)(z1 + k0) * MM;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    v[b] = k0 + b < nv ? *pz : (T)0;
                    pz += MM;
                }
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    if (k0 + b < npl) {
                        // ring slot of plane z1 + k0 + b: s1 < EZ and k0 + b < npl <= EZ
                        const int sl = s1 + k0 + b;
                        dst[(sl >= EZ ? sl - EZ : sl) * PS] = in ? v[b] : (T)0;
                    }
                }
            }
        }
    };
    for (int q = tid; q < NCS * CS; q += 64 * NW) sm[q] = (T)0;
    for (int bm = bm0; bm < bm1; ++bm) {
        for (int cs = 0; cs < 3; cs += NCS) {
            const T* fb = field + ((int64_t)bm * 3 + cs) * M3;
            // initial ring: planes [tz0 TB, tz0 TB + EZ)
            __syncthreads();
            stage_planes(fb, tz0 * TB, EZ);
            __syncthreads();
            for (int tz = tz0; tz < tz1; ++tz) {
                const int z0 = tz * TB;
                if (tz > tz0) {
                    // planes [z0 - TB + EZ, z0 + EZ) replace [z0 - TB, z0) in the ring
                    __syncthreads();
                    stage_planes(fb, z0 - TB + EZ, TB);
                    __syncthreads();
                }
                // the points of the z-bin tz in this tile (one contiguous range per bin row)
                for (int by = by0; by <= by1; ++by) {
                    const int rowb = (tz * nb + by) * nb;
                    const int j0 = tile_start[rowb + bx0], j1 = tile_start[rowb + bx1 + 1];
                    for (int jb = j0 + wid * GP; jb < j1; jb += NW * GP) {
                        const int j = jb + grp;
                        const bool valid = j < j1;
                        const int bp = valid ? bpack_s[j] : 0;
                        const int lbx = (bp & 1023) - lox, lby = ((bp >> 10) & 1023) - loy, bz = bp >> 20;
                        // 1-D factors of this group's point: entries q = d P4 + i, d = x, y, z
                        T cxyz[3] = {(T)0, (T)0, (T)0};
                        if (valid) {
#pragma unroll
                            for (int d = 0; d < 3; ++d) cxyz[d] = coff_s[3 * (int64_t)j + d];
                        }
                        for (int q = gl; q < 3 * P4; q += GL) {
                            const int d = small_div(q, P4), i = q - d * P4;
                            const T c0 = d == 0 ? cxyz[0] : (d == 1 ? cxyz[1] : cxyz[2]);
                            const T e = c0 + (half - (T)i);
                            const T w = (valid && i < P) ? gauss<T>(gk * e * e) : (T)0;
                            s_w[d * P4 + i] = w;
                            s_w[(3 + d) * P4 + i] = dfac * e * w;
                        }
                        wave_lds_sync();
                        T pv[NCS];
#pragma unroll
                        for (int c = 0; c < NCS; ++c)
                            pv[c] = (MODE != 0 && valid) ? vec_s[((int64_t)bm * n + j) * 3 + cs + c] : (T)0;
                        T v[NCS];
#pragma unroll
                        for (int c = 0; c < NCS; ++c) v[c] = (T)0;
                        T g0 = 0, g1 = 0, g2 = 0;
                        const T* wxr = s_w;
                        const T* dwxr = s_w + 3 * P4;
                        const int rows = valid ? PP : 0;
                        // the lane's rows r = gl, gl + GL, ...: (iz, iy) = divmod(r, P) and
                        // the ring offset advance incrementally, (iz, iy) by divmod(GL, P)
                        int iz = small_div(gl, P), iy = gl - iz * P;
                        int slot = bz + iz;
                        slot -= small_div(slot, EZ) * EZ;
                        int ro = slot * PS + (lby + iy) * ES + lbx;
                        for (int r = gl; r < rows; r += GL) {
                            const T* row = sm + ro;
                            T S[NCS], D[NCS];
#pragma unroll
                            for (int c = 0; c < NCS; ++c) S[c] = D[c] = (T)0;
                            // mode 1 needs only p . F: contract the components first, then
                            // one x-sum each for the value and the x-derivative
                            T Sp1 = (T)0, Dp1 = (T)0;
                            if constexpr (PT > 0 && MODE == 1) {
#pragma unroll
                                for (int ix = 0; ix < PT; ++ix) {
                                    T ap = pv[0] * row[ix];
#pragma unroll
                                    for (int c = 1; c < NCS; ++c) ap += pv[c] * row[c * CS + ix];
                                    Sp1 += wxr[ix] * ap;
                                    Dp1 += dwxr[ix] * ap;
                                }
                            } else if constexpr (PT > 0) {
#pragma unroll
                                for (int ix = 0; ix < PT; ++ix) {
                                    const T wxu = wxr[ix];
                                    const T dwxu = MODE != 0 ? dwxr[ix] : (T)0;
#pragma unroll
                                    for (int c = 0; c < NCS; ++c) {
                                        const T a = row[c * CS + ix];
                                        S[c] += wxu * a;
                                        if (MODE != 0) D[c] += dwxu * a;
                                    }
                                }
                            } else {
                                for (int ix = 0; ix < P4; ix += 4) {
#pragma unroll
                                    for (int u = 0; u < 4; ++u) {
                                        const T wxu = wxr[ix + u];
                                        const T dwxu = MODE != 0 ? dwxr[ix + u] : (T)0;
#pragma unroll
                                        for (int c = 0; c < NCS; ++c) {
                                            const T a = row[c * CS + ix + u];
                                            S[c] += wxu * a;
                                            if (MODE != 0) D[c] += dwxu * a;
                                        }
                                    }
                                }
                            }
                            const T wy = s_w[P4 + iy], wz = s_w[2 * P4 + iz];
                            if (MODE != 1) {
                                const T wyz = wy * wz;
#pragma unroll
                                for (int c = 0; c < NCS; ++c) v[c] += wyz * S[c];
                            }
                            if (MODE != 0) {
                                T Sp = Sp1, Dp = Dp1;
                                if (!(PT > 0 && MODE == 1)) {
#pragma unroll
                                    for (int c = 0; c < NCS; ++c) {
                                        Sp += pv[c] * S[c];
                                        Dp += pv[c] * D[c];
                                    }
                                }
                                const T dwy = s_w[4 * P4 + iy], dwz = s_w[5 * P4 + iz];
                                g0 += wy * wz * Dp;
                                g1 += dwy * wz * Sp;
                                g2 += wy * dwz * Sp;
                            }
                            iy += dr;
                            iz += dq;
                            slot += dq;
                            ro += step_r;
                            if (iy >= P) {
                                iy -= P;
                                ++iz;
                                ++slot;
                                ro += step_c;
                            }
                            while (slot >= EZ) {
                                slot -= EZ;
                                ro -= EZ * PS;
                            }
                        }
                        const int64_t i = valid ? perm_s[j] : 0;
                        if (MODE != 1) {
#pragma unroll
                            for (int c = 0; c < NCS; ++c) v[c] = group_sum<GL>(v[c]);
                            if (gl == 0 && valid && out) {
                                T* o = out + ((int64_t)bm * n + i) * 3 + cs;
#pragma unroll
                                for (int c = 0; c < NCS; ++c) o[c] = v[c];
                            }
                        }
                        if (MODE != 0) {
                            g0 = group_sum<GL>(g0);
                            g1 = group_sum<GL>(g1);
                            g2 = group_sum<GL>(g2);
                            if (gl == 0 && valid && dx) {
                                // the first contribution (forward field, first batch member,
                                // first component pass) overwrites; the same lane adds the rest
                                const bool first = ((MODE == 1 || MODE == 3) && bm == 0 && cs == 0);
                                dx[3 * i] = (first ? (T)0 : dx[3 * i]) + g0;
                                dx[3 * i + 1] = (first ? (T)0 : dx[3 * i + 1]) + g1;
                                dx[3 * i + 2] = (first ? (T)0 : dx[3 * i + 2]) + g2;
                            }
                        }
                        wave_lds_sync();
                    }
                }
            }
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
    const T gk = gauss_coef<T>(g.ahh);
    const T half = (T)(0.5 * (P - 1));
    const T* fb0 = field + (int64_t)bm * 3 * M3;
    for (int j = j0 + wid; j < j1; j += 4) {
        const int bp = bpack_s[j];
        const int bx = bp & 1023, by = (bp >> 10) & 1023, bz = bp >> 20;
        const T cx = coff_s[3 * (int64_t)j], cy = coff_s[3 * (int64_t)j + 1], cz = coff_s[3 * (int64_t)j + 2];
        const T ex = cx + (half - (T)gx);
        const T wx = (gx < P) ? gauss<T>(gk * ex * ex) : (T)0;
        if (lane < P) {
            const T ey = cy + (half - (T)lane), ez = cz + (half - (T)lane);
            wsh[wid][0][lane] = gauss<T>(gk * ey * ey);
            wsh[wid][1][lane] = gauss<T>(gk * ez * ez);
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
    const T gk = gauss_coef<T>(g.ahh);
    const T dfac = (T)(-2.0 * g.ahh / g.h);
    const T half = (T)(0.5 * (P - 1));
    for (int j = j0 + wid; j < j1; j += 4) {
        const int bp = bpack_s[j];
        const int bx = bp & 1023, by = (bp >> 10) & 1023, bz = bp >> 20;
        const T cx = coff_s[3 * (int64_t)j], cy = coff_s[3 * (int64_t)j + 1], cz = coff_s[3 * (int64_t)j + 2];
        const T ex = cx + (half - (T)gx);
        const T wx = (gx < P) ? gauss<T>(gk * ex * ex) : (T)0;
        const T dwx = dfac * ex * wx;
        if (lane < P) {
            const T ey = cy + (half - (T)lane), ez = cz + (half - (T)lane);
            const T wy = gauss<T>(gk * ey * ey), wz = gauss<T>(gk * ez * ez);
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

// Components staged per pass (3 or 1) of the LDS quadrature and its dynamic
// LDS bytes, or 0 if even one component's block does not fit.
template <typename T> int gather_ncs(const GridGeo& g, size_t* bytes) {
    const size_t E = (size_t)g.TS + g.P - 1;
    const size_t comp = (E * E * E + 4) * sizeof(T);
    const size_t limit = 160 * 1024 - GW * 6 * 32 * sizeof(T);
    if (3 * comp <= limit) { *bytes = 3 * comp; return 3; }
    if (comp <= limit) { *bytes = comp; return 1; }
    *bytes = 0;
    return 0;
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
                   T* grid, hipStream_t st, const T* src2, T* grid2) {
    // cores of 16 x 16 x TZ nodes: TZ = 16 (FP32) or 8 (FP64) register accumulators per component
    constexpr int TZ = sizeof(T) == 4 ? 16 : 8;
    const unsigned ncxy = (unsigned)((g.Mt + 15) / 16), ncz = (unsigned)((g.Mt + TZ - 1) / TZ);
    dim3 grd(ncxy * ncxy * ncz, batch);
#define SPREAD(NC, CHK)                                                                                      \
    hipLaunchKernelGGL((k_spread<T, NC, TZ, CHK>), grd, dim3(256), 0, st, g, p.tile_start, p.bpack_s,     \
                       p.coff_s, src_s, p.n, grid, src2, grid2)
#define SPREAD_MFMA(NC, CHK)                                                                                 \
    hipLaunchKernelGGL((k_spread_mfma<NC, CHK>), grd, dim3(256), 0, st, g, p.tile_start, p.bpack_s, p.coff_s, \
                       src_s, p.n, grid, src2, grid2)
    if constexpr (sizeof(T) == 4) {
        // six components stage 160 points per chunk: more work per barrier for the same
        // four waves per SIMD (f and w of the headline 1.41 -> 1.35 ms; 192 and 224
        // leave LDS for fewer workgroups and took 1.63 ms)
        if (c_in == 3) SPREAD_MFMA(3, 128); else SPREAD_MFMA(6, 160);
    } else {
        if (c_in == 3) SPREAD(3, 128); else SPREAD(6, 128);
    }
#undef SPREAD_MFMA
#undef SPREAD
}

// Sweeping-quadrature configuration: components per pass, tile side in bins,
// z-bins per workgroup and dynamic LDS bytes; ncs = 0 when it does not fit.
struct ColCfg {
    int ncs, kx, segb, nseg, ncol, es, ps;
    size_t lds;
};

// Worst LDS bank multiplicity of one quadrature read (64 lanes on window rows
// r = l + 64 k, iy = r mod P, iz = r / P) for row stride es and plane stride ps
// (elements of elem_bytes), summed over the passes, for 32 and 64 banks.
static int bank_cost(int P, int es, int ps, int elem_bytes) {
    const int wpe = elem_bytes / 4;
    int tot = 0;
    for (int nbk : {32, 64})
        for (int base = 0; base < P * P; base += 64) {
            int cnt[64] = {0};
            int worst = 0;
            for (int r = base; r < base + 64 && r < P * P; ++r) {
                const int a = ((r / P) * ps + (r % P) * es) * wpe;
                for (int w = 0; w < wpe; ++w) worst = std::max(worst, ++cnt[(a + w) % nbk]);
            }
            tot += worst;
        }
    return tot;
}

// points per wave of the sweeping quadrature: 4 in FP32 (16 lanes each), 1 in
// FP64 (whose field ring leaves no LDS for four points' factors)
template <typename T> constexpr int col_gp() { return sizeof(T) == 4 ? 4 : 1; }

template <typename T> ColCfg col_config(const GridGeo& g, int waves = CW) {
    ColCfg best{0, 0, 0, 0, 0, 0, 0, 0};
    const size_t wbytes = (size_t)waves * col_gp<T>() * 6 * col_p4<T>(g.P) * sizeof(T);
    const size_t limit = 160 * 1024 - wbytes;
    // all components per pass when they fit; one-bin tiles measured as fast as
    // two-bin ones (less LDS, two workgroups per CU)
    const int opts[3][2] = {{3, 1}, {1, 2}, {1, 1}};
    for (auto& o : opts) {
        const int ncs = o[0], kx = o[1];
        const int E = kx * g.TS + g.P - 1, EZ = g.TS + g.P - 1;
        // padded strides with the fewest modelled bank conflicts that keep as
        // many workgroups per CU as the unpadded layout
        const size_t stat = wbytes;
        const size_t lds0 = ncs * ((size_t)EZ * E * E + 4) * sizeof(T);
        if (lds0 > limit) continue;
        const size_t per_cu0 = (160 * 1024) / (lds0 + stat);
        const size_t budget = std::min(limit, (160 * 1024) / per_cu0 - stat);
        int es = E, ps = E * E, cost = 1 << 30;
        for (int e2 = E; e2 <= E + 3; ++e2)
            for (int pad = 0; pad < 64; ++pad) {
                const int p2 = e2 * E + pad;
                if ((size_t)ncs * ((size_t)EZ * p2 + 4) * sizeof(T) > budget) break;
                const int c = bank_cost(g.P, e2, p2, (int)sizeof(T)) * 256 + (e2 - E) * E + pad;
                if (c < cost) { cost = c; es = e2; ps = p2; }
            }
        const size_t ring = ((ncs * ((size_t)EZ * ps + 4) + 3) & ~(size_t)3) * sizeof(T);
        if (ring > limit) continue;
        const size_t lds = ring + wbytes;  // dynamic: the ring, then the factors
        const int ncx = (g.nt + kx - 1) / kx;
        const int per_cu = (int)((160 * 1024) / lds);
        const int target = 2 * 256 * (per_cu < 1 ? 1 : per_cu);
        int nseg = (target + ncx * ncx - 1) / (ncx * ncx);
        nseg = nseg < 1 ? 1 : (nseg > g.nt ? g.nt : nseg);
        const int segb = (g.nt + nseg - 1) / nseg;
        best = ColCfg{ncs, kx, segb, (g.nt + segb - 1) / segb, ncx * ncx, es, ps, lds};
        break;
    }
    return best;
}

template <typename T>
void launch_gather(const GridGeo& g, const PointsDev<T>& p, const T* field, int batch, T* u,
                   hipStream_t st) {
    ColCfg cc = col_config<T>(g);
    bool wide = false;  // CW64V waves (FP64, one component per pass)
    if (sizeof(T) == 8 && cc.ncs == 1) {
        const ColCfg cw = col_config<T>(g, CW64V);
        if (cw.ncs == 1) { cc = cw; wide = true; }
    }
    if (cc.ncs) {
        const dim3 grd(cc.ncol * cc.nseg, batch);
#define GCOL(NC, PT, NWV)                                                                                      \
    allow_lds(k_gather_col<T, 0, NC, col_gp<T>(), PT, NWV>, cc.lds);                                           \
    hipLaunchKernelGGL((k_gather_col<T, 0, NC, col_gp<T>(), PT, NWV>), grd, dim3(64 * NWV), cc.lds, st, g,     \
                       cc.kx, cc.segb, cc.es, cc.ps, p.tile_start, p.perm_s, p.bpack_s, p.coff_s, field,       \
                       (const T*)nullptr, p.n, batch, u, (T*)nullptr)
#define GCOLP(NC, NWV)                                                                                         \
    switch (col_pt<T>(g.P)) {                                                                                  \
        case 11: if constexpr (sizeof(T) == 4) { GCOL(NC, 11, NWV); } break;                                   \
        case 12: GCOL(NC, 12, NWV); break;                                                                     \
        case 16: GCOL(NC, 16, NWV); break;                                                                     \
        case 18: if constexpr (sizeof(T) == 8) { GCOL(NC, 18, NWV); } break;                                   \
        case 20: GCOL(NC, 20, NWV); break;                                                                     \
        default: GCOL(NC, 0, NWV); break;                                                                      \
    }
        if (cc.ncs == 3) {
            GCOLP(3, CW);
        } else if (wide) {
            GCOLP(1, CW64V);
        } else {
            GCOLP(1, CW);
        }
#undef GCOLP
#undef GCOL
        return;
    }
    size_t lds = 0;
    const int ncs = gather_ncs<T>(g, &lds);
    if (ncs) {
        const dim3 grd(nbins(g), batch);
        if (ncs == 3) {
            allow_lds(k_gather_lds<T, 0, 3>, lds);
            hipLaunchKernelGGL((k_gather_lds<T, 0, 3>), grd, dim3(64 * GW), lds, st, g, p.tile_start, p.perm_s,
                               p.bpack_s, p.coff_s, field, (const T*)nullptr, p.n, batch, u, (T*)nullptr);
        } else {
            allow_lds(k_gather_lds<T, 0, 1>, lds);
            hipLaunchKernelGGL((k_gather_lds<T, 0, 1>), grd, dim3(64 * GW), lds, st, g, p.tile_start, p.perm_s,
                               p.bpack_s, p.coff_s, field, (const T*)nullptr, p.n, batch, u, (T*)nullptr);
        }
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
    if (!dx) {
        if (dsrc) launch_gather<T>(g, p, phi_w, batch, dsrc, st);
        return;
    }
    const ColCfg cc = col_config<T>(g);
    if (cc.ncs) {
        const dim3 grd(cc.ncol * cc.nseg, 1);
        // pass 1: forward field contracted with w; pass 2: phi_w value and contraction with f
#define GCOLG(NC, PT)                                                                                          \
    allow_lds(k_gather_col<T, 1, NC, col_gp<T>(), PT>, cc.lds);                                                \
    allow_lds(k_gather_col<T, 2, NC, col_gp<T>(), PT>, cc.lds);                                                \
    hipLaunchKernelGGL((k_gather_col<T, 1, NC, col_gp<T>(), PT>), grd, dim3(64 * CW), cc.lds, st, g, cc.kx,    \
                       cc.segb, cc.es, cc.ps, p.tile_start, p.perm_s, p.bpack_s, p.coff_s, phi_f, w_s, p.n,    \
                       batch, (T*)nullptr, dx);                                                                \
    hipLaunchKernelGGL((k_gather_col<T, 2, NC, col_gp<T>(), PT>), grd, dim3(64 * CW), cc.lds, st, g, cc.kx,    \
                       cc.segb, cc.es, cc.ps, p.tile_start, p.perm_s, p.bpack_s, p.coff_s, phi_w, f_s, p.n,    \
                       batch, dsrc, dx)
#define GCOLGP(NC)                                                                                             \
    switch (col_pt<T>(g.P)) {                                                                                  \
        case 11: if constexpr (sizeof(T) == 4) { GCOLG(NC, 11); } break;                                       \
        case 12: GCOLG(NC, 12); break;                                                                         \
        case 16: GCOLG(NC, 16); break;                                                                         \
        case 18: if constexpr (sizeof(T) == 8) { GCOLG(NC, 18); } break;                                       \
        case 20: GCOLG(NC, 20); break;                                                                         \
        default: GCOLG(NC, 0); break;                                                                          \
    }
        if (cc.ncs == 3) { GCOLGP(3); } else { GCOLGP(1); }
#undef GCOLGP
#undef GCOLG
        return;
    }
    size_t lds = 0;
    const int ncs = gather_ncs<T>(g, &lds);
    if (ncs) {
        // pass 1: forward field contracted with w; pass 2: phi_w value and contraction with f
#define GGRAD(NC)                                                                                              \
    allow_lds(k_gather_lds<T, 1, NC>, lds);                                                                    \
    allow_lds(k_gather_lds<T, 2, NC>, lds);                                                                    \
    hipLaunchKernelGGL((k_gather_lds<T, 1, NC>), dim3(nbins(g)), dim3(64 * GW), lds, st, g, p.tile_start,      \
                       p.perm_s, p.bpack_s, p.coff_s, phi_f, w_s, p.n, batch, (T*)nullptr, dx);                \
    hipLaunchKernelGGL((k_gather_lds<T, 2, NC>), dim3(nbins(g)), dim3(64 * GW), lds, st, g, p.tile_start,      \
                       p.perm_s, p.bpack_s, p.coff_s, phi_w, f_s, p.n, batch, dsrc, dx)
        if (ncs == 3) { GGRAD(3); } else { GGRAD(1); }
#undef GGRAD
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

// The forward quadrature and both gradient quadratures of the adjoint: u from phi_f
// with the first term of dx (w contracted) in one sweep (mode 3), then dsrc from
// phi_w with the second (f contracted; mode 2).  Without the sweeping kernel (its
// block exceeds LDS) the separate passes run.
template <typename T>
void launch_gather_fused(const GridGeo& g, const PointsDev<T>& p, const T* phi_f, const T* phi_w, const T* f_s,
                         const T* w_s, int batch, T* u, T* dsrc, T* dx, hipStream_t st) {
    const ColCfg cc = col_config<T>(g);
    if (!cc.ncs) {
        launch_gather<T>(g, p, phi_f, batch, u, st);
        launch_gather_grad<T>(g, p, phi_f, phi_w, f_s, w_s, batch, dsrc, dx, st);
        return;
    }
    const dim3 grd(cc.ncol * cc.nseg, 1);
#define GFK(MD, NC, PT, FLD, VEC, OUT)                                                                         \
    allow_lds(k_gather_col<T, MD, NC, col_gp<T>(), PT>, cc.lds);                                               \
    hipLaunchKernelGGL((k_gather_col<T, MD, NC, col_gp<T>(), PT>), grd, dim3(64 * CW), cc.lds, st, g, cc.kx,   \
                       cc.segb, cc.es, cc.ps, p.tile_start, p.perm_s, p.bpack_s, p.coff_s, FLD, VEC, p.n,      \
                       batch, OUT, dx)
#define GF(NC, PT)                                                                                             \
    GFK(3, NC, PT, phi_f, w_s, u);                                                                             \
    GFK(2, NC, PT, phi_w, f_s, dsrc)
#define GFP(NC)                                                                                                \
    switch (col_pt<T>(g.P)) {                                                                                  \
        case 11: if constexpr (sizeof(T) == 4) { GF(NC, 11); } break;                                          \
        case 12: GF(NC, 12); break;                                                                            \
        case 16: GF(NC, 16); break;                                                                            \
        case 18: if constexpr (sizeof(T) == 8) { GF(NC, 18); } break;                                          \
        case 20: GF(NC, 20); break;                                                                            \
        default: GF(NC, 0); break;                                                                             \
    }
    if (cc.ncs == 3) { GFP(3); } else { GFP(1); }
#undef GFP
#undef GF
#undef GFK
}

// Default bin side for the point binning: the largest side <= 7 whose quadrature
// block still fits in LDS for one component, at least 2.  At 1e-6 (FP32, P = 12) and
// 1e-10 (FP64, P = 20) settings of the headline workload, sides 4 to 8 (FP32) and 4 to 7 (FP64)
// measured fastest at 7: larger bins stage fewer ring planes per point, and at
// 8 the FP32 ring leaves room for one workgroup per CU instead of two.  A plan's
// tuning may set another side (the autotuned FP64 headline at P = 18 takes 6).
#ifndef FSE_TBMAX32
#define FSE_TBMAX32 7
#endif
#ifndef FSE_TBMAX64
#define FSE_TBMAX64 7
#endif
int bin_side(int elem_bytes, int P) {
    const int tb_max = elem_bytes == 4 ? FSE_TBMAX32 : FSE_TBMAX64;
    const size_t limit = 160 * 1024 - GW * 6 * 32 * (size_t)elem_bytes;
    for (int tb = tb_max; tb >= 2; --tb) {
        const size_t E = (size_t)tb + P - 1;
        if ((E * E * E + 4) * elem_bytes <= limit) return tb;
    }
    return tb_max;  // too large for LDS: the quadrature reads global memory
}

#define INST(T)                                                                                      \
    template void launch_spread<T>(const GridGeo&, const PointsDev<T>&, const T*, int, int, T*,      \
                                   hipStream_t, const T*, T*);                                       \
    template void launch_gather<T>(const GridGeo&, const PointsDev<T>&, const T*, int, T*,           \
                                   hipStream_t);                                                     \
    template void launch_gather_grad<T>(const GridGeo&, const PointsDev<T>&, const T*, const T*,     \
                                        const T*, const T*, int, T*, T*, hipStream_t);            \
    template void launch_gather_fused<T>(const GridGeo&, const PointsDev<T>&, const T*, const T*,    \
                                         const T*, const T*, int, T*, T*, T*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace fse
