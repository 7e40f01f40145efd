// Binning of the points (integer work): Gaussian-window starts and offsets in
// FP64 (the P^3 windows of the fast Gaussian gridding, Section 5.2), and a
// stable sort by spreading tile and by real-space cell (the cell list of
// Section 6).  The sort is a stable LSD radix sort of (key, point index), so
// within a tile or cell the points keep their input order and every later
// summation order is the same from run to run.
#include <rocprim/device/device_radix_sort.hpp>

#include "fse_common.h"

namespace fse {

namespace {

__global__ void k_fill_i32(int* p, int64_t n, int v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Block-level exclusive scan of 4 items per thread; writes the block total.
constexpr int SCAN_T = 256, SCAN_ITEMS = 4, SCAN_BLOCK = SCAN_T * SCAN_ITEMS;

__global__ __launch_bounds__(SCAN_T) void k_scan_block(const int* in, int* out, int64_t n, int* sums) {
    __shared__ int s[SCAN_T];
    int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int tot = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        tot += v[k];
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread totals
    for (int o = 1; o < SCAN_T; o <<= 1) {
        int t = (threadIdx.x >= o) ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int run = s[threadIdx.x] - tot;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == SCAN_T - 1 && sums) sums[blockIdx.x] = s[SCAN_T - 1];
}

__global__ void k_scan_add(int* out, int64_t n, const int* offs) {
    int64_t i = (int64_t)blockIdx.x * SCAN_BLOCK + threadIdx.x;
    int add = offs[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k, i += SCAN_T)
        if (i < n) out[i] += add;
}

template <typename T>
__global__ void k_bin(const T* __restrict__ x, int64_t n, GridGeo g, CellGeo c, int* key_s, int* key_r,
                      int* idx, int* bpack, T* coff, int* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b[3], cl[3];
    bool bad = false;
    for (int d = 0; d < 3; ++d) {
        double v = (double)x[3 * i + d];
        if (!(v >= c.lo[d] && v < c.lo[d] + c.L)) bad = true;  // also catches NaN
        // continuous grid coordinate and window start, FP64
        double t = (v - g.x0[d]) / g.h;
        double bb = floor(t - 0.5 * g.P + 1.0);
        if (!(bb >= 0.0)) bb = 0.0;
        if (!(bb <= (double)(g.Mt - g.P))) bb = (double)(g.Mt - g.P);
        b[d] = (int)bb;
        coff[3 * i + d] = (T)(t - bb - 0.5 * (g.P - 1));
        double cc = floor((v - c.lo[d]) / c.cell);
        if (!(cc >= 0.0)) cc = 0.0;
        if (!(cc <= (double)(c.ncell - 1))) cc = (double)(c.ncell - 1);
        cl[d] = (int)cc;
    }
    bpack[i] = b[0] | (b[1] << 10) | (b[2] << 20);
    int ks = ((b[2] / g.TS) * g.nt + b[1] / g.TS) * g.nt + b[0] / g.TS;
    int kr = (cl[2] * c.ncell + cl[1]) * c.ncell + cl[0];
    key_s[i] = ks;
    key_r[i] = kr;
    idx[i] = (int)i;
    if (bad) atomicOr(flag, 1);
}

// Counts per key from the sorted keys: the thread at the start of each run of equal
// keys finds the run's end by binary search and writes its length (cnt holds
// zeros beforehand; keys without points keep them).  Counting from the sorted
// keys spares the per-point atomics on a few hundred hot cache lines.
__global__ void k_run_counts(const int* __restrict__ keys, int64_t n, int* cnt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int k = keys[j];
    if (j > 0 && keys[j - 1] == k) return;
    int64_t lo = j + 1, hi = n;  // the first index in [j + 1, n] whose key exceeds k
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] > k) hi = mid; else lo = mid + 1;
    }
    cnt[k] = (int)(lo - j);
}

// Gather the per-point data into the two sorted orders (perm_s and perm_r hold
// the point index at each sorted position).
template <typename T>
__global__ void k_scatter(const T* __restrict__ x, int64_t n, const int* __restrict__ perm_s,
                          const int* __restrict__ perm_r, const int* __restrict__ bpack,
                          const T* __restrict__ coff, int* bpack_s, T* coff_s, T* x_r, int* inv_r) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int is = perm_s[j];
    bpack_s[j] = bpack[is];
    const int ir = perm_r[j];
    inv_r[ir] = (int)j;
    for (int d = 0; d < 3; ++d) {
        coff_s[3 * j + d] = coff[3 * (int64_t)is + d];
        x_r[3 * j + d] = x[3 * (int64_t)ir + d];
    }
}

// Per-point grid components in spread order.  Stokeslet/rotlet: f_l (3).
// Stresslet: the symmetric part of f_lm = n_l q_m in the order
// (00, 11, 22, 01, 02, 12); T_jlm is symmetric in (l, m), so the symmetric
// part carries the whole sum.
template <typename T>
__global__ void k_permute_sources(int kernel, const T* __restrict__ a, const T* __restrict__ b,
                                  int64_t n, int batch, const int* __restrict__ perm, T* out) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bm = blockIdx.y;
    if (j >= n) return;
    int64_t i = perm[j];
    const T* ai = a + ((int64_t)bm * n + i) * 3;
    if (kernel == FSE_STRESSLET) {
        const T* ni = b + ((int64_t)bm * n + i) * 3;
        T* o = out + ((int64_t)bm * n + j) * 6;
        T q0 = ai[0], q1 = ai[1], q2 = ai[2], n0 = ni[0], n1 = ni[1], n2 = ni[2];
        o[0] = n0 * q0;
        o[1] = n1 * q1;
        o[2] = n2 * q2;
        o[3] = (T)0.5 * (n0 * q1 + n1 * q0);
        o[4] = (T)0.5 * (n0 * q2 + n2 * q0);
        o[5] = (T)0.5 * (n1 * q2 + n2 * q1);
    } else {
        T* o = out + ((int64_t)bm * n + j) * 3;
        o[0] = ai[0];
        o[1] = ai[1];
        o[2] = ai[2];
    }
}

template <typename T>
__global__ void k_permute3(const T* __restrict__ a, int64_t n, const int* __restrict__ perm, T* out) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int bm = blockIdx.y;
    if (j >= n) return;
    int64_t i = perm[j];
    const T* ai = a + ((int64_t)bm * n + i) * 3;
    T* o = out + ((int64_t)bm * n + j) * 3;
    o[0] = ai[0];
    o[1] = ai[1];
    o[2] = ai[2];
}

template <typename T>
__global__ void k_tadj_contract(const T* __restrict__ dg, const T* __restrict__ q, const T* __restrict__ nrm,
                                int64_t n, T* dq, T* dn) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int bm = blockIdx.y;
    if (i >= n) return;
    const T* d0 = dg + ((int64_t)(2 * bm) * n + i) * 3;
    const T* d1 = dg + ((int64_t)(2 * bm + 1) * n + i) * 3;
    const T D[3][3] = {{d0[0], d1[0], d1[1]}, {d1[0], d0[1], d1[2]}, {d1[1], d1[2], d0[2]}};
    const int64_t o = ((int64_t)bm * n + i) * 3;
    const T nv[3] = {nrm[o], nrm[o + 1], nrm[o + 2]}, qv[3] = {q[o], q[o + 1], q[o + 2]};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        dq[o + l] = D[l][0] * nv[0] + D[l][1] * nv[1] + D[l][2] * nv[2];
        dn[o + l] = D[0][l] * qv[0] + D[1][l] * qv[1] + D[2][l] * qv[2];
    }
}

template <typename T>
__global__ void k_fold(const T* __restrict__ ext, int Me, int M, int s, T* grid) {
    const int64_t M3 = (int64_t)M * M * M;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (q >= M3) return;
    const int x = (int)(q % M), y = (int)((q / M) % M), z = (int)(q / ((int64_t)M * M));
    // the extended indices of periodic index j: j + s, and j + s - M or j + s + M when in range
    int ex[3], ey[3], ez[3], nx = 0, ny = 0, nz = 0;
    auto images = [&](int j, int* e, int& k) {
        for (int a = j + s - M; a < Me; a += M)
            if (a >= 0) e[k++] = a;
    };
    images(x, ex, nx);
    images(y, ey, ny);
    images(z, ez, nz);
    const T* src = ext + (int64_t)c * Me * Me * Me;
    T v = (T)0;
    for (int a = 0; a < nz; ++a)
        for (int b = 0; b < ny; ++b)
            for (int d = 0; d < nx; ++d) v += src[((int64_t)ez[a] * Me + ey[b]) * Me + ex[d]];
    grid[(int64_t)c * M3 + q] = v;
}

template <typename T>
__global__ void k_unfold(const T* __restrict__ field, int M, int Me, int s, T* ext) {
    const int64_t E3 = (int64_t)Me * Me * Me;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (q >= E3) return;
    const int x = (int)(q % Me), y = (int)((q / Me) % Me), z = (int)(q / ((int64_t)Me * Me));
    auto wrap = [&](int e) { const int j = e - s; return j < 0 ? j + M : (j >= M ? j - M : j); };
    ext[(int64_t)c * E3 + q] = field[(int64_t)c * M * M * M + ((int64_t)wrap(z) * M + wrap(y)) * M + wrap(x)];
}

// per-cell work items of the real-space pass: ceil(count / S); the extra entry is 0
__global__ void k_cell_slices(int* cnt, int64_t ncells, int S) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncells) cnt[c] = (cnt[c] + S - 1) / S;
    else if (c == ncells) cnt[c] = 0;
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

void launch_fill_i32(int* p, int64_t n, int v, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n, 256)), dim3(256), 0, st, p, n, v);
}

void launch_cell_slices(int* cnt, int64_t ncells, int S, hipStream_t st) {
    hipLaunchKernelGGL(k_cell_slices, dim3(nblk(ncells + 1, 256)), dim3(256), 0, st, cnt, ncells, S);
}

size_t scan_tmp_ints(int64_t n) {
    size_t tot = 0;
    while (n > SCAN_BLOCK) {
        int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
        tot += 2 * (size_t)nb + 2;
        n = nb;
    }
    return tot + 2;
}

// Exclusive scan of n ints; `tmp` holds scan_tmp_ints(n) ints.
void launch_scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t st) {
    if (n <= 0) return;
    int64_t nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(SCAN_T), 0, st, in, out, n, (int*)nullptr);
        return;
    }
    int* sums = tmp;
    int* offs = tmp + nb + 1;
    hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(SCAN_T), 0, st, in, out, n, sums);
    launch_scan_exclusive(sums, offs, nb, offs + nb + 1, st);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(SCAN_T), 0, st, out, n, offs);
}

template <typename T>
void launch_bin(const T* x, int64_t n, const GridGeo& g, const CellGeo& c, int* key_s, int* key_r, int* idx,
                int* bpack, T* coff, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_bin<T>, dim3(nblk(n, 256)), dim3(256), 0, st, x, n, g, c, key_s, key_r, idx, bpack,
                       coff, flag);
}

void launch_run_counts(const int* keys_sorted, int64_t n, int* cnt, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_run_counts, dim3(nblk(n, 256)), dim3(256), 0, st, keys_sorted, n, cnt);
}

int key_bits(int64_t nkeys) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < nkeys) ++b;
    return b;
}

// rocPRIM's onesweep LSD radix sort at every size above one block: by default it
// takes a merge sort up to 2^20 items, five merge levels (ten launches) per sort at
// 10^6 points.  Both are stable, so the permutations are the same.
using SortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                              rocprim::default_config, 0>;

size_t sort_tmp_bytes(int64_t n, int bits) {
    size_t b = 0;
    if (rocprim::radix_sort_pairs<SortConfig>(nullptr, b, (const int*)nullptr, (int*)nullptr, (const int*)nullptr,
                                              (int*)nullptr, (unsigned int)n, 0u, (unsigned int)bits,
                                              (hipStream_t)0) != hipSuccess)
        return 0;
    return b;
}

hipError_t launch_sort_pairs(void* tmp, size_t tmp_bytes, const int* keys, int* keys_out, const int* vals,
                             int* vals_out, int64_t n, int bits, hipStream_t st) {
    size_t b = tmp_bytes;
    return rocprim::radix_sort_pairs<SortConfig>(tmp, b, keys, keys_out, vals, vals_out, (unsigned int)n, 0u,
                                                 (unsigned int)bits, st);
}

template <typename T>
void launch_scatter(const T* x, int64_t n, const int* perm_s, const int* perm_r, const int* bpack, const T* coff,
                    int* bpack_s, T* coff_s, T* x_r, int* inv_r, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter<T>, dim3(nblk(n, 256)), dim3(256), 0, st, x, n, perm_s, perm_r, bpack, coff,
                       bpack_s, coff_s, x_r, inv_r);
}

template <typename T>
void launch_permute_sources(int kernel, const T* a, const T* b, int64_t n, int batch, const int* perm,
                            T* out, hipStream_t st) {
    hipLaunchKernelGGL(k_permute_sources<T>, dim3(nblk(n, 256), batch), dim3(256), 0, st, kernel, a,
                       b, n, batch, perm, out);
}

template <typename T>
void launch_fold(const T* ext, int Me, int M, int s, int ncomp, T* grid, hipStream_t st) {
    const int64_t M3 = (int64_t)M * M * M;
    hipLaunchKernelGGL(k_fold<T>, dim3(nblk(M3, 256), ncomp), dim3(256), 0, st, ext, Me, M, s, grid);
}

template <typename T>
void launch_unfold(const T* field, int M, int Me, int s, int ncomp, T* ext, hipStream_t st) {
    const int64_t E3 = (int64_t)Me * Me * Me;
    hipLaunchKernelGGL(k_unfold<T>, dim3(nblk(E3, 256), ncomp), dim3(256), 0, st, field, M, Me, s, ext);
}

template <typename T>
void launch_tadj_contract(const T* dg, const T* q, const T* nrm, int64_t n, int batch, T* dq, T* dn,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_tadj_contract<T>, dim3(nblk(n, 256), batch), dim3(256), 0, st, dg, q, nrm, n, dq, dn);
}

template <typename T>
void launch_permute3(const T* a, int64_t n, int batch, const int* perm, T* out, hipStream_t st) {
    hipLaunchKernelGGL(k_permute3<T>, dim3(nblk(n, 256), batch), dim3(256), 0, st, a, n, perm, out);
}

#define INST(T)                                                                                     \
    template void launch_bin<T>(const T*, int64_t, const GridGeo&, const CellGeo&, int*, int*, int*, int*, \
                                T*, int*, hipStream_t);                                             \
    template void launch_scatter<T>(const T*, int64_t, const int*, const int*, const int*, const T*,   \
                                    int*, T*, T*, int*, hipStream_t);                               \
    template void launch_permute_sources<T>(int, const T*, const T*, int64_t, int, const int*, T*,  \
                                            hipStream_t);                                           \
    template void launch_permute3<T>(const T*, int64_t, int, const int*, T*, hipStream_t);                 \
    template void launch_tadj_contract<T>(const T*, const T*, const T*, int64_t, int, T*, T*, hipStream_t); \
    template void launch_fold<T>(const T*, int, int, int, int, T*, hipStream_t);                           \
    template void launch_unfold<T>(const T*, int, int, int, int, T*, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace fse
