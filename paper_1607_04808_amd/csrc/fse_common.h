// Internal declarations shared by the HIP translation units of libfse.
// gfx950 (CDNA4): 64-wide wavefronts, 160 KB LDS per workgroup.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fse.h"

namespace fse {

constexpr int WAVE = 64;
// Kernel index of the stresslet's transpose (its adjoint from a 3-vector field to
// the symmetric 2-tensor D_lm), beside FSE_STOKESLET / FSE_STRESSLET / FSE_ROTLET.
constexpr int KTADJ = 3;
// Kernel index of the plain scalar convolution (the free-space solver): each of
// three components multiplied by the scalar transform.
constexpr int KSCALAR = 4;

// ---------------------------------------------------------------------------
// complex helpers (float2 / double2)
// ---------------------------------------------------------------------------
template <typename T> struct cplx;
template <> struct cplx<float> { using type = float2; };
template <> struct cplx<double> { using type = double2; };
template <typename T> using C2 = typename cplx<T>::type;

template <typename V> __device__ __forceinline__ V cmk(decltype(V::x) a, decltype(V::x) b) {
    V v; v.x = a; v.y = b; return v;
}
template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return cmk<V>(a.x + b.x, a.y + b.y); }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return cmk<V>(a.x - b.x, a.y - b.y); }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
    return cmk<V>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename V> __device__ __forceinline__ V cmulc(V a, V b) {
    return cmk<V>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename V> __device__ __forceinline__ V cscale(V a, decltype(V::x) s) { return cmk<V>(a.x * s, a.y * s); }
template <typename V> __device__ __forceinline__ V cconj(V a) { return cmk<V>(a.x, -a.y); }
// multiply by -i (dir=-1) or +i (dir=+1)
template <int DIR, typename V> __device__ __forceinline__ V cmuli(V a) {
    return DIR < 0 ? cmk<V>(a.y, -a.x) : cmk<V>(-a.y, a.x);
}

// ---------------------------------------------------------------------------
// cross-lane helpers
// ---------------------------------------------------------------------------

// floor(a / b) for 0 <= a < 2^21 and b >= 1 via a float reciprocal: (a + 0.5) / b
// lies at least 1/(2b) from the integers on both sides, and the relative error
// of (a + 0.5) * rcp(b) (about 1.5 ulp) keeps it within (a + 0.5) 2^-22.4 / b < 1/(2b).
__device__ __forceinline__ int small_div(int a, int b) {
    return (int)(((float)a + 0.5f) * __builtin_amdgcn_rcpf((float)b));
}

// Copy `total` elements into LDS (or any per-element destination) with B
// independent loads per thread in flight: ld(q) reads element q, st(q, v) stores
// it.  A plain strided loop of load-then-store waits out one memory latency per
// element, since each LDS store needs its load to have returned.
template <int B, typename LD, typename ST>
__device__ __forceinline__ void staged_copy(int total, LD&& ld, ST&& st) {
    const int nthr = blockDim.x;
    for (int q0 = threadIdx.x; q0 < total; q0 += B * nthr) {
        decltype(ld(0)) v[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int q = q0 + b * nthr;
            if (q < total) v[b] = ld(q);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int q = q0 + b * nthr;
            if (q < total) st(q, v[b]);
        }
    }
}

__device__ __forceinline__ float readlane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double readlane(double v, int lane) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Sum over each aligned group of G lanes (G a power of two dividing 64).
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Order this wave's own LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// plan-level constants passed to kernels by value
// ---------------------------------------------------------------------------
struct GridGeo {
    int Mt;          // grid points per side
    int n;           // FFT size 2*Mt
    int P;           // Gaussian support
    int TS;          // spreading/quadrature tile side (grid points)
    int nt;          // tiles per side = ceil(Mt/TS)
    double x0[3];    // first grid node
    double h;        // grid spacing
    double ahh;      // alpha h^2: Gaussian exponent in grid units
};

struct CellGeo {
    int ncell;       // cells per side
    double lo[3];    // box corner
    double L;        // box side
    double cell;     // cell side (>= rc)
    double rc2;      // rc^2
    int periodic;    // 1: the cells wrap with period L (triply periodic sums)
    int qcap;        // real-space hit-queue entries per thread: value pass
    int qcap_grad;   // and gradient pass (>= 16; tuned per plan)
};

constexpr int MAX_RADICES = 12;
struct FftGeo {
    int n;                    // transform length
    int ns;                   // number of radix stages
    int rad[MAX_RADICES];     // radix per stage (DIF order)
    int Ls[MAX_RADICES];      // block length at each stage
    int pair[MAX_RADICES];    // 1: stages s and s+1 run as one register-resident pass
    int sy, sz;               // padded line strides (elements) of the y- and z-lines of the
                              // intermediate spectra, multiples of 128 bytes
    int lines_cap;            // 0, or the most lines (rows) per workgroup of a pass (tuning)
};

// Stage pairs that run fused (both radices' butterflies of one element group
// in registers): the product bounds the registers a thread holds.
__host__ __device__ constexpr bool fft_pair_ok(int r1, int r2, int elem_bytes) {
    return r1 * r2 <= (elem_bytes == 4 ? 32 : 16) &&
           ((r1 == 8 && (r2 == 2 || r2 == 3 || r2 == 4)) || (r1 == 7 && (r2 == 2 || r2 == 3 || r2 == 4)) ||
            (r1 == 5 && (r2 == 2 || r2 == 3 || r2 == 4 || r2 == 5)) || (r1 == 4 && r2 == 3) ||
            (r1 == 2 && r2 == 3) || (r1 == 3 && r2 == 3));
}

// Points binned for one evaluation (device pointers)
template <typename T> struct PointsDev {
    int64_t n;
    const int* perm_s;        // spread order -> user index
    const int* bpack_s;       // packed window start (bx | by<<10 | bz<<20), spread order
    const T* coff_s;          // window-centre offsets (n,3), spread order, in [-0.5,0.5)
    const int* tile_start;    // (nt^3 + 1) offsets into spread order
    const int* perm_r;        // real-space order -> user index
    const T* x_r;             // positions (n,3), real-space order
    const int* cell_start;    // (ncell^3 + 1) offsets into real-space order
    const int* inv_r;         // user index -> real-space order
    const int* work_start;    // (ncell^3 + 1) real-space work items: cell c owns items
                              // [work_start[c], work_start[c+1]), each of up to real_S targets
    int real_S;               // targets per real-space work item (= threads per workgroup)
    // Targets of the real-space pass (the same arrays as above when the targets
    // are the sources): positions in their cell order, cell offsets, cell order
    // -> user index, work items, and their count.
    int64_t t_n;
    const T* t_x_r;
    const int* t_cell_start;
    const int* t_perm_r;
    const int* t_work_start;
    int t_real_S;
};

// thread-local message returned by fse_last_error (printf format)
void set_error(const char* fmt, ...);

// ---------------------------------------------------------------------------
// launchers (one per translation unit); all enqueue on `st`
// ---------------------------------------------------------------------------
void launch_fill_i32(int* p, int64_t n, int v, hipStream_t st);
void launch_scan_exclusive(const int* in, int* out, int64_t n, int* tmp, hipStream_t st);
// cnt[c] <- ceil(cnt[c] / S) for c < ncells, cnt[ncells] <- 0
void launch_cell_slices(int* cnt, int64_t ncells, int S, hipStream_t st);
// threads (= targets) per real-space work item for n points in ncells cells
// (at most max_waves waves, 1..4)
int default_qcap(int elem_bytes, bool grad);
unsigned real_threads(int64_t n, int64_t ncells, int max_waves = 4);
size_t scan_tmp_ints(int64_t n);

// window starts/offsets, tile and cell keys, per-key counts (cnt_s, cnt_r
// accumulate), idx[i] = i, flag |= 1 for a point outside the box
template <typename T>
void launch_bin(const T* x, int64_t n, const GridGeo& g, const CellGeo& c, int* key_s, int* key_r, int* idx,
                int* bpack, T* coff, int* flag, hipStream_t st);
// cnt[k] <- the number of entries equal to k in the ascending keys_sorted[0, n)
// (cnt zero beforehand)
void launch_run_counts(const int* keys_sorted, int64_t n, int* cnt, hipStream_t st);
// bits that hold keys in [0, nkeys)
int key_bits(int64_t nkeys);
// device scratch bytes of one launch_sort_pairs over n keys of `bits` bits (0 on failure)
size_t sort_tmp_bytes(int64_t n, int bits);
// stable radix sort of (keys, vals) by the low `bits` bits of the keys
hipError_t launch_sort_pairs(void* tmp, size_t tmp_bytes, const int* keys, int* keys_out, const int* vals,
                             int* vals_out, int64_t n, int bits, hipStream_t st);
// sorted copies: bpack_s/coff_s in spread order (perm_s), x_r in real-space
// order (perm_r), inv_r = the inverse of perm_r
template <typename T>
void launch_scatter(const T* x, int64_t n, const int* perm_s, const int* perm_r, const int* bpack, const T* coff,
                    int* bpack_s, T* coff_s, T* x_r, int* inv_r, hipStream_t st);

// source permutation to spread order: out (batch, n, c_in) with the per-point
// components the grid carries (f_l, or the symmetric n_l q_m for the stresslet)
template <typename T>
void launch_permute_sources(int kernel, const T* a, const T* b, int64_t n, int batch, const int* perm,
                            T* out, hipStream_t st);
// Contract the quadrature of the stresslet-transpose field with the points' own
// q and n: dg (2 batch, n, 3) holds D = (D00, D11, D22) in row 2b and (D01, D02,
// D12) in row 2b + 1 (user order); dq_l = D_lm n_m, dn_m = D_lm q_l (overwritten).
template <typename T>
void launch_tadj_contract(const T* dg, const T* q, const T* nrm, int64_t n, int batch, T* dq, T* dn,
                          hipStream_t st);
// Periodic grids: the spreading grid extends the M^3 period by P - 1 nodes (P
// for odd P; index e = j + s, s = ceil(P/2) - 1, j the periodic index), so that
// windows never wrap.  fold: grid(j) = sum of ext(e) over the e = j + s (mod M) in range;
// unfold: ext(e) = field((e - s) mod M).  ncomp components of M^3 / Me^3 each.
template <typename T>
void launch_fold(const T* ext, int Me, int M, int s, int ncomp, T* grid, hipStream_t st);
template <typename T>
void launch_unfold(const T* field, int M, int Me, int s, int ncomp, T* ext, hipStream_t st);
// permute plain 3-vectors (batch, n, 3) by perm
template <typename T>
void launch_permute3(const T* a, int64_t n, int batch, const int* perm, T* out, hipStream_t st);

// src2 / grid2 (c_in = 6): two 3-component source sets spread together, the first
// into grid and the second into grid2 (3 components per batch member each)
template <typename T>
void launch_spread(const GridGeo& g, const PointsDev<T>& p, const T* src_s, int c_in, int batch,
                   T* grid, hipStream_t st, const T* src2 = nullptr, T* grid2 = nullptr);
// bin side (grid points) of the point binning for the element size and P
int bin_side(int elem_bytes, int P);
template <typename T>
void launch_gather(const GridGeo& g, const PointsDev<T>& p, const T* field, int batch, T* u,
                   hipStream_t st);
template <typename T>
void launch_gather_grad(const GridGeo& g, const PointsDev<T>& p, const T* phi_f, const T* phi_w,
                        const T* f_s, const T* w_s, int batch, T* dsrc, T* dx, hipStream_t st);
template <typename T>
void launch_gather_fused(const GridGeo& g, const PointsDev<T>& p, const T* phi_f, const T* phi_w,
                         const T* f_s, const T* w_s, int batch, T* u, T* dsrc, T* dx, hipStream_t st);

// Grid sides the FFT passes take: whether every pass fits in LDS at Mt, and the
// largest Mt <= 1024 that does for a kernel (FSE_STRESSLET: six grid components)
bool fft_fits(int kernel, int elem_bytes, int Mt);
int fft_max_mt(int kernel, int elem_bytes);

template <typename T>
void launch_fft_forward(const FftGeo& fg, const GridGeo& g, const T* grid, void* A, void* B,
                        int ncomp, const T* tw, const int* rev, const int* revinv, hipStream_t st,
                        int passes = 3);  // bit 0: x pass, bit 1: y pass
template <typename T>
void launch_fft_zscale(const FftGeo& fg, const GridGeo& g, int kernel, void* B, int c_in, int batch,
                       const T* sig, double kscale, const T* tw, const int* rev, const int* revinv,
                       hipStream_t st);
template <typename T>
void launch_fft_inverse(const FftGeo& fg, const GridGeo& g, void* B, void* A, T* field, int c_in,
                        int batch, const T* tw, const int* rev, const int* revinv, hipStream_t st,
                        int passes = 3);  // bit 0: inverse y pass, bit 1: inverse x pass

template <typename T>
void launch_real(int kernel, const CellGeo& c, const PointsDev<T>& p, const T* src_a_r,
                 const T* src_b_r, int batch, double xi, double self_coef, T* u, int accumulate,
                 hipStream_t st);
template <typename T>
// dx += real-space gradient; when dsrc is given, also dsrc += the real-space
// part of K w (with the self term) in the same pass
void launch_real_grad(int kernel, const CellGeo& c, const PointsDev<T>& p, const T* f_r, const T* w_r,
                      int batch, double xi, double self_coef, T* dx, T* dsrc, hipStream_t st,
                      T* u = nullptr);  // u: with dsrc and batch 1, also u += u^R + self term

// dq += D^R n, dn += D^R q with D^R_lm(t) = sum_s T^R_jlm(x_s - x_t) w_j(s), the
// real-space part of the stresslet adjoint (q_r, n_r, w_r in real-space order)
template <typename T>
void launch_real_tadj(const CellGeo& c, const PointsDev<T>& p, const T* q_r, const T* n_r, const T* w_r,
                      int batch, double xi, T* dq, T* dn, hipStream_t st);

// precompute (FP64)
void launch_pre_fill(double* out, int Mg, double h, double R, int family, hipStream_t st);
void launch_pre_contract(const double* in, double* out, const double* Cm, int J, int K, int64_t A,
                         hipStream_t st);
template <typename T>
void launch_pre_finalize(const double* Bt, int Mt, double kunit, double xi, double eta, int kernel,
                         double norm, double* sig64, T* sig, hipStream_t st);
// periodic stokeslet: the eq. ShatH kernel at the even indices of the (2 Mt)^3 grid
template <typename T>
void launch_pre_periodic(int Mt, double kunit, double xi, double eta, double norm, double* sig64, T* sig,
                         hipStream_t st);

}  // namespace fse
