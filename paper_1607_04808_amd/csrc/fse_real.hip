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
// neighbour cells staged in LDS (three x-adjacent cells are one contiguous
// range in cell order, so each chunk is a coalesced read), hits queued per
// thread and evaluated wave-wide.
#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>

#include "fse_common.h"

namespace fse {

namespace {

constexpr double INV_SQRTPI = 0.56418958354775628695;

// Radial factors of a pair at squared distance r2 > 0:
// r, 1/r, e = exp(-xi^2 r^2) and ec = erfc(xi r), with
// erfc(x) = e t Q(t), t = 1/(1 + p x), Q fitted for small relative error of
// exp(x^2) erfc(x) (the generator and its error report are fit_erfcx.py
// beside this file):
//   FP32: p = 0.4, Q a degree-10 polynomial in t, relative error about 3e-7
//         in FP32 for all x >= 0; hardware rsqrt, exp2 and rcp.
//   FP64: p = 0.5, Q a degree-20 Chebyshev series in s = 2(t - t0)/(1 - t0) - 1,
//         t0 = 1/6 (x <= 10; s is clamped at -1 beyond, where erfc < 1e-44),
//         relative error about 3e-15; the reciprocal of 1 + p x from the
//         hardware estimate and two Newton steps.
template <typename T>
__device__ __forceinline__ void radial(T xi, T xi2, T r2, T& r, T& ir, T& e, T& ec);

__constant__ double ERFC_CHEB64[21] = {
    0.62088859609968661,     0.33031317717291347,     0.048190528012879576,    0.0013007898942622317,
    -0.00067070511569872345, -3.7277111326298097e-05, 1.4963307669145149e-05,  3.0797536323925218e-07,
    -4.1390867160614104e-07, 2.5753677315551033e-08,  9.9127889901883903e-09,  -1.9949429131729499e-09,
    -6.7533070604464365e-11, 7.9914175529419191e-11,  -1.0272660257690479e-11, -1.2644162927243331e-12,
    6.3097653465346595e-13,  -7.0177374122948254e-14, -1.1900996748257948e-14, 5.5584172623120927e-15,
    -6.8688868596316233e-16};

template <>
__device__ __forceinline__ void radial<double>(double xi, double xi2, double r2, double& r, double& ir,
                                               double& e, double& ec) {
    ir = rsqrt(r2);
    r = r2 * ir;
    e = exp(-xi2 * r2);
    const double d = fma(0.5 * xi, r, 1.0);
    double t = __builtin_amdgcn_rcp(d);
    t = fma(t, fma(-d, t, 1.0), t);
    t = fma(t, fma(-d, t, 1.0), t);
    // s = 2 (t - 1/6) / (5/6) - 1 = 2.4 t - 1.4
    const double s = fmax(fma(2.4, t, -1.4), -1.0);
    const double s2 = 2.0 * s;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = 20; k >= 1; --k) {
        const double b0 = fma(s2, b1, ERFC_CHEB64[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    const double q = fma(s, b1, ERFC_CHEB64[0] - b2);
    ec = e * t * q;
}

template <>
__device__ __forceinline__ void radial<float>(float xi, float xi2, float r2, float& r, float& ir, float& e,
                                              float& ec) {
    constexpr float LOG2E = 1.44269504f;
    ir = __builtin_amdgcn_rsqf(r2);
    r = r2 * ir;
    // the factors xi^2 log2(e) and 0.4 xi are loop invariants
    e = __builtin_amdgcn_exp2f((xi2 * -LOG2E) * r2);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.4f * xi, r, 1.0f));
    float q = -0.0292195667f;
    q = fmaf(q, t, 0.140469076f);
    q = fmaf(q, t, -0.235575206f);
    q = fmaf(q, t, 0.137618668f);
    q = fmaf(q, t, -0.046936828f);
    q = fmaf(q, t, 0.0839353831f);
    q = fmaf(q, t, 0.11900294f);
    q = fmaf(q, t, 0.171740179f);
    q = fmaf(q, t, 0.20761365f);
    q = fmaf(q, t, 0.225675863f);
    q = fmaf(q, t, 0.225675835f);
    ec = e * t * q;
}

// source slots per LDS chunk (a multiple of 8): 128 FP32, 160 FP64 measured best
// of 128, 160 and 192 with the staging cull
#ifndef FSE_REAL_CH32
#define FSE_REAL_CH32 128
#endif
#ifndef FSE_REAL_CH64
#define FSE_REAL_CH64 160
#endif
// queued hits per thread before the wave flushes (deeper FP64 queues cost less
// occupancy than the extra flushes; in FP32 the gradient pass, whose pairs cost twice
// as much, measured faster at 48 and the value pass at 32, of 24, 32 and 48)
#ifndef FSE_QCAP32
#define FSE_QCAP32 32
#endif
#ifndef FSE_QCAP32G
#define FSE_QCAP32G 48
#endif
template <typename T, bool GRAD>
constexpr int qcap() { return sizeof(T) == 4 ? (GRAD ? FSE_QCAP32G : FSE_QCAP32) : 48; }
// source slots per chunk, and the chunk buffers a pass keeps: two (queued hits may
// outlive their chunk) for single FP64 passes, measured 6 % faster there.  FP32
// passes keep one: with two, even at the same four waves per SIMD (112-slot chunks,
// 32-entry queues), the fused gradient pass took 2.23 ms against 2.18 and the value
// pass 1.56 against 1.36.  Batched passes hold four times the values per chunk.
template <typename T, int NB> constexpr int real_nbuf() { return NB == 1 && sizeof(T) == 8 ? 2 : 1; }
template <typename T> constexpr int real_chunk() { return sizeof(T) == 4 ? FSE_REAL_CH32 : FSE_REAL_CH64; }
// queue entries: buffer slot indices, 16 bits (one-byte entries, which would fit
// the FP32 passes' 128 slots, measured 6 % slower in the FP32 value pass)
using QE = unsigned short;

// 1 when the sign bit of v is set (v < 0 or v = -0), else 0
__device__ __forceinline__ unsigned sign_bit(float v) { return __float_as_uint(v) >> 31; }
__device__ __forceinline__ unsigned sign_bit(double v) {
    return (unsigned)((unsigned long long)__double_as_longlong(v) >> 63);
}
// Wave-wide max (MAX) or min of an int, the same in every lane: an inclusive
// scan within each row of 16 lanes by DPP row shifts, then the row totals
// carried across rows by DPP row broadcasts, read from the last lane.  Lanes a
// DPP source does not reach take the identity.  No LDS traffic.
template <bool MAX> __device__ __forceinline__ int wave_reduce(int v) {
    constexpr int id = MAX ? INT_MIN : INT_MAX;
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));  // row_shr:1
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));  // row_shr:2
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));  // row_shr:4
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));  // row_shr:8
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max(int v) { return wave_reduce<true>(v); }
__device__ __forceinline__ int wave_min(int v) { return wave_reduce<false>(v); }

// queue row stride: the workgroup size rounded up to a power of two, so that a
// hit advances the queue pointer by a shift of the hit bit
__host__ __device__ inline int queue_row(int nthr) { return nthr <= 64 ? 64 : nthr <= 128 ? 128 : 256; }
// Far-away position for padding slots and idle lanes: every distance to it
// exceeds rc (its square may overflow to +inf, which fails the test as well).
constexpr double FAR = 1e18;

template <typename T>
struct __align__(4 * sizeof(T)) Pos4 {
    T x, y, z, pad;
};

// One pass over the pairs 0 < |x_t - x_s| <= rc of the targets of one cell.
// Every thread owns one target.  For each LDS chunk of neighbour sources the
// thread first tests all candidates and queues the hits (chunk indices) in a
// private LDS queue; the wave then evaluates the queued pairs together, so the
// erfc/exp work runs only for interacting pairs instead of for every candidate
// that some lane of the wave happens to hit.
//   GRAD = false: out = (accumulate ? out : 0) + sum_b-wise u^R + self_coef a   (NB batch members)
//   GRAD = true:  out(dx) += sum_b sum_pairs grad_r[w_t . G^R f_s + sgn w_s . G^R f_t]
//   WVAL (with GRAD): also out2 += sum_pairs G^R w_s + self_coef w_t per batch
//                 member (the real-space part of dL/df = K w), in the same pass
//   FVAL (with GRAD): also out3 += sum_pairs G^R f_s + self_coef f_t (the forward
//                 sum u's real-space part and self term), in the same pass
template <typename T, int KERNEL, int NB, bool GRAD, bool WVAL = false, bool FVAL = false>
__global__ __launch_bounds__(256) void k_real(CellGeo cg, PointsDev<T> pd, const T* __restrict__ a_r,
                                             const T* __restrict__ b_r, const T* __restrict__ w_r,
                                             int batch, T xi, T self_coef, T* out, int accumulate,
                                             T* out2, T* out3) {
    // sources: the cell list of the points; targets: their own cell list (the
    // same one when the targets are the sources; GRAD needs that)
    const int* __restrict__ cell_start = pd.cell_start;
    const T* __restrict__ x_r = pd.x_r;
    const int64_t n = pd.n;
    const int* __restrict__ tcell_start = pd.t_cell_start;
    const T* __restrict__ tx_r = pd.t_x_r;
    const int64_t nt = pd.t_n;
    const int* __restrict__ perm_r = pd.t_perm_r;
    const int* __restrict__ work_start = pd.t_work_start;
    constexpr bool TADJ = KERNEL == KTADJ;  // the stresslet adjoint: sources carry w, targets q and n
    constexpr int NS = TADJ ? 3 : ((KERNEL == FSE_STRESSLET || GRAD) ? 6 : 3);  // staged values per source
    constexpr int NO = (TADJ || FVAL) ? 6 : 3;  // accumulated values per target and batch member
    // source slots per LDS chunk
    constexpr int CH = real_chunk<T>();
    static_assert(CH % 8 == 0, "candidates are tested in groups of 8");
    // CARRY: queued hits may outlive their chunk by one chunk, so a chunk's end
    // evaluates only as many entries as keep every lane busy (plus what must go);
    // the chunks' positions and values alternate between two buffers.
    constexpr int NBUF = real_nbuf<T, NB>();
    constexpr bool CARRY = NBUF == 2;
    // sources in test form about the origin o: -2 (x - o) and |x - o|^2; a pair's
    // r = (x_t - o) - (x_s - o) comes from it too
    __shared__ Pos4<T> xq[NBUF * CH];
    __shared__ T ss[NB][NS][NBUF * CH];
    extern __shared__ __align__(16) unsigned char qd_raw[];
    QE* const qd = (QE*)qd_raw;  // hit queues: qcap (+ 8 with CARRY) rows of queue_row(blockDim.x) entries
    const int tid = threadIdx.x;
    const int nc = cg.ncell;
    const int nthr = blockDim.x;
    // work item -> (cell, slice): the last cell c with work_start[c] <= item
    const int ncells = nc * nc * nc;
    const int item = blockIdx.x;
    if (item >= work_start[ncells]) return;
    int lo = 0, hi = ncells;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (work_start[mid] <= item) lo = mid; else hi = mid;
    }
    const int cell = lo;
    const int cx = cell % nc, cy = (cell / nc) % nc, cz = cell / (nc * nc);
    const int b0 = blockIdx.y * NB;
    const int t0 = tcell_start[cell] + (item - work_start[cell]) * nthr;
    const int t1 = min(tcell_start[cell + 1], t0 + nthr);
    const T rc2 = (T)cg.rc2;
    // The origin o of the local coordinates: the cell corner c, or 0 in a direction
    // where -4 cells < c < 2 cells.  Then every target (in [c, c + cell)) and source
    // (in [c - cell, c + 2 cell)) is within a factor 2 of o, or o = 0, so x - o is
    // exact and a pair's (x_t - o) - (x_s - o) rounds to the same r as x_t - x_s.
    auto origin = [&](double c) { return (T)(c >= 2.0 * cg.cell || c <= -4.0 * cg.cell ? c : 0.0); };
    const T ox = origin(cg.lo[0] + cx * cg.cell), oy = origin(cg.lo[1] + cy * cg.cell),
            oz = origin(cg.lo[2] + cz * cg.cell);
    // the candidate test uses |xl|^2 + |xs_l|^2 - 2 xl . xs_l in these coordinates
    // (at most 5 cells from o in each direction), widened by 2^-13 cell^2: its FP32
    // rounding stays below 4e-5 cell^2; the exact r^2 <= rc^2 decides when a queued
    // pair is evaluated
    const T rc2t = (T)(cg.rc2 + cg.cell * cg.cell / 8192.0);
    const T xi2 = xi * xi;
    const T c2x = (T)(2.0 * INV_SQRTPI) * xi;       // 2 xi / sqrt(pi)
    const T c4x3 = (T)(4.0 * INV_SQRTPI) * xi * xi2;  // 4 xi^3 / sqrt(pi)
    const T sgn = (KERNEL == FSE_STOKESLET) ? (T)1 : (T)-1;
    // the 27 neighbour cells (empty beyond the box): lane k < 27 of every wave
    // holds the start and count of cell k
    __shared__ int ch_off[28], ch_base[27];
    __shared__ T ch_sh[27][3];  // periodic: the image shift of each neighbour cell's sources
    __shared__ int s_kc[4];    // kept sources per wave in a staging round
    __shared__ T s_bb[4][6];   // per wave: target bounding box (low x, y, z, high x, y, z)
    __shared__ T s_box[6];     // the work item's target bounding box
    int nb_s = 0, nb_n = 0;
    {
        const int lane = tid & 63;
        if (lane < 27) {
            int nb[3] = {cx + lane % 3 - 1, cy + (lane / 3) % 3 - 1, cz + lane / 9 - 1};
            T sh[3] = {(T)0, (T)0, (T)0};
            bool ok = true;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (cg.periodic) {
                    // the neighbour beyond a face is the cell across the box, its
                    // sources taken at their image next to this cell
                    if (nb[d] < 0) { nb[d] += nc; sh[d] = (T)-cg.L; }
                    else if (nb[d] >= nc) { nb[d] -= nc; sh[d] = (T)cg.L; }
                } else if (nb[d] < 0 || nb[d] >= nc) {
                    ok = false;
                }
            }
            if (ok) {
                const int cc = (nb[2] * nc + nb[1]) * nc + nb[0];
                nb_s = cell_start[cc];
                nb_n = cell_start[cc + 1] - nb_s;
            }
            if (tid < 27)
#pragma unroll
                for (int d = 0; d < 3; ++d) ch_sh[tid][d] = sh[d];
        }
    }
    int tot = nb_n;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) tot += __shfl_xor(tot, d);
    // chunks: at most CH - 27 sources on average, so that no chunk exceeds CH
    const int nch = (tot + (CH - 28)) / (CH - 27);
    for (int tb = t0; tb < t1; tb += nthr) {
        const int j = tb + tid;
        const bool act = j < t1;
        T xt0 = 0, xt1 = 0, xt2 = 0;
        if (act) {
            xt0 = tx_r[3 * (int64_t)j];
            xt1 = tx_r[3 * (int64_t)j + 1];
            xt2 = tx_r[3 * (int64_t)j + 2];
        }
        const T xl0 = xt0 - ox, xl1 = xt1 - oy, xl2 = xt2 - oz;
        // idle lanes: a squared norm beyond any cutoff
        const T At = act ? xl0 * xl0 + xl1 * xl1 + xl2 * xl2 : (T)FAR;
        // target-side values: f_t, w_t per batch member (gradient), or the target's
        // own q_t, n_t (stresslet adjoint)
        T ft[NB][3], wt[NB][3];
        // acc holds the pairs of one flush; sum the flush totals: the FP32 rounding of
        // a target whose total is dominated by a close pair then grows with the
        // number of flushes, not with the number of pairs
        // the gradient pass keeps its flush totals in FP64 (FP32 form): dL/dx sums
        // 1/r^2-type terms whose FP32 totals lose digits in dense clusters
        using S = typename std::conditional<GRAD, double, T>::type;
        T acc[NB][NO];
        S sum[NB][NO];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
            for (int d = 0; d < NO; ++d) {
                acc[b][d] = (T)0;
                sum[b][d] = (S)0;
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                ft[b][d] = wt[b][d] = (T)0;
                if ((GRAD || TADJ) && act && b0 + b < batch) {
                    ft[b][d] = a_r[((int64_t)(b0 + b) * n + j) * 3 + d];
                    wt[b][d] = (TADJ ? b_r : w_r)[((int64_t)(b0 + b) * n + j) * 3 + d];
                }
            }
        }
        T g0 = 0, g1 = 0, g2 = 0;
        double gs0 = 0, gs1 = 0, gs2 = 0;
        // stokeslet gradient, one batch member: the terms w_t (B f_s.r) and f_t (B w_s.r)
        // of every pair share the target's w_t and f_t, so their scalar factors add up
        // here (h1, h2, flush totals hs1, hs2) and meet w_t, f_t once at the end
        T h1 = 0, h2 = 0;
        double hs1 = 0, hs2 = 0;
        // this thread's hit queue: column tid of qd, QROW entries per row
        const int QROW = queue_row(nthr);
        const int qlog = QROW == 64 ? 6 : QROW == 128 ? 7 : 8;  // log2 of a row in entries
        const int qsh = qlog + 1;                               // and in bytes
        QE* const q0 = qd + tid;
        const int qcap = GRAD ? cg.qcap_grad : cg.qcap;
        QE* const qlim = q0 + (qcap - 8) * QROW;
        QE* qp = q0;
        int old = 0;  // CARRY: entries at the front of the queue from the previous chunk
        // widened test threshold folded into the target term: a hit is a negative sign
        const T Atc = At - rc2t;
        const bool wave_active = __any(act);
        // bounding box of the work item's targets about the origin o
        T bb_lo[3] = {act ? xl0 : (T)FAR, act ? xl1 : (T)FAR, act ? xl2 : (T)FAR};
        T bb_hi[3] = {act ? xl0 : (T)-FAR, act ? xl1 : (T)-FAR, act ? xl2 : (T)-FAR};
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                bb_lo[d] = min(bb_lo[d], __shfl_xor(bb_lo[d], o));
                bb_hi[d] = max(bb_hi[d], __shfl_xor(bb_hi[d], o));
            }
        if ((tid & 63) == 0)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                s_bb[tid >> 6][d] = bb_lo[d];
                s_bb[tid >> 6][3 + d] = bb_hi[d];
            }
        __syncthreads();
        if (tid < 6) {
            T v = s_bb[0][tid];
            for (int w = 1; w < (nthr >> 6); ++w) v = tid < 3 ? min(v, s_bb[w][tid]) : max(v, s_bb[w][tid]);
            s_box[tid] = v;
        }

        // One queued pair, without branches: a pair that is off (a lane past its
        // queue, the self pair, coincident points, or beyond the cutoff) adds exactly
        // zero (see the two precisions below).
        auto eval = [&](int kk, bool on) {
            const Pos4<T> pk = xq[kk];
            const T r0 = xl0 + (T)0.5 * pk.x, r1 = xl1 + (T)0.5 * pk.y, r2v = xl2 + (T)0.5 * pk.z;
            const T r2q = r0 * r0 + r1 * r1 + r2v * r2v;
            const bool use = on && r2q != (T)0 && r2q <= rc2;
            // FP32: r^2 = 1e30 makes e (and with it ec) exactly zero, and every kernel
            // term carries one of them, so the pair adds zero with no selects.  FP64:
            // exp of a huge argument takes the library's slow path, so evaluate at
            // r = r_c and zero the factors.
            const T r2 = use ? r2q : (sizeof(T) == 4 ? (T)1e30f : rc2);
            T r, ir, e, ec;
            radial<T>(xi, xi2, r2, r, ir, e, ec);
            if constexpr (sizeof(T) == 8) {
                ir = use ? ir : (T)0;
                e = use ? e : (T)0;
                ec = use ? ec : (T)0;
            }
            if constexpr (!GRAD) {
                if constexpr (KERNEL == FSE_STOKESLET) {
                    const T cd = ec * ir - c2x * e;
                    const T c1 = (ec * ir + c2x * e) * ir * ir;  // on r r^T
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const T f0 = ss[b][0][kk], f1 = ss[b][1][kk], f2 = ss[b][2][kk];
                        const T rf = (r0 * f0 + r1 * f1 + r2v * f2) * c1;
                        acc[b][0] += cd * f0 + rf * r0;
                        acc[b][1] += cd * f1 + rf * r1;
                        acc[b][2] += cd * f2 + rf * r2v;
                    }
                } else if constexpr (KERNEL == FSE_ROTLET) {
                    const T c = (ec * ir * ir + c2x * e * ir) * ir;  // on f x r
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const T f0 = ss[b][0][kk], f1 = ss[b][1][kk], f2 = ss[b][2][kk];
                        acc[b][0] += c * (f1 * r2v - f2 * r1);
                        acc[b][1] += c * (f2 * r0 - f0 * r2v);
                        acc[b][2] += c * (f0 * r1 - f1 * r0);
                    }
                } else if constexpr (TADJ) {
                    // D_lm(t) += T^R_jlm(x_s - x_t) w_j = -T^R_jlm(r) w_j, r = x_t - x_s:
                    //   -(A1 (h.w) h_l h_m + A2 (w_l h_m + w_m h_l + d_lm h.w)),
                    // contracted at once with the target's n (dq) and q (dn)
                    const T A1 = -(T)2 * ir * ((T)3 * ec * ir + c2x * ((T)3 + (T)2 * xi2 * r2) * e);
                    const T A2 = c4x3 * r * e;
                    const T h0 = r0 * ir, h1 = r1 * ir, h2 = r2v * ir;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const T w0 = ss[b][0][kk], w1 = ss[b][1][kk], w2 = ss[b][2][kk];
                        const T* qv = ft[b];
                        const T* nv = wt[b];
                        const T hw = h0 * w0 + h1 * w1 + h2 * w2;
                        // r . n_t in FP64: n_t is the target's normal, so for points on a
                        // smooth surface r . n_t ~ r^2 / 2 cancels as in the forward pass
                        const T hn = (T)((double)r0 * nv[0] + (double)r1 * nv[1] + (double)r2v * nv[2]) * ir;
                        const T hq = h0 * qv[0] + h1 * qv[1] + h2 * qv[2];
                        const T wn = w0 * nv[0] + w1 * nv[1] + w2 * nv[2];
                        const T wq = w0 * qv[0] + w1 * qv[1] + w2 * qv[2];
                        const T cq = A1 * hw * hn + A2 * wn, cn = A1 * hw * hq + A2 * wq;
                        const T a2hw = A2 * hw;
                        acc[b][0] -= cq * h0 + A2 * hn * w0 + a2hw * nv[0];
                        acc[b][1] -= cq * h1 + A2 * hn * w1 + a2hw * nv[1];
                        acc[b][2] -= cq * h2 + A2 * hn * w2 + a2hw * nv[2];
                        acc[b][3] -= cn * h0 + A2 * hq * w0 + a2hw * qv[0];
                        acc[b][4] -= cn * h1 + A2 * hq * w1 + a2hw * qv[1];
                        acc[b][5] -= cn * h2 + A2 * hq * w2 + a2hw * qv[2];
                    }
                } else {
                    const T A1 = -(T)2 * ir * ((T)3 * ec * ir + c2x * ((T)3 + (T)2 * xi2 * r2) * e);
                    const T A2 = c4x3 * r * e;
                    const T h0 = r0 * ir, h1 = r1 * ir, h2 = r2v * ir;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const T q0 = ss[b][0][kk], q1 = ss[b][1][kk], q2 = ss[b][2][kk];
                        const T n0 = ss[b][3][kk], n1 = ss[b][4][kk], n2 = ss[b][5][kk];
                        const T hq = h0 * q0 + h1 * q1 + h2 * q2;
                        // r . n in FP64: for sources on a smooth surface with n its normal,
                        // r . n ~ r^2 / 2 cancels in the sum, so FP32 products would lose
                        // it for close pairs (the FP32 products are exact in FP64)
                        const T hn = (T)((double)r0 * n0 + (double)r1 * n1 + (double)r2v * n2) * ir;
                        const T nq = n0 * q0 + n1 * q1 + n2 * q2;
                        const T s1c = A1 * hn * hq + A2 * nq;
                        acc[b][0] += s1c * h0 + A2 * (n0 * hq + q0 * hn);
                        acc[b][1] += s1c * h1 + A2 * (n1 * hq + q1 * hn);
                        acc[b][2] += s1c * h2 + A2 * (n2 * hq + q2 * hn);
                    }
                }
            } else {
                const T rv[3] = {r0, r1, r2v};
                if constexpr (KERNEL == FSE_STOKESLET) {
                    // w.S^R f = a(r) (w.f) + (b(r)/r^2) (w.r)(f.r), a = t1 - t2, b = t1 + t2 with
                    // t1 = erfc/r, t2 = 2 xi e/sqrt(pi): a' = -b/r + t3, b' = -b/r - t3,
                    // t3 = 4 xi^3 r e/sqrt(pi), and (b/r^2)' = (b' - 2 b/r)/r^2
                    const T t1 = ec * ir, t2 = c2x * e, t3 = c4x3 * r * e;
                    const T b_ = t1 + t2, bir = b_ * ir, ir2 = ir * ir;
                    const T da = t3 - bir;
                    const T db = -bir - t3;
                    const T Bc = b_ * ir2;
                    const T dB = (db - (T)2 * bir) * ir2;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const T fn[3] = {ss[b][0][kk], ss[b][1][kk], ss[b][2][kk]};
                        const T wn[3] = {ss[b][3][kk], ss[b][4][kk], ss[b][5][kk]};
                        const T* fp = ft[b];
                        const T* wp = wt[b];
                        const T wf1 = wp[0] * fn[0] + wp[1] * fn[1] + wp[2] * fn[2];
                        const T wr1 = wp[0] * rv[0] + wp[1] * rv[1] + wp[2] * rv[2];
                        const T fr1 = fn[0] * rv[0] + fn[1] * rv[1] + fn[2] * rv[2];
                        const T wf2 = wn[0] * fp[0] + wn[1] * fp[1] + wn[2] * fp[2];
                        const T wr2 = wn[0] * rv[0] + wn[1] * rv[1] + wn[2] * rv[2];
                        const T fr2 = fp[0] * rv[0] + fp[1] * rv[1] + fp[2] * rv[2];
                        const T rad = (da * (wf1 + sgn * wf2) + dB * (wr1 * fr1 + sgn * wr2 * fr2)) * ir;
                        const T a_ = t1 - t2;
                        if constexpr (WVAL) {
                            const T bw = Bc * wr2;
                            acc[b][0] += a_ * wn[0] + bw * rv[0];
                            acc[b][1] += a_ * wn[1] + bw * rv[1];
                            acc[b][2] += a_ * wn[2] + bw * rv[2];
                        }
                        if constexpr (FVAL) {
                            const T bf = Bc * fr1;
                            acc[b][3] += a_ * fn[0] + bf * rv[0];
                            acc[b][4] += a_ * fn[1] + bf * rv[1];
                            acc[b][5] += a_ * fn[2] + bf * rv[2];
                        }
                        if constexpr (NB == 1) {
                            const T al = Bc * wr1, be = Bc * fr2;  // sgn = 1 for the stokeslet
                            g0 += rad * rv[0] + al * fn[0] + be * wn[0];
                            g1 += rad * rv[1] + al * fn[1] + be * wn[1];
                            g2 += rad * rv[2] + al * fn[2] + be * wn[2];
                            h1 += Bc * fr1;
                            h2 += Bc * wr2;
                        } else {
                            g0 += rad * rv[0] + Bc * (wp[0] * fr1 + fn[0] * wr1 + sgn * (wn[0] * fr2 + fp[0] * wr2));
                            g1 += rad * rv[1] + Bc * (wp[1] * fr1 + fn[1] * wr1 + sgn * (wn[1] * fr2 + fp[1] * wr2));
                            g2 += rad * rv[2] + Bc * (wp[2] * fr1 + fn[2] * wr1 + sgn * (wn[2] * fr2 + fp[2] * wr2));
                        }
                    }
                } else {
                    // w.Omega^R f = psi(r) r.(w x f), psi = rho/r
                    const T rho = ec * ir * ir + c2x * e * ir;
                    const T drho = -(T)2 * ec * ir * ir * ir - (T)2 * c2x * e * ir * ir - c4x3 * e;
                    const T psi = rho * ir;
                    const T dpsi = drho * ir - rho * ir * ir;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const T fn[3] = {ss[b][0][kk], ss[b][1][kk], ss[b][2][kk]};
                        const T wn[3] = {ss[b][3][kk], ss[b][4][kk], ss[b][5][kk]};
                        const T* fp = ft[b];
                        const T* wp = wt[b];
                        const T cc0 = (wp[1] * fn[2] - wp[2] * fn[1]) + sgn * (wn[1] * fp[2] - wn[2] * fp[1]);
                        const T cc1 = (wp[2] * fn[0] - wp[0] * fn[2]) + sgn * (wn[2] * fp[0] - wn[0] * fp[2]);
                        const T cc2 = (wp[0] * fn[1] - wp[1] * fn[0]) + sgn * (wn[0] * fp[1] - wn[1] * fp[0]);
                        const T rc = (rv[0] * cc0 + rv[1] * cc1 + rv[2] * cc2) * dpsi * ir;
                        if constexpr (WVAL) {
                            acc[b][0] += psi * (wn[1] * rv[2] - wn[2] * rv[1]);
                            acc[b][1] += psi * (wn[2] * rv[0] - wn[0] * rv[2]);
                            acc[b][2] += psi * (wn[0] * rv[1] - wn[1] * rv[0]);
                        }
                        if constexpr (FVAL) {
                            acc[b][3] += psi * (fn[1] * rv[2] - fn[2] * rv[1]);
                            acc[b][4] += psi * (fn[2] * rv[0] - fn[0] * rv[2]);
                            acc[b][5] += psi * (fn[0] * rv[1] - fn[1] * rv[0]);
                        }
                        g0 += rc * rv[0] + psi * cc0;
                        g1 += rc * rv[1] + psi * cc1;
                        g2 += rc * rv[2] + psi * cc2;
                    }
                }
            }
        };
        // Evaluate the first E entries of every lane's queue (E the same for the
        // whole wave; a lane with fewer entries idles for the rest).  mode 2 (the
        // work item's last chunk, or no CARRY): E = the longest queue, all of it.
        // mode 0 (a queue near full inside a chunk) and mode 1 (a chunk's end):
        // E = the shortest queue, so every lane is busy, but at least what leaves
        // each queue at most qcap - 16 entries and, at a chunk's end, at least the
        // entries of the previous chunk, whose buffer the next chunk overwrites.
        // The entries left move to the front of the queue, in order.
        auto flush = [&](int mode) {
            const int qn = (int)(qp - q0) >> qlog;
            const int qmax = wave_max(qn);
            int E = qmax;
            if (CARRY && mode != 2) {
                // (lanes without a target have empty queues and do not count)
                E = max(wave_min(act ? qn : 1 << 20), qmax - (qcap - 16));
                if (mode == 1) E = max(E, wave_max(old));
            }
            for (int e = 0; e < E; ++e) {
                const bool on = e < qn;
                const int kk = q0[e * QROW];
                eval(on ? kk : 0, on);
            }
            if constexpr (CARRY) {
                const int rest = max(qn - E, 0);
                // move rows [E, qmax) to [0, qmax - E), eight at a time, in every lane:
                // rows past a lane's own entries carry stale values that are never
                // read as entries (the queue has 8 spare rows for the last group).  A
                // group reads before it writes, and reads only rows above every row
                // written so far.
                if (E > 0) {
                    const QE* src = q0 + E * QROW;
                    for (int k = 0; k < qmax - E; k += 8) {
                        QE v[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) v[u] = src[(k + u) * QROW];
#pragma unroll
                        for (int u = 0; u < 8; ++u) q0[(k + u) * QROW] = v[u];
                    }
                }
                qp = q0 + rest * QROW;
                old = mode == 1 ? rest : max(old - E, 0);
            } else {
                qp = q0;
            }
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int d = 0; d < NO; ++d) {
                    sum[b][d] += (S)acc[b][d];
                    acc[b][d] = (T)0;
                }
            if constexpr (GRAD) {
                gs0 += g0;
                hs1 += h1;
                hs2 += h2;
                h1 = h2 = (T)0;
                gs1 += g1;
                gs2 += g2;
                g0 = g1 = g2 = (T)0;
            }
        };

        // Each chunk takes the same fraction of every neighbour cell: chunk c of NCH
        // holds sources [lo(c), lo(c + 1)) of cell k, lo(c) = floor(c n_k / NCH).
        // Every target then sees a sample of its whole neighbourhood in each chunk,
        // so the hit counts of the lanes are alike and the flushes waste few lanes
        // (cell-by-cell chunks give hit counts that depend on where the target
        // sits in its cell).
        // lo(c + 1) - lo(c) = nq + (1 if the running remainder wraps), nq = n_k / NCH
        const int nq = nb_n / nch;
        const int nr = nb_n - nq * nch;
        int cur = nb_s, rem = 0;
        for (int c = 0; c < nch; ++c) {
            const int base = CARRY ? (c & 1) * CH : 0;  // this chunk's buffer
            __syncthreads();
            if (tid < 32) {
                int cnt = 0, base = 0;
                if (tid < 27) {
                    rem += nr;
                    const int wrap = rem >= nch ? 1 : 0;
                    rem -= wrap * nch;
                    cnt = nq + wrap;
                    base = cur;
                    cur += cnt;
                }
                int inc = cnt;
#pragma unroll
                for (int d = 1; d < 32; d <<= 1) {
                    const int v = __shfl_up(inc, d, 32);
                    if (tid >= d) inc += v;
                }
                if (tid < 27) {
                    ch_off[tid + 1] = inc;
                    ch_base[tid] = base - (inc - cnt);  // slot q of cell k holds source ch_base[k] + q
                }
                if (tid == 0) ch_off[0] = 0;
            }
            __syncthreads();
            const int cntc = ch_off[27];
            // stage the chunk's sources, dropping those farther than rc from the
            // targets' bounding box (about a quarter of the 27 cells' volume): the
            // kept ones are compacted in slot order (wave ballots), so the candidate
            // loop below runs over fewer slots
            int kept = 0;
            for (int q0 = 0; q0 < cntc; q0 += nthr) {
                const int q = q0 + tid;
                Pos4<T> pq;
                bool keep = false;
                int src = 0;
                if (q < cntc) {
                    int kc = 0;  // the last cell whose slots start at or before q
#pragma unroll
                    for (int st = 16; st > 0; st >>= 1)
                        if (kc + st <= 26 && ch_off[kc + st] <= q) kc += st;
                    const int k = ch_base[kc] + q;
                    T px = x_r[3 * (int64_t)k], py = x_r[3 * (int64_t)k + 1], pz = x_r[3 * (int64_t)k + 2];
                    if (cg.periodic) {
                        px += ch_sh[kc][0];
                        py += ch_sh[kc][1];
                        pz += ch_sh[kc][2];
                    }
                    src = k;
                    const T l0 = px - ox, l1 = py - oy, l2 = pz - oz;
                    pq.x = (T)-2 * l0;
                    pq.y = (T)-2 * l1;
                    pq.z = (T)-2 * l2;
                    pq.pad = l0 * l0 + l1 * l1 + l2 * l2;
                    const T e0 = max(max(s_box[0] - l0, l0 - s_box[3]), (T)0);
                    const T e1 = max(max(s_box[1] - l1, l1 - s_box[4]), (T)0);
                    const T e2 = max(max(s_box[2] - l2, l2 - s_box[5]), (T)0);
                    keep = e0 * e0 + e1 * e1 + e2 * e2 <= rc2t;
                }
                const unsigned long long m = __ballot(keep);
                if ((tid & 63) == 0) s_kc[tid >> 6] = __popcll(m);
                __syncthreads();
                int off = kept, all = 0;
                for (int w = 0; w < (nthr >> 6); ++w) {
                    const int cw = s_kc[w];
                    off += w < (tid >> 6) ? cw : 0;
                    all += cw;
                }
                if (keep) {
                    const int slot = off + __popcll(m & ((1ull << (tid & 63)) - 1ull));
                    xq[base + slot] = pq;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if (b0 + b < batch) {
                            const T* ap = (TADJ ? w_r : a_r) + ((int64_t)(b0 + b) * n + src) * 3;
#pragma unroll
                            for (int d = 0; d < 3; ++d) ss[b][d][base + slot] = ap[d];
                            if constexpr (NS == 6) {
                                const T* bp = (GRAD ? w_r : b_r) + ((int64_t)(b0 + b) * n + src) * 3;
#pragma unroll
                                for (int d = 0; d < 3; ++d) ss[b][3 + d][base + slot] = bp[d];
                            }
                        } else {
#pragma unroll
                            for (int d = 0; d < NS; ++d) ss[b][d][base + slot] = (T)0;
                        }
                    }
                }
                kept += all;
                __syncthreads();
            }
            // slots up to the next multiple of 8: never within the cutoff
            if (tid < ((kept + 7) & ~7) - kept) {
                Pos4<T> pf;
                pf.x = pf.y = pf.z = (T)0;
                pf.pad = (T)FAR;
                xq[base + kept + tid] = pf;
            }
            __syncthreads();
            if (!wave_active) continue;
            // candidates in groups of 8 (padding slots are far away); the self pair
            // and coincident points (r^2 = 0) are queued and skipped when evaluated
            const int cnt8 = (kept + 7) & ~7;
            // buffer slot indices two to a register (low, high half), advanced by 8 per group
            unsigned kp[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) kp[v] = (unsigned)(base + 2 * v) | ((unsigned)(base + 2 * v + 1) << 16);
            for (int k8 = 0; k8 < cnt8; k8 += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const Pos4<T> pq = xq[base + k8 + u];
                    const T d = fma(xl0, pq.x, fma(xl1, pq.y, fma(xl2, pq.z, Atc + pq.pad)));
                    *qp = (QE)((u & 1) ? (kp[u >> 1] >> 16) : kp[u >> 1]);
                    qp = (QE*)((char*)qp + (sign_bit(d) << qsh));
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) kp[v] += 0x00080008u;
                if (__any(qp > qlim)) flush(0);
            }
            flush(c == nch - 1 ? 2 : 1);
        }
        if (act) {
            const int64_t i = perm_r[j];
            if constexpr (TADJ) {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (b0 + b >= batch) break;
                    T* o1 = out + ((int64_t)(b0 + b) * nt + i) * 3;
                    T* o2 = out2 + ((int64_t)(b0 + b) * nt + i) * 3;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        o1[d] += sum[b][d];
                        o2[d] += sum[b][3 + d];
                    }
                }
            } else if constexpr (!GRAD) {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (b0 + b >= batch) break;
                    T* o = out + ((int64_t)(b0 + b) * nt + i) * 3;
                    // the self term exists only where a target is its own source
                    // (self_coef = 0 for separate targets)
                    T self[3] = {(T)0, (T)0, (T)0};
                    if (self_coef != (T)0) {
                        const T* a = a_r + ((int64_t)(b0 + b) * n + j) * 3;
#pragma unroll
                        for (int d = 0; d < 3; ++d) self[d] = self_coef * a[d];
                    }
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const T prev = accumulate ? o[d] : (T)0;
                        o[d] = prev + sum[b][d] + self[d];
                    }
                }
            } else {
                if constexpr (KERNEL == FSE_STOKESLET && NB == 1) {
                    gs0 += (double)wt[0][0] * hs1 + (double)ft[0][0] * hs2;
                    gs1 += (double)wt[0][1] * hs1 + (double)ft[0][1] * hs2;
                    gs2 += (double)wt[0][2] * hs1 + (double)ft[0][2] * hs2;
                }
                out[3 * i] = (T)((double)out[3 * i] + gs0);
                out[3 * i + 1] = (T)((double)out[3 * i + 1] + gs1);
                out[3 * i + 2] = (T)((double)out[3 * i + 2] + gs2);
                if constexpr (WVAL) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if (b0 + b >= batch) break;
                        T* o = out2 + ((int64_t)(b0 + b) * n + i) * 3;
#pragma unroll
                        for (int d = 0; d < 3; ++d) o[d] = (T)((S)o[d] + sum[b][d] + (S)(self_coef * wt[b][d]));
                    }
                }
                if constexpr (FVAL) {
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        if (b0 + b >= batch) break;
                        T* o = out3 + ((int64_t)(b0 + b) * n + i) * 3;
#pragma unroll
                        for (int d = 0; d < 3; ++d)
                            o[d] = (T)((S)o[d] + sum[b][3 + d] + (S)(self_coef * ft[b][d]));
                    }
                }
            }
        }
    }
}

}  // namespace

// Threads per work item (= targets per slice of a cell): the whole waves that
// hold a cell of mean occupancy, at most 256; fuller cells are cut into several
// work items, so no wave of a workgroup sits idle for the typical cell.
// the plan's queue depths start at these defaults and may be tuned (fse_plan_autotune)
int default_qcap(int elem_bytes, bool grad) {
    return elem_bytes == 4 ? (grad ? qcap<float, true>() : qcap<float, false>()) : qcap<double, false>();
}

// dynamic LDS of a pass's hit queues: qcap rows of queue_row(thr) entries, and 8
// spare rows for the queue moves of two-buffer passes (the FP32 passes keep their
// LDS within what eight workgroups per CU hold)
template <typename T> size_t queue_bytes(int qcap, unsigned thr, int NB) {
    const int spare = (NB == 1 ? real_nbuf<T, 1>() : real_nbuf<T, 4>()) == 2 ? 8 : 0;
    return (size_t)(qcap + spare) * queue_row((int)thr) * sizeof(QE);
}

unsigned real_threads(int64_t n, int64_t ncells, int max_waves) {
    const double mean = (double)n / (double)ncells;
    const int waves = (int)std::ceil(mean / 64.0);
    return 64u * (unsigned)std::min(std::max(1, std::min(4, max_waves)), std::max(1, waves));
}

template <typename T>
void launch_real(int kernel, const CellGeo& c, const PointsDev<T>& p, const T* src_a_r,
                 const T* src_b_r, int batch, double xi, double self_coef, T* u, int accumulate,
                 hipStream_t st) {
    const unsigned ncells = (unsigned)c.ncell * c.ncell * c.ncell;
    const int NBc = batch == 1 ? 1 : 4;
    const unsigned thr = (unsigned)p.t_real_S;
    // at most ceil(nt / S) + ncells work items; the surplus workgroups return at once
    const unsigned items = (unsigned)((p.t_n + thr - 1) / thr + ncells);
    const size_t qbytes = queue_bytes<T>(c.qcap, thr, NBc);
    dim3 grd(items, (batch + NBc - 1) / NBc);
#define LAUNCH(K, NB)                                                                                     \
    hipLaunchKernelGGL((k_real<T, K, NB, false>), grd, dim3(thr), qbytes, st, c, p, src_a_r, src_b_r,        \
                       (const T*)nullptr, batch, (T)xi, (T)self_coef, u, accumulate, (T*)nullptr, (T*)nullptr)
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
                      int batch, double xi, double self_coef, T* dx, T* dsrc, hipStream_t st, T* u) {
    // u (with dsrc, batch 1 only; ignored otherwise): the forward sum's real part and
    // self term are added to u in the same pass over the pairs
    const unsigned ncells = (unsigned)c.ncell * c.ncell * c.ncell;
    const unsigned thr = (unsigned)p.real_S;
    const unsigned items = (unsigned)((p.n + thr - 1) / thr + ncells);
    // batch members in groups of 4 per pass; each pass adds to dx (and dsrc)
    for (int b0 = 0; b0 < batch; b0 += 4) {
        const int nb = batch - b0 < 4 ? batch - b0 : 4;
        const size_t qbytes = queue_bytes<T>(c.qcap_grad, thr, nb == 1 ? 1 : 4);
        const T* f = f_r + (int64_t)b0 * p.n * 3;
        const T* w = w_r + (int64_t)b0 * p.n * 3;
        T* ds = dsrc ? dsrc + (int64_t)b0 * p.n * 3 : nullptr;
        T* uo = (u && batch == 1) ? u : nullptr;
#define LAUNCHG(K, NB, WV, FV)                                                                            \
        hipLaunchKernelGGL((k_real<T, K, NB, true, WV, FV>), dim3(items), dim3(thr), qbytes, st, c, p, f,      \
                           (const T*)nullptr, w, nb, (T)xi, (T)self_coef, dx, 1, ds, uo)
#define LAUNCHK(K)                                                                                        \
        if (ds && uo && nb == 1) LAUNCHG(K, 1, true, true);                                               \
        else if (ds) { if (nb == 1) LAUNCHG(K, 1, true, false); else LAUNCHG(K, 4, true, false); }        \
        else { if (nb == 1) LAUNCHG(K, 1, false, false); else LAUNCHG(K, 4, false, false); }
        if (kernel == FSE_STOKESLET) {
            LAUNCHK(FSE_STOKESLET)
        } else {
            LAUNCHK(FSE_ROTLET)
        }
#undef LAUNCHK
#undef LAUNCHG
    }
}

template <typename T>
void launch_real_tadj(const CellGeo& c, const PointsDev<T>& p, const T* q_r, const T* n_r, const T* w_r,
                      int batch, double xi, T* dq, T* dn, hipStream_t st) {
    const unsigned ncells = (unsigned)c.ncell * c.ncell * c.ncell;
    const unsigned thr = (unsigned)p.t_real_S;
    const unsigned items = (unsigned)((p.t_n + thr - 1) / thr + ncells);
    const size_t qbytes = queue_bytes<T>(c.qcap, thr, 1);
    // one batch member per workgroup row (six accumulators per member)
    hipLaunchKernelGGL((k_real<T, KTADJ, 1, false>), dim3(items, batch), dim3(thr), qbytes, st, c, p, q_r, n_r,
                       w_r, batch, (T)xi, (T)0, dq, 1, dn, (T*)nullptr);
}

#define INST(T)                                                                                     \
    template void launch_real_tadj<T>(const CellGeo&, const PointsDev<T>&, const T*, const T*, const T*, \
                                      int, double, T*, T*, hipStream_t);                            \
    template void launch_real<T>(int, const CellGeo&, const PointsDev<T>&, const T*, const T*, int, \
                                 double, double, T*, int, hipStream_t);                             \
    template void launch_real_grad<T>(int, const CellGeo&, const PointsDev<T>&, const T*, const T*, \
                                      int, double, double, T*, T*, hipStream_t, T*);
INST(float)
INST(double)
#undef INST

}  // namespace fse
