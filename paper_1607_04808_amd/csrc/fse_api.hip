// C ABI of libfse (declared in include/fse.h): parameters and geometry, plan
// workspace, the FP64 precompute, and the orchestration of the hot path
// (bin -> spread -> FFT/scale/IFFT -> gather -> real space).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "fse_common.h"

using namespace fse;

namespace {

thread_local char g_err[512] = "";

void set_err(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

#define HIPCHK(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            set_err("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
            return FSE_EHIP;                                                      \
        }                                                                         \
    } while (0)

#define LAUNCHCHK()                                                               \
    do {                                                                          \
        hipError_t e_ = hipGetLastError();                                        \
        if (e_ != hipSuccess) {                                                   \
            set_err("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
            return FSE_EHIP;                                                      \
        }                                                                         \
    } while (0)

constexpr double PI = 3.14159265358979323846;
// Mt <= 1024: window starts are packed in 10 bits per direction, and n = 2 Mt <= 2048
// keeps one line set of every FFT pass within 160 KB of LDS (fft_fits checks the
// six-component stresslet z-pass, whose FP64 lines stop at n = 1364)
constexpr int MAX_MT = 1024;
constexpr int MAX_CELLS_PER_SIDE = 128;
constexpr int MIN_BIN_SIDE = 4, MAX_BIN_SIDE = 8;  // the range a tuning may set

bool smooth7(int n) {
    if (n <= 0) return false;
    for (int p : {2, 3, 5, 7})
        while (n % p == 0) n /= p;
    return n == 1;
}

// radix stages (DIF order) for n: 8s first, then 7, 5, a final 4 or 2, then 3s
int factorize(int n, int* rad) {
    int ns = 0;
    int m = n;
    int c7 = 0, c5 = 0, c3 = 0, c2 = 0;
    while (m % 7 == 0) { m /= 7; ++c7; }
    while (m % 5 == 0) { m /= 5; ++c5; }
    while (m % 3 == 0) { m /= 3; ++c3; }
    while (m % 2 == 0) { m /= 2; ++c2; }
    if (m != 1) return -1;
    while (c2 >= 3) { rad[ns++] = 8; c2 -= 3; }
    for (int i = 0; i < c7; ++i) rad[ns++] = 7;
    for (int i = 0; i < c5; ++i) rad[ns++] = 5;
    if (c2 == 2) rad[ns++] = 4;
    else if (c2 == 1) rad[ns++] = 2;
    for (int i = 0; i < c3; ++i) rad[ns++] = 3;
    return ns;
}

// position p of the in-place DIF output holds frequency rev[p]
void digit_reverse(const int* rad, int ns, int n, std::vector<int>& rev) {
    rev.assign(n, 0);
    for (int p = 0; p < n; ++p) {
        // walk the stages: p = k2 * m + q; frequency = r * rev_sub(q) + k2
        int q = p, L = n;
        int mult = 1, acc = 0;
        for (int s = 0; s < ns; ++s) {
            const int r = rad[s], m = L / r;
            const int k2 = q / m;
            q -= k2 * m;
            acc += mult * k2;
            mult *= r;
            L = m;
        }
        rev[p] = acc;
    }
}

fse_status_t compute_geometry(fse_kernel_t kernel, const fse_params_t* p, fse_geometry_t* g) {
    if (!p || !g) { set_err("null argument"); return FSE_EINVAL; }
    if (kernel < FSE_STOKESLET || kernel > FSE_ROTLET) { set_err("unknown kernel %d", (int)kernel); return FSE_EINVAL; }
    if (!(p->xi > 0 && isfinite(p->xi))) { set_err("xi must be > 0"); return FSE_EINVAL; }
    if (!(p->rc > 0 && isfinite(p->rc))) { set_err("rc must be > 0"); return FSE_EINVAL; }
    if (p->M < 1) { set_err("M must be >= 1"); return FSE_EINVAL; }
    if (p->P < 2 || p->P > 32) { set_err("P must be in [2, 32]"); return FSE_EINVAL; }
    if (!(p->L > 0 && isfinite(p->L))) { set_err("L must be > 0"); return FSE_EINVAL; }
    for (int d = 0; d < 3; ++d)
        if (!isfinite(p->box_lo[d])) { set_err("box_lo must be finite"); return FSE_EINVAL; }
    if (p->deltaL_rule != 0 && p->deltaL_rule != 1) { set_err("deltaL_rule must be 0 or 1"); return FSE_EINVAL; }
    if (!(p->C >= 0 && p->C < 10)) { set_err("C out of range"); return FSE_EINVAL; }
    if (p->periodic != 0 && p->periodic != 1) { set_err("periodic must be 0 or 1"); return FSE_EINVAL; }
    memset(g, 0, sizeof *g);
    const double C = p->C > 0 ? p->C : 0.976;
    if (p->periodic) {
        // Section 1.1: the M^3 grid covers one period; its DFT is taken as the even
        // frequencies of the doubled grid the transforms work on
        if (kernel != FSE_STOKESLET) { set_err("the triply periodic sum is the stokeslet's (Section 1.1)"); return FSE_EINVAL; }
        if (!(p->rc <= 0.5 * p->L)) { set_err("periodic: rc must be <= L/2"); return FSE_EINVAL; }
        if (p->P > p->M) { set_err("periodic: P must be <= M"); return FSE_EINVAL; }
        if (!smooth7(2 * p->M)) { set_err("periodic: 2*M=%d does not factor into 2,3,5,7", 2 * p->M); return FSE_EINVAL; }
        // the extended grid's last window start is M - 1 (even P) or M (odd P)
        if (p->M + (p->P & 1) > MAX_MT) {
            set_err("grid size M=%d above the supported %d (%d for odd P)", p->M, MAX_MT, MAX_MT - 1);
            return FSE_EINVAL;
        }
        const double h = p->L / p->M, d = h * p->P, m = C * sqrt(PI * p->P);
        g->Mt = p->M;
        g->n_fft = 2 * p->M;
        g->h = h;
        g->d = d;
        g->m = m;
        g->eta = (p->xi * d / m) * (p->xi * d / m);
        g->alpha = 2.0 * p->xi * p->xi / g->eta;
        g->Lt = p->L;
        g->deltaL = 0.0;
        for (int k = 0; k < 3; ++k) g->x0[k] = p->box_lo[k];
        g->Mg = 0;
        g->R = 0.0;
        g->kinf = PI / h;
        int nc = (int)floor(p->L / p->rc);
        if (nc < 1) nc = 1;
        if (nc > MAX_CELLS_PER_SIDE) nc = MAX_CELLS_PER_SIDE;
        g->ncell = nc;
        g->cell = p->L / nc;
        int rad[MAX_RADICES];
        const int ns = factorize(g->n_fft, rad);
        if (ns < 0 || ns > 7) { set_err("cannot factor n=%d", g->n_fft); return FSE_EINVAL; }
        for (int s = 0; s < ns; ++s) g->radices[s] = rad[s];
        return FSE_OK;
    }
    const double h = p->L / p->M;
    const double d = h * p->P;
    const double m = C * sqrt(PI * p->P);
    const double eta = (p->xi * d / m) * (p->xi * d / m);
    double dL = d;
    if (p->deltaL_rule == 1 && eta < 1.0) {
        const double need = sqrt(2.0 * (1.0 - eta) * m * m / (p->xi * p->xi));
        if (need > dL) dL = need;
    }
    const int Mt_min = p->M + (int)ceil(dL / h - 1e-12);
    int Mt;
    if (p->Mt > 0) {
        Mt = p->Mt;
        if (Mt < Mt_min) { set_err("Mt=%d below the minimum %d", Mt, Mt_min); return FSE_EINVAL; }
        if (!smooth7(2 * Mt)) { set_err("2*Mt=%d does not factor into 2,3,5,7", 2 * Mt); return FSE_EINVAL; }
    } else {
        Mt = Mt_min;
        while (!smooth7(2 * Mt)) ++Mt;
    }
    if (Mt > MAX_MT) { set_err("grid size Mt=%d above the supported %d", Mt, MAX_MT); return FSE_EINVAL; }
    g->Mt = Mt;
    g->n_fft = 2 * Mt;
    g->h = h;
    g->d = d;
    g->m = m;
    g->eta = eta;
    g->alpha = 2.0 * p->xi * p->xi / eta;
    g->Lt = Mt * h;
    g->deltaL = g->Lt - p->L;
    for (int k = 0; k < 3; ++k) g->x0[k] = p->box_lo[k] - 0.5 * (g->Lt - p->L);
    int Mg = (int)floor((1.0 + sqrt(3.0)) * Mt) + 1;
    if (Mg % 2) ++Mg;
    g->Mg = Mg;
    g->R = sqrt(3.0) * g->Lt;
    g->kinf = PI / h;
    int nc = (int)floor(p->L / p->rc);
    if (nc < 1) nc = 1;
    if (nc > MAX_CELLS_PER_SIDE) nc = MAX_CELLS_PER_SIDE;
    g->ncell = nc;
    g->cell = p->L / nc;
    int rad[MAX_RADICES];
    const int ns = factorize(g->n_fft, rad);
    if (ns < 0 || ns > 7) { set_err("cannot factor n=%d", g->n_fft); return FSE_EINVAL; }
    for (int s = 0; s < ns; ++s) g->radices[s] = rad[s];
    return FSE_OK;
}

// Optional per-stage timing with HIP events on the plan's stream.
enum Stage {
    ST_BIN, ST_PERMUTE, ST_SPREAD, ST_FFTX, ST_FFTY, ST_FFTZ, ST_FFTYI, ST_FFTXI, ST_GATHER, ST_REAL,
    ST_GGRAD, ST_RGRAD, ST_COUNT
};
static_assert(ST_COUNT == FSE_NSTAGES, "stage count");
const char* const STAGE_NAMES[ST_COUNT] = {"bin",       "permute",    "spread",  "fft_x",
                                           "fft_y",     "fft_z_scale", "fft_yinv", "fft_xinv",
                                           "gather",    "real",       "gather_grad", "real_grad"};

struct Timer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int stage; hipEvent_t a, b; };
    std::vector<Rec> recs;
    hipEvent_t get() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    ~Timer() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

struct TimedStage {
    Timer& t;
    int stage;
    hipStream_t st;
    hipEvent_t a = nullptr;
    TimedStage(Timer& t_, int s, hipStream_t st_) : t(t_), stage(s), st(st_) {
        if (t.on && (a = t.get())) (void)hipEventRecord(a, st);
    }
    ~TimedStage() {
        if (!a) return;
        hipEvent_t b = t.get();
        if (!b) return;
        (void)hipEventRecord(b, st);
        t.recs.push_back({stage, a, b});
    }
};

}  // namespace

namespace fse {
void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}
}  // namespace fse

struct fse_plan {
    fse_kernel_t kernel;
    fse_dtype_t dtype;
    fse_params_t prm;
    fse_geometry_t geo;
    int batch;
    int64_t nmax;
    int64_t n = 0;
    hipStream_t stream;
    int c_in;
    GridGeo gg;  // the spreading and quadrature grid
    GridGeo gf;  // the transforms' grid (gg, except for periodic sums: the M^3 period)
    CellGeo cg;
    bool periodic = false;
    bool solver = false;  // fse_freespace_solve: sigma is the plain truncated kernel transform
    int family = 0;       // 0 biharmonic (eq. BhatR), 1 harmonic (eq. HhatR)
    int pshift = 0;  // periodic: index of period node 0 in the extended grid (ceil(P/2) - 1)
    void* gext = nullptr;  // periodic: spread grid and quadrature field on the extended grid
    FftGeo fg;
    size_t bytes = 0;
    bool forward_valid = false;
    std::vector<void*> allocs;
    Timer timer;

    // points
    int *key_s, *key_r, *idx, *key_tmp, *bpack, *perm_s, *bpack_s, *perm_r, *inv_r;
    void* sort_tmp;
    size_t sort_bytes = 0;
    int bits_s = 1, bits_r = 1;
    int64_t ntiles_max = 0;  // tiles at the smallest bin side a tuning may set
    int real_waves = 4;      // tuning: most waves per real-space work item
    void *coff, *coff_s, *x_r;
    int *cnt_s, *start_s, *cnt_r, *start_r, *work_r, *scan_tmp, *flag;
    int real_S = 256;
    int64_t ntiles3, ncells3;
    // separate targets (fse_set_targets): binned like the points, own buffers
    struct Targets {
        int64_t cap = 0, n = 0;
        int *key_s, *key_r, *idx, *key_tmp, *bpack, *perm_s, *bpack_s, *perm_r, *inv_r;
        void *coff, *coff_s, *x_r, *sort_tmp;
        size_t sort_bytes = 0;
        int *cnt_s, *start_s, *cnt_r, *start_r, *work_r;
        int real_S = 64;
        std::vector<void*> allocs;
    } tg;
    // sources
    void *src_s, *src_ra, *src_rb, *adj_s, *adj_r;
    void* tadj;  // stresslet adjoint: quadrature of its transpose field (2 batch, n, 3)
    // grids
    void *grid, *A, *B, *phi, *phi_w;
    double* sig64;
    void* sig;
    void* tw;
    int *rev, *revinv;

    // Workspace source: hipMalloc (a plan), or carved in 256-byte steps from a
    // caller-owned device arena (the no-allocation entry point); `dry` counts the
    // carved bytes without touching memory.
    char* arena = nullptr;
    size_t arena_cap = 0;
    bool dry = false;

    template <typename X> fse_status_t alloc(X** p, size_t count) {
        void* q = nullptr;
        size_t b = count * sizeof(X);
        if (b == 0) b = 16;
        if (arena || dry) {
            b = (b + 255) & ~(size_t)255;
            if (dry) {
                *p = nullptr;
                bytes += b;
                return FSE_OK;
            }
            if (bytes + b > arena_cap) {
                set_err("workspace of %zu bytes exceeds the %zu-byte arena", bytes + b, arena_cap);
                return FSE_EINVAL;
            }
            *p = (X*)(arena + bytes);
            bytes += b;
            return FSE_OK;
        }
        hipError_t e = hipMalloc(&q, b);
        if (e != hipSuccess) {
            set_err("hipMalloc(%zu bytes) failed: %s", b, hipGetErrorString(e));
            return FSE_ENOMEM;
        }
        allocs.push_back(q);
        bytes += b;
        *p = (X*)q;
        return FSE_OK;
    }
    void free_targets() {
        for (void* q : tg.allocs) (void)hipFree(q);
        tg.allocs.clear();
        tg.cap = tg.n = 0;
    }
    ~fse_plan() {
        free_targets();
        for (void* q : allocs) (void)hipFree(q);
    }
};

namespace {

template <typename T> PointsDev<T> points(const fse_plan* p) {
    PointsDev<T> d;
    d.n = p->n;
    d.perm_s = p->perm_s;
    d.bpack_s = p->bpack_s;
    d.coff_s = (const T*)p->coff_s;
    d.tile_start = p->start_s;
    d.perm_r = p->perm_r;
    d.x_r = (const T*)p->x_r;
    d.cell_start = p->start_r;
    d.inv_r = p->inv_r;
    d.work_start = p->work_r;
    d.real_S = p->real_S;
    d.t_n = d.n;
    d.t_x_r = d.x_r;
    d.t_cell_start = d.cell_start;
    d.t_perm_r = d.perm_r;
    d.t_work_start = d.work_start;
    d.t_real_S = d.real_S;
    return d;
}

#define TRY(x)                        \
    do {                              \
        fse_status_t s_ = (x);        \
        if (s_ != FSE_OK) return s_;  \
    } while (0)

template <typename T> fse_status_t allocate(fse_plan* p) {
    const int64_t nm = p->nmax, B = p->batch;
    const int64_t Mt = p->geo.Mt, n = p->geo.n_fft, Mp = Mt + 1;
    const int64_t M3 = Mt * Mt * Mt;
    using V = C2<T>;
    TRY(p->alloc(&p->key_s, nm));
    TRY(p->alloc(&p->key_r, nm));
    TRY(p->alloc(&p->idx, nm));
    TRY(p->alloc(&p->key_tmp, nm));
    TRY(p->alloc(&p->bpack, nm));
    TRY(p->alloc(&p->perm_s, nm));
    TRY(p->alloc(&p->bpack_s, nm));
    TRY(p->alloc(&p->perm_r, nm));
    TRY(p->alloc(&p->inv_r, nm));
    TRY(p->alloc((T**)&p->coff, 3 * nm));
    TRY(p->alloc((T**)&p->coff_s, 3 * nm));
    TRY(p->alloc((T**)&p->x_r, 3 * nm));
    p->ntiles3 = (int64_t)p->gg.nt * p->gg.nt * p->gg.nt;
    {
        // the most bins any bin side this plan may take gives: the smallest a tuning
        // may set, or the default where the LDS bound makes that smaller (large P)
        const int side = std::min(MIN_BIN_SIDE, p->gg.TS);
        const int64_t ntm = (p->gg.Mt + side - 1) / side;
        p->ntiles_max = ntm * ntm * ntm;
    }
    p->ncells3 = (int64_t)p->cg.ncell * p->cg.ncell * p->cg.ncell;
    TRY(p->alloc(&p->cnt_s, p->ntiles_max + 1));
    TRY(p->alloc(&p->start_s, p->ntiles_max + 1));
    TRY(p->alloc(&p->cnt_r, p->ncells3 + 1));
    TRY(p->alloc(&p->start_r, p->ncells3 + 1));
    TRY(p->alloc(&p->work_r, p->ncells3 + 1));
    const size_t st = scan_tmp_ints(p->ntiles_max + 1) > scan_tmp_ints(p->ncells3 + 1)
                          ? scan_tmp_ints(p->ntiles_max + 1) : scan_tmp_ints(p->ncells3 + 1);
    TRY(p->alloc(&p->scan_tmp, st));
    p->bits_s = key_bits(p->ntiles3);
    p->bits_r = key_bits(p->ncells3);
    {
        const size_t b1 = sort_tmp_bytes(nm, key_bits(p->ntiles_max)), b2 = sort_tmp_bytes(nm, p->bits_r);
        if (b1 == 0 || b2 == 0) { set_err("sort workspace query failed"); return FSE_EHIP; }
        p->sort_bytes = b1 > b2 ? b1 : b2;
        TRY(p->alloc((char**)&p->sort_tmp, p->sort_bytes));
    }
    TRY(p->alloc(&p->flag, 1));
    TRY(p->alloc((T**)&p->src_s, B * nm * p->c_in));
    TRY(p->alloc((T**)&p->src_ra, B * nm * 3));
    TRY(p->alloc((T**)&p->src_rb, p->kernel == FSE_STRESSLET ? B * nm * 3 : 1));
    TRY(p->alloc((T**)&p->adj_s, B * nm * 3));
    TRY(p->alloc((T**)&p->adj_r, B * nm * 3));
    TRY(p->alloc((T**)&p->grid, B * p->c_in * M3));
    if (p->periodic) {
        const int64_t Me = p->gg.Mt;
        TRY(p->alloc((T**)&p->gext, B * 3 * Me * Me * Me));
    }
    TRY(p->alloc((V**)&p->A, B * p->c_in * Mp * Mt * (size_t)p->fg.sy));
    TRY(p->alloc((V**)&p->B, B * p->c_in * Mp * n * (size_t)p->fg.sz));
    // the stresslet's adjoint field has 6 components (the symmetric D_lm)
    TRY(p->alloc((T**)&p->phi, B * (p->kernel == FSE_STRESSLET ? 6 : 3) * M3));
    TRY(p->alloc((T**)&p->tadj, p->kernel == FSE_STRESSLET ? 6 * B * nm : 1));
    TRY(p->alloc((T**)&p->phi_w, p->kernel == FSE_STRESSLET ? 1 : B * 3 * M3));
    TRY(p->alloc(&p->sig64, Mp * Mp * Mp));
    TRY(p->alloc((T**)&p->sig, Mp * Mp * Mp));
    TRY(p->alloc((T**)&p->tw, 2 * n));
    TRY(p->alloc(&p->rev, n));
    TRY(p->alloc(&p->revinv, n));
    return FSE_OK;
}

template <typename T> fse_status_t upload_fft_tables(fse_plan* p) {
    const int n = p->geo.n_fft;
    std::vector<T> tw(2 * (size_t)n);
    for (int e = 0; e < n; ++e) {
        const double a = 2.0 * PI * (double)e / (double)n;
        tw[2 * e] = (T)cos(a);
        tw[2 * e + 1] = (T)(-sin(a));
    }
    std::vector<int> rev, revinv(n);
    digit_reverse(p->fg.rad, p->fg.ns, n, rev);
    for (int q = 0; q < n; ++q) revinv[rev[q]] = q;
    HIPCHK(hipMemcpyAsync(p->tw, tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipMemcpyAsync(p->rev, rev.data(), n * sizeof(int), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipMemcpyAsync(p->revinv, revinv.data(), n * sizeof(int), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return FSE_OK;
}

// Section 4.3 precompute, FP64, then fold in the scalar factors.  Its four
// temporaries come from hipMalloc (freed at the end), or from the plan's arena.
// Process-wide cache of the mollified transform Bt (the FP64 octant, Section 4.3),
// one entry per (device, Mt, kernel family).  Bt depends on the grid spacing h only
// through a factor: the truncated transform is homogeneous in (k, R), k = 2 pi kbar /
// (Mg h) and R = sqrt(3) Mt h, so Bt(h) = (h / h0)^p Bt(h0) with p = 4 for the
// biharmonic kernel (eq. BhatR) and 2 for the harmonic one (eq. HhatR).  Entries
// are written once, never changed or freed (device memory held until the process
// ends), up to BT_CACHE_MAX bytes in all; plans that find their entry skip the
// fill and the six contractions.  The no-allocation entry point reads entries but
// adds none (an entry costs an allocation).
struct BtEntry {
    int dev, Mt, family;
    double h0;
    const double* buf;
};
constexpr size_t BT_CACHE_MAX = (size_t)2 << 30;
std::mutex bt_mu;
std::vector<BtEntry> bt_cache;
size_t bt_bytes = 0;
int64_t bt_hits = 0, bt_misses = 0;

template <typename T> fse_status_t precompute(fse_plan* p) {
    if (p->periodic) {
        if (p->dry) return FSE_OK;
        const double nn = (double)p->geo.n_fft;
        const double norm = 8.0 * pow(p->geo.alpha / PI, 3.0) * pow(p->geo.h, 3.0) / (nn * nn * nn);
        launch_pre_periodic<T>(p->geo.Mt, PI / p->geo.Lt, p->prm.xi, p->geo.eta, norm, p->sig64, (T*)p->sig,
                               p->stream);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) {
            set_err("precompute failed: %s", hipGetErrorString(e));
            return FSE_EHIP;
        }
        return FSE_OK;
    }
    const int Mt = p->geo.Mt, Mg = p->geo.Mg, Mp = Mt + 1, H = Mg / 2 + 1;
    const int64_t big = (int64_t)H * H * H > (int64_t)Mp * H * H ? (int64_t)H * H * H : (int64_t)Mp * H * H;
    double *t0 = nullptr, *t1 = nullptr, *c1 = nullptr, *c2 = nullptr;
    const bool carve = p->arena || p->dry;
    const double a = p->geo.alpha;
    const double nn = (double)p->geo.n_fft;
    // the Gaussian normalisations (alpha/pi)^{3/2} of spreading and quadrature, the
    // quadrature weight h^3 and the inverse transform's 1/n^3 (the transform Bt
    // already carries the convolution's h^3: the solver's plain convolution is 1/n^3)
    const double norm = p->solver ? 1.0 / (nn * nn * nn) : pow(a / PI, 3.0) * pow(p->geo.h, 3.0) / (nn * nn * nn);
    const int fin_kernel = p->solver ? KSCALAR : (int)p->kernel;
    const double hpow = p->family == 0 ? 4.0 : 2.0;  // Bt's degree of homogeneity in h
    int dev = -1;
    if (!p->dry) {
        // plans look up and add entries; the no-allocation entry point only looks up
        HIPCHK(hipGetDevice(&dev));
        const double* hit = nullptr;
        double h0 = 0.0;
        {
            std::lock_guard<std::mutex> lk(bt_mu);
            for (const BtEntry& e : bt_cache)
                if (e.dev == dev && e.Mt == Mt && e.family == p->family) {
                    hit = e.buf;
                    h0 = e.h0;
                }
            if (hit) ++bt_hits; else ++bt_misses;
        }
        if (hit) {
            launch_pre_finalize<T>(hit, Mt, PI / p->geo.Lt, p->prm.xi, p->geo.eta, fin_kernel,
                                   norm * pow(p->geo.h / h0, hpow), p->sig64, (T*)p->sig, p->stream);
            hipError_t e = hipGetLastError();
            if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
            if (e != hipSuccess) {
                set_err("precompute failed: %s", hipGetErrorString(e));
                return FSE_EHIP;
            }
            return FSE_OK;
        }
    }
    auto cleanup = [&]() {
        if (carve) return;
        if (t0) (void)hipFree(t0);
        if (t1) (void)hipFree(t1);
        if (c1) (void)hipFree(c1);
        if (c2) (void)hipFree(c2);
    };
    if (carve) {
        TRY(p->alloc(&t0, big));
        TRY(p->alloc(&t1, big));
        TRY(p->alloc(&c1, (size_t)Mp * H));
        TRY(p->alloc(&c2, (size_t)Mp * Mp));
        if (p->dry) return FSE_OK;
    } else if (hipMalloc(&t0, big * sizeof(double)) != hipSuccess ||
               hipMalloc(&t1, big * sizeof(double)) != hipSuccess ||
               hipMalloc(&c1, (size_t)Mp * H * sizeof(double)) != hipSuccess ||
               hipMalloc(&c2, (size_t)Mp * Mp * sizeof(double)) != hipSuccess) {
        cleanup();
        set_err("precompute: out of device memory");
        return FSE_ENOMEM;
    }
    // C1[j][k] = w_k cos(2 pi j k / Mg), k in [0, Mg/2]: inverse transform on Mg
    std::vector<double> h1((size_t)Mp * H), h2((size_t)Mp * Mp);
    for (int j = 0; j < Mp; ++j)
        for (int k = 0; k < H; ++k) {
            const double w = (k == 0 || k == Mg / 2) ? 1.0 : 2.0;
            const long long e = ((long long)j * k) % Mg;
            h1[(size_t)j * H + k] = w * cos(2.0 * PI * (double)e / (double)Mg);
        }
    // C2[k][j] = w_j cos(pi k j / Mt), j in [0, Mt]: forward transform on 2 Mt
    for (int k = 0; k < Mp; ++k)
        for (int j = 0; j < Mp; ++j) {
            const double w = (j == 0 || j == Mt) ? 1.0 : 2.0;
            const long long e = ((long long)k * j) % (2 * Mt);
            h2[(size_t)k * Mp + j] = w * cos(PI * (double)e / (double)Mt);
        }
    hipStream_t st = p->stream;
    fse_status_t rc = FSE_OK;
    if (hipMemcpyAsync(c1, h1.data(), h1.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(c2, h2.data(), h2.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess) {
        cleanup();
        set_err("precompute: copy failed");
        return FSE_EHIP;
    }
    launch_pre_fill(t0, Mg, p->geo.h, p->geo.R, p->family, st);
    launch_pre_contract(t0, t1, c1, Mp, H, (int64_t)H * H, st);    // [j3][k1][k2]
    launch_pre_contract(t1, t0, c1, Mp, H, (int64_t)Mp * H, st);   // [j2][j3][k1]
    launch_pre_contract(t0, t1, c1, Mp, H, (int64_t)Mp * Mp, st);  // [j1][j2][j3]: G octant
    launch_pre_contract(t1, t0, c2, Mp, Mp, (int64_t)Mp * Mp, st);
    launch_pre_contract(t0, t1, c2, Mp, Mp, (int64_t)Mp * Mp, st);
    launch_pre_contract(t1, t0, c2, Mp, Mp, (int64_t)Mp * Mp, st); // [k1][k2][k3]: mollified transform
    // a copy of Bt for the cache, when it has room (published after the stream sync)
    const size_t bt_size = (size_t)Mp * Mp * Mp * sizeof(double);
    double* keep = nullptr;
    if (!carve) {
        bool room;
        {
            std::lock_guard<std::mutex> lk(bt_mu);
            room = bt_bytes + bt_size <= BT_CACHE_MAX;
        }
        if (room && hipMalloc(&keep, bt_size) == hipSuccess) {
            if (hipMemcpyAsync(keep, t0, bt_size, hipMemcpyDeviceToDevice, st) != hipSuccess) {
                (void)hipStreamSynchronize(st);
                (void)hipFree(keep);
                keep = nullptr;
            }
        } else {
            (void)hipGetLastError();  // a failed cache allocation is not an error of the plan
            keep = nullptr;
        }
    }
    launch_pre_finalize<T>(t0, Mt, PI / p->geo.Lt, p->prm.xi, p->geo.eta, fin_kernel, norm, p->sig64, (T*)p->sig,
                           st);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_err("precompute failed: %s", hipGetErrorString(e));
        rc = FSE_EHIP;
    }
    if (keep) {
        bool stored = false;
        if (rc == FSE_OK) {
            std::lock_guard<std::mutex> lk(bt_mu);
            bool dup = false;
            for (const BtEntry& en : bt_cache) dup = dup || (en.dev == dev && en.Mt == Mt && en.family == p->family);
            if (!dup && bt_bytes + bt_size <= BT_CACHE_MAX) {
                bt_cache.push_back(BtEntry{dev, Mt, p->family, p->geo.h, keep});
                bt_bytes += bt_size;
                stored = true;
            }
        }
        if (!stored) (void)hipFree(keep);
    }
    cleanup();
    return rc;
}

template <typename T> fse_status_t plan_init(fse_plan* p) {
    TRY(allocate<T>(p));
    TRY(upload_fft_tables<T>(p));
    TRY(precompute<T>(p));
    return FSE_OK;
}

// Device bytes plan_init would take (workspace plus the precompute's temporaries).
template <typename T> fse_status_t plan_bytes(fse_plan* p, size_t* out) {
    p->dry = true;
    p->bytes = 0;
    fse_status_t rc = allocate<T>(p);
    if (rc == FSE_OK) rc = precompute<T>(p);
    p->dry = false;
    *out = p->bytes;
    p->bytes = 0;
    return rc;
}

template <typename T> fse_status_t set_points_t(fse_plan* p, int64_t n, const T* x, int validate) {
    hipStream_t st = p->stream;
    {
        TimedStage ts(p->timer, ST_BIN, st);
        launch_fill_i32(p->cnt_s, p->ntiles3 + 1, 0, st);
        launch_fill_i32(p->cnt_r, p->ncells3 + 1, 0, st);
        launch_fill_i32(p->flag, 1, 0, st);
        launch_bin<T>(x, n, p->gg, p->cg, p->key_s, p->key_r, p->idx, p->bpack, (T*)p->coff,
                      p->flag, st);
        // stable sorts by tile and by cell: perm_s and perm_r list the point indices in order
        if (sort_tmp_bytes(n, p->bits_s) > p->sort_bytes || sort_tmp_bytes(n, p->bits_r) > p->sort_bytes) {
            set_err("sort workspace too small for n=%lld", (long long)n);
            return FSE_EINVAL;
        }
        // (the counts per tile and cell come from the sorted keys)
        HIPCHK(launch_sort_pairs(p->sort_tmp, p->sort_bytes, p->key_s, p->key_tmp, p->idx, p->perm_s, n, p->bits_s, st));
        launch_run_counts(p->key_tmp, n, p->cnt_s, st);
        HIPCHK(launch_sort_pairs(p->sort_tmp, p->sort_bytes, p->key_r, p->key_tmp, p->idx, p->perm_r, n, p->bits_r, st));
        launch_run_counts(p->key_tmp, n, p->cnt_r, st);
        launch_scan_exclusive(p->cnt_s, p->start_s, p->ntiles3 + 1, p->scan_tmp, st);
        launch_scan_exclusive(p->cnt_r, p->start_r, p->ncells3 + 1, p->scan_tmp, st);
        // real-space work items: slices of up to real_S targets of one cell
        p->real_S = (int)real_threads(n, p->ncells3, p->real_waves);
        launch_cell_slices(p->cnt_r, p->ncells3, p->real_S, st);
        launch_scan_exclusive(p->cnt_r, p->work_r, p->ncells3 + 1, p->scan_tmp, st);
        launch_scatter<T>(x, n, p->perm_s, p->perm_r, p->bpack, (const T*)p->coff, p->bpack_s, (T*)p->coff_s,
                          (T*)p->x_r, p->inv_r, st);
    }
    LAUNCHCHK();
    p->n = n;
    p->forward_valid = false;
    if (validate) {
        int flag = 0;
        HIPCHK(hipMemcpyAsync(&flag, p->flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (flag) {
            set_err("a point lies outside [box_lo, box_lo + L)^3 or is not finite");
            return FSE_ERANGE;
        }
    }
    return FSE_OK;
}

template <typename X> fse_status_t talloc(fse_plan* p, X** q, size_t count) {
    void* v = nullptr;
    const size_t b = count * sizeof(X) > 0 ? count * sizeof(X) : 16;
    hipError_t e = hipMalloc(&v, b);
    if (e != hipSuccess) {
        set_err("hipMalloc(%zu bytes) for targets failed: %s", b, hipGetErrorString(e));
        return FSE_ENOMEM;
    }
    p->tg.allocs.push_back(v);
    *q = (X*)v;
    return FSE_OK;
}

// (Re)allocate the target buffers for nt targets (plan dtype T).
template <typename T> fse_status_t reserve_targets(fse_plan* p, int64_t nt) {
    auto& t = p->tg;
    if (t.cap >= nt) return FSE_OK;
    HIPCHK(hipStreamSynchronize(p->stream));  // earlier work may still read the old buffers
    p->free_targets();
    TRY(talloc(p, &t.key_s, nt));
    TRY(talloc(p, &t.key_r, nt));
    TRY(talloc(p, &t.idx, nt));
    TRY(talloc(p, &t.key_tmp, nt));
    TRY(talloc(p, &t.bpack, nt));
    TRY(talloc(p, &t.perm_s, nt));
    TRY(talloc(p, &t.bpack_s, nt));
    TRY(talloc(p, &t.perm_r, nt));
    TRY(talloc(p, &t.inv_r, nt));
    TRY(talloc(p, (T**)&t.coff, 3 * nt));
    TRY(talloc(p, (T**)&t.coff_s, 3 * nt));
    TRY(talloc(p, (T**)&t.x_r, 3 * nt));
    TRY(talloc(p, &t.cnt_s, p->ntiles_max + 1));
    TRY(talloc(p, &t.start_s, p->ntiles_max + 1));
    TRY(talloc(p, &t.cnt_r, p->ncells3 + 1));
    TRY(talloc(p, &t.start_r, p->ncells3 + 1));
    TRY(talloc(p, &t.work_r, p->ncells3 + 1));
    const size_t b1 = sort_tmp_bytes(nt, key_bits(p->ntiles_max)), b2 = sort_tmp_bytes(nt, p->bits_r);
    if (b1 == 0 || b2 == 0) { set_err("sort workspace query failed"); return FSE_EHIP; }
    t.sort_bytes = b1 > b2 ? b1 : b2;
    TRY(talloc(p, (char**)&t.sort_tmp, t.sort_bytes));
    t.cap = nt;
    return FSE_OK;
}

// Bin the targets exactly as the points (window starts for the quadrature,
// cells for the real-space pass), into the target buffers.
template <typename T> fse_status_t set_targets_t(fse_plan* p, int64_t nt, const T* y, int validate) {
    TRY(reserve_targets<T>(p, nt));
    auto& t = p->tg;
    hipStream_t st = p->stream;
    {
        TimedStage ts(p->timer, ST_BIN, st);
        launch_fill_i32(t.cnt_s, p->ntiles3 + 1, 0, st);
        launch_fill_i32(t.cnt_r, p->ncells3 + 1, 0, st);
        launch_fill_i32(p->flag, 1, 0, st);
        launch_bin<T>(y, nt, p->gg, p->cg, t.key_s, t.key_r, t.idx, t.bpack, (T*)t.coff, p->flag,
                      st);
        HIPCHK(launch_sort_pairs(t.sort_tmp, t.sort_bytes, t.key_s, t.key_tmp, t.idx, t.perm_s, nt, p->bits_s, st));
        launch_run_counts(t.key_tmp, nt, t.cnt_s, st);
        HIPCHK(launch_sort_pairs(t.sort_tmp, t.sort_bytes, t.key_r, t.key_tmp, t.idx, t.perm_r, nt, p->bits_r, st));
        launch_run_counts(t.key_tmp, nt, t.cnt_r, st);
        launch_scan_exclusive(t.cnt_s, t.start_s, p->ntiles3 + 1, p->scan_tmp, st);
        launch_scan_exclusive(t.cnt_r, t.start_r, p->ncells3 + 1, p->scan_tmp, st);
        t.real_S = (int)real_threads(nt, p->ncells3, p->real_waves);
        launch_cell_slices(t.cnt_r, p->ncells3, t.real_S, st);
        launch_scan_exclusive(t.cnt_r, t.work_r, p->ncells3 + 1, p->scan_tmp, st);
        launch_scatter<T>(y, nt, t.perm_s, t.perm_r, t.bpack, (const T*)t.coff, t.bpack_s, (T*)t.coff_s,
                          (T*)t.x_r, t.inv_r, st);
    }
    LAUNCHCHK();
    t.n = nt;
    if (validate) {
        int flag = 0;
        HIPCHK(hipMemcpyAsync(&flag, p->flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (flag) {
            set_err("a target lies outside [box_lo, box_lo + L)^3 or is not finite");
            return FSE_ERANGE;
        }
    }
    return FSE_OK;
}

// The targets as the points of a quadrature (their spread-order arrays).
template <typename T> PointsDev<T> target_points(const fse_plan* p) {
    const auto& t = p->tg;
    PointsDev<T> d = points<T>(p);
    d.n = t.n;
    d.perm_s = t.perm_s;
    d.bpack_s = t.bpack_s;
    d.coff_s = (const T*)t.coff_s;
    d.tile_start = t.start_s;
    return d;
}

// The points as real-space sources and the targets as real-space targets.
template <typename T> PointsDev<T> source_target_points(const fse_plan* p) {
    const auto& t = p->tg;
    PointsDev<T> d = points<T>(p);
    d.t_n = t.n;
    d.t_x_r = (const T*)t.x_r;
    d.t_cell_start = t.start_r;
    d.t_perm_r = t.perm_r;
    d.t_work_start = t.work_r;
    d.t_real_S = t.real_S;
    return d;
}

// spread -> FFT -> scale -> IFFT into `field` (periodic: spread onto the
// extended grid and fold it onto the period first)
template <typename T> void fft_chain(fse_plan* p, const T* grid, T* field);

template <typename T> void fourier_chain(fse_plan* p, const T* src_s, T* field) {
    hipStream_t st = p->stream;
    PointsDev<T> pd = points<T>(p);
    Timer& tm = p->timer;
    if (p->periodic) {
        TimedStage ts(tm, ST_SPREAD, st);
        launch_spread<T>(p->gg, pd, src_s, p->c_in, p->batch, (T*)p->gext, st);
        launch_fold<T>((const T*)p->gext, p->gg.Mt, p->gf.Mt, p->pshift, p->batch * p->c_in, (T*)p->grid, st);
    } else {
        TimedStage ts(tm, ST_SPREAD, st);
        launch_spread<T>(p->gg, pd, src_s, p->c_in, p->batch, (T*)p->grid, st);
    }
    fft_chain<T>(p, (const T*)p->grid, field);
}

// Steps 2-4 of Section 5.2 on a spread grid: forward transforms, the scaling, the
// inverse transforms into field (which may be the grid itself: the first pass has
// read all of it before the last one writes).
template <typename T> void fft_chain(fse_plan* p, const T* grid, T* field) {
    hipStream_t st = p->stream;
    Timer& tm = p->timer;
    { TimedStage ts(tm, ST_FFTX, st);
      launch_fft_forward<T>(p->fg, p->gf, grid, p->A, p->B, p->batch * p->c_in, (const T*)p->tw, p->rev,
                            p->revinv, st, 1); }
    { TimedStage ts(tm, ST_FFTY, st);
      launch_fft_forward<T>(p->fg, p->gf, grid, p->A, p->B, p->batch * p->c_in, (const T*)p->tw, p->rev,
                            p->revinv, st, 2); }
    { TimedStage ts(tm, ST_FFTZ, st);
      launch_fft_zscale<T>(p->fg, p->gf, (int)p->kernel, p->B, p->c_in, p->batch, (const T*)p->sig,
                           PI / p->geo.Lt, (const T*)p->tw, p->rev, p->revinv, st); }
    { TimedStage ts(tm, ST_FFTYI, st);
      launch_fft_inverse<T>(p->fg, p->gf, p->B, p->A, field, p->c_in, p->batch, (const T*)p->tw, p->rev,
                            p->revinv, st, 1); }
    { TimedStage ts(tm, ST_FFTXI, st);
      launch_fft_inverse<T>(p->fg, p->gf, p->B, p->A, field, p->c_in, p->batch, (const T*)p->tw, p->rev,
                            p->revinv, st, 2); }
}

// The field the quadrature reads: `field` itself, or for periodic sums its
// copy unfolded onto the extended grid.
template <typename T> const T* quad_field(fse_plan* p, const T* field) {
    if (!p->periodic) return field;
    launch_unfold<T>(field, p->gf.Mt, p->gg.Mt, p->pshift, p->batch * 3, (T*)p->gext, p->stream);
    return (const T*)p->gext;
}

double self_coef(const fse_plan* p) {
    return p->kernel == FSE_STOKESLET ? -4.0 * p->prm.xi / sqrt(PI) : 0.0;
}

template <typename T>
fse_status_t eval_t(fse_plan* p, const T* a, const T* b, T* u_real, T* u_four, bool combined) {
    hipStream_t st = p->stream;
    const int64_t n = p->n;
    PointsDev<T> pd = points<T>(p);
    Timer& tm = p->timer;
    {
        TimedStage ts(tm, ST_PERMUTE, st);
        launch_permute_sources<T>((int)p->kernel, a, b, n, p->batch, p->perm_s, (T*)p->src_s, st);
        launch_permute3<T>(a, n, p->batch, p->perm_r, (T*)p->src_ra, st);
        if (p->kernel == FSE_STRESSLET) launch_permute3<T>(b, n, p->batch, p->perm_r, (T*)p->src_rb, st);
    }
    fourier_chain<T>(p, (const T*)p->src_s, (T*)p->phi);
    p->forward_valid = true;
    if (combined) {
        { TimedStage ts(tm, ST_GATHER, st);
          launch_gather<T>(p->gg, pd, quad_field<T>(p, (const T*)p->phi), p->batch, u_real, st); }
        { TimedStage ts(tm, ST_REAL, st);
          launch_real<T>((int)p->kernel, p->cg, pd, (const T*)p->src_ra, (const T*)p->src_rb, p->batch,
                         p->prm.xi, self_coef(p), u_real, 1, st); }
    } else {
        if (u_four) {
            TimedStage ts(tm, ST_GATHER, st);
            launch_gather<T>(p->gg, pd, quad_field<T>(p, (const T*)p->phi), p->batch, u_four, st);
        }
        if (u_real) {
            TimedStage ts(tm, ST_REAL, st);
            launch_real<T>((int)p->kernel, p->cg, pd, (const T*)p->src_ra, (const T*)p->src_rb, p->batch,
                           p->prm.xi, self_coef(p), u_real, 0, st);
        }
    }
    LAUNCHCHK();
    return FSE_OK;
}

// u at the separate targets: u^F by quadrature at the targets, plus u^R over
// the sources within r_c of each target (no self term: a target is no source).
template <typename T> fse_status_t eval_targets_t(fse_plan* p, const T* a, const T* b, T* u_real, T* u_four) {
    hipStream_t st = p->stream;
    const int64_t n = p->n;
    Timer& tm = p->timer;
    {
        TimedStage ts(tm, ST_PERMUTE, st);
        launch_permute_sources<T>((int)p->kernel, a, b, n, p->batch, p->perm_s, (T*)p->src_s, st);
        launch_permute3<T>(a, n, p->batch, p->perm_r, (T*)p->src_ra, st);
        if (p->kernel == FSE_STRESSLET) launch_permute3<T>(b, n, p->batch, p->perm_r, (T*)p->src_rb, st);
    }
    fourier_chain<T>(p, (const T*)p->src_s, (T*)p->phi);
    p->forward_valid = true;
    const bool combined = u_four == nullptr;
    T* uf = combined ? u_real : u_four;
    if (uf) {
        TimedStage ts(tm, ST_GATHER, st);
        launch_gather<T>(p->gg, target_points<T>(p), (const T*)p->phi, p->batch, uf, st);
    }
    if (u_real) {
        TimedStage ts(tm, ST_REAL, st);
        launch_real<T>((int)p->kernel, p->cg, source_target_points<T>(p), (const T*)p->src_ra,
                       (const T*)p->src_rb, p->batch, p->prm.xi, 0.0, u_real, combined ? 1 : 0, st);
    }
    LAUNCHCHK();
    return FSE_OK;
}

template <typename T>
fse_status_t adjoint_t(fse_plan* p, const T* f, const T* w, T* dsrc, T* dx, int recompute) {
    hipStream_t st = p->stream;
    const int64_t n = p->n;
    PointsDev<T> pd = points<T>(p);
    Timer& tm = p->timer;
    // f in spread and real-space order (also needed when the forward field is reused)
    {
        TimedStage ts(tm, ST_PERMUTE, st);
        launch_permute_sources<T>((int)p->kernel, f, nullptr, n, p->batch, p->perm_s, (T*)p->src_s, st);
        launch_permute3<T>(f, n, p->batch, p->perm_r, (T*)p->src_ra, st);
    }
    if (recompute || !p->forward_valid) {
        fourier_chain<T>(p, (const T*)p->src_s, (T*)p->phi);
        p->forward_valid = true;
    }
    {
        TimedStage ts(tm, ST_PERMUTE, st);
        launch_permute3<T>(w, n, p->batch, p->perm_s, (T*)p->adj_s, st);
        launch_permute3<T>(w, n, p->batch, p->perm_r, (T*)p->adj_r, st);
    }
    fourier_chain<T>(p, (const T*)p->adj_s, (T*)p->phi_w);
    { TimedStage ts(tm, ST_GGRAD, st);
      launch_gather_grad<T>(p->gg, pd, (const T*)p->phi, (const T*)p->phi_w, (const T*)p->src_s,
                            (const T*)p->adj_s, p->batch, dsrc, dx, st); }
    if (dx) {
        // gradient and (when requested) the real-space part of K w in one pass over the pairs
        TimedStage ts(tm, ST_RGRAD, st);
        launch_real_grad<T>((int)p->kernel, p->cg, pd, (const T*)p->src_ra, (const T*)p->adj_r, p->batch,
                            p->prm.xi, self_coef(p), dx, dsrc, st);
    } else if (dsrc) {
        TimedStage ts(tm, ST_REAL, st);
        launch_real<T>((int)p->kernel, p->cg, pd, (const T*)p->adj_r, nullptr, p->batch, p->prm.xi,
                       self_coef(p), dsrc, 1, st);
    }
    LAUNCHCHK();
    return FSE_OK;
}

// Forward sum and adjoint together, for L = sum_m w_m . u(x_m) with w known: f and
// w spread in one pass (six components, into the forward grid and phi_w), the two
// transform chains, the forward quadrature with the first gradient term in one
// sweep and the second with K w's quadrature, then (one batch member) one pass over
// the pairs for u^R + self, the real part of K w and dL/dx.
template <typename T>
fse_status_t eval_with_adjoint_t(fse_plan* p, const T* f, const T* w, T* u, T* dsrc, T* dx) {
    hipStream_t st = p->stream;
    const int64_t n = p->n;
    const int B = p->batch;
    PointsDev<T> pd = points<T>(p);
    Timer& tm = p->timer;
    {
        TimedStage ts(tm, ST_PERMUTE, st);
        launch_permute_sources<T>((int)p->kernel, f, nullptr, n, B, p->perm_s, (T*)p->src_s, st);
        launch_permute3<T>(f, n, B, p->perm_r, (T*)p->src_ra, st);
        launch_permute3<T>(w, n, B, p->perm_s, (T*)p->adj_s, st);
        launch_permute3<T>(w, n, B, p->perm_r, (T*)p->adj_r, st);
    }
    { TimedStage ts(tm, ST_SPREAD, st);
      launch_spread<T>(p->gg, pd, (const T*)p->src_s, 6, B, (T*)p->grid, st, (const T*)p->adj_s, (T*)p->phi_w); }
    fft_chain<T>(p, (const T*)p->grid, (T*)p->phi);
    fft_chain<T>(p, (const T*)p->phi_w, (T*)p->phi_w);
    p->forward_valid = true;
    { TimedStage ts(tm, ST_GGRAD, st);
      launch_gather_fused<T>(p->gg, pd, (const T*)p->phi, (const T*)p->phi_w, (const T*)p->src_s,
                             (const T*)p->adj_s, B, u, dsrc, dx, st); }
    {
        TimedStage ts(tm, ST_RGRAD, st);
        if (B > 1)
            launch_real<T>((int)p->kernel, p->cg, pd, (const T*)p->src_ra, nullptr, B, p->prm.xi, self_coef(p), u,
                           1, st);
        launch_real_grad<T>((int)p->kernel, p->cg, pd, (const T*)p->src_ra, (const T*)p->adj_r, B, p->prm.xi,
                            self_coef(p), dx, dsrc, st, B == 1 ? u : nullptr);
    }
    LAUNCHCHK();
    return FSE_OK;
}

// Stresslet adjoint for L = sum_m w_m . u(x_m): D_lm(x_b) = sum_a w_j(a)
// T_jlm(x_a - x_b) by the transposed chain (w spread as 3 components, each
// member's spectrum duplicated so that the z-pass with the transposed
// multiplier fills the six symmetric components as two halves of three, the
// inverse passes and quadrature of those six), contracted with the points' own
// n and q, plus the real-space part over the pairs within r_c.
template <typename T>
fse_status_t adjoint_stresslet_t(fse_plan* p, const T* q, const T* nrm, const T* w, T* dq, T* dn) {
    using V = C2<T>;
    hipStream_t st = p->stream;
    const int64_t n = p->n;
    const int B = p->batch;
    PointsDev<T> pd = points<T>(p);
    Timer& tm = p->timer;
    {
        TimedStage ts(tm, ST_PERMUTE, st);
        launch_permute3<T>(w, n, B, p->perm_s, (T*)p->adj_s, st);
        launch_permute3<T>(w, n, B, p->perm_r, (T*)p->adj_r, st);
        launch_permute3<T>(q, n, B, p->perm_r, (T*)p->src_ra, st);
        launch_permute3<T>(nrm, n, B, p->perm_r, (T*)p->src_rb, st);
    }
    const int64_t lstride = (int64_t)(p->geo.Mt + 1) * p->fg.n * p->fg.sz;  // one component of B
    V* Bs = (V*)p->B;
    for (int b = 0; b < B; ++b) {
        const T* wb = (const T*)p->adj_s + (int64_t)b * n * 3;
        { TimedStage ts(tm, ST_SPREAD, st); launch_spread<T>(p->gg, pd, wb, 3, 1, (T*)p->grid, st); }
        { TimedStage ts(tm, ST_FFTX, st);
          launch_fft_forward<T>(p->fg, p->gf, (const T*)p->grid, p->A, Bs + 6 * b * lstride, 3, (const T*)p->tw,
                                p->rev, p->revinv, st, 1); }
        { TimedStage ts(tm, ST_FFTY, st);
          launch_fft_forward<T>(p->fg, p->gf, (const T*)p->grid, p->A, Bs + 6 * b * lstride, 3, (const T*)p->tw,
                                p->rev, p->revinv, st, 2);
          HIPCHK(hipMemcpyAsync(Bs + (6 * b + 3) * lstride, Bs + 6 * b * lstride, 3 * lstride * sizeof(V),
                                hipMemcpyDeviceToDevice, st)); }
    }
    { TimedStage ts(tm, ST_FFTZ, st);
      launch_fft_zscale<T>(p->fg, p->gf, KTADJ, p->B, 3, 2 * B, (const T*)p->sig, PI / p->geo.Lt,
                           (const T*)p->tw, p->rev, p->revinv, st); }
    { TimedStage ts(tm, ST_FFTYI, st);
      launch_fft_inverse<T>(p->fg, p->gf, p->B, p->A, (T*)p->phi, 3, 2 * B, (const T*)p->tw, p->rev, p->revinv,
                            st, 1); }
    { TimedStage ts(tm, ST_FFTXI, st);
      launch_fft_inverse<T>(p->fg, p->gf, p->B, p->A, (T*)p->phi, 3, 2 * B, (const T*)p->tw, p->rev, p->revinv,
                            st, 2); }
    p->forward_valid = false;  // phi now holds the adjoint field
    { TimedStage ts(tm, ST_GATHER, st);
      launch_gather<T>(p->gg, pd, (const T*)p->phi, 2 * B, (T*)p->tadj, st);
      launch_tadj_contract<T>((const T*)p->tadj, q, nrm, n, B, dq, dn, st); }
    { TimedStage ts(tm, ST_REAL, st);
      launch_real_tadj<T>(p->cg, pd, (const T*)p->src_ra, (const T*)p->src_rb, (const T*)p->adj_r, B, p->prm.xi,
                          dq, dn, st); }
    LAUNCHCHK();
    return FSE_OK;
}

}  // namespace

namespace {

fse_status_t check_plan_args(fse_kernel_t kernel, fse_dtype_t dtype, const fse_params_t* params, int32_t batch,
                             int64_t nmax, fse_geometry_t* geo) {
    if (dtype != FSE_F32 && dtype != FSE_F64) { set_err("unknown dtype"); return FSE_EINVAL; }
    if (batch < 1) { set_err("batch must be >= 1"); return FSE_EINVAL; }
    if (nmax < 2 || nmax > (int64_t)1 << 30) { set_err("nmax must be in [2, 2^30]"); return FSE_EINVAL; }
    TRY(compute_geometry(kernel, params, geo));
    if (dtype == FSE_F32 && !(geo->eta < 1.0)) {
        // for eta >= 1 the scaling factor exp(-(1 - eta) k^2 / 4 xi^2) of Section 5.3
        // grows with k and amplifies the FP32 rounding of the spread grid and the FFTs
        set_err("eta = %.3f >= 1: the FP32 form needs eta < 1 (smaller xi h P, or larger M)", geo->eta);
        return FSE_EINVAL;
    }
    if (!fft_fits((int)kernel, dtype == FSE_F32 ? 4 : 8, geo->Mt)) {
        set_err("Mt=%d: the %s %s transforms of length %d do not fit in LDS (largest Mt for this kernel and dtype: "
                "%d)", geo->Mt, kernel == FSE_STRESSLET ? "six-component" : "three-component",
                dtype == FSE_F32 ? "FP32" : "FP64", 2 * geo->Mt, fft_max_mt((int)kernel, dtype == FSE_F32 ? 4 : 8));
        return FSE_EINVAL;
    }
    return FSE_OK;
}

// Fill a plan's constants: kernel, dtype, geometry, bin/cell/FFT descriptors.
void setup_plan(fse_plan* p, fse_kernel_t kernel, fse_dtype_t dtype, const fse_params_t* params,
                const fse_geometry_t& geo, int32_t batch, int64_t nmax, void* stream) {
    p->kernel = kernel;
    p->dtype = dtype;
    p->prm = *params;
    p->geo = geo;
    p->batch = batch;
    p->nmax = nmax;
    p->stream = (hipStream_t)stream;
    p->c_in = kernel == FSE_STRESSLET ? 6 : 3;
    GridGeo& gg = p->gg;
    gg.Mt = geo.Mt;
    gg.n = geo.n_fft;
    gg.P = params->P;
    gg.TS = bin_side(dtype == FSE_F32 ? 4 : 8, gg.P);  // bin side of the point binning
    gg.nt = (geo.Mt + gg.TS - 1) / gg.TS;
    for (int d = 0; d < 3; ++d) gg.x0[d] = geo.x0[d];
    gg.h = geo.h;
    gg.ahh = geo.alpha * geo.h * geo.h;
    p->gf = gg;
    p->family = kernel == FSE_ROTLET ? 1 : 0;
    p->periodic = params->periodic != 0;
    if (p->periodic) {
        // windows start at floor(t - P/2 + 1) >= -(ceil(P/2) - 1) in period units:
        // the extended grid starts that many nodes below the box and has P - 1
        // nodes more than the period, so no window wraps
        p->pshift = (params->P + 1) / 2 - 1;
        // window starts run from -pshift to M - P/2 (even P) or M - (P - 1)/2 (odd
        // P), so the windows span M + P - 1 (even) or M + P (odd) nodes
        gg.Mt = geo.Mt + params->P - 1 + (params->P & 1);
        gg.nt = (gg.Mt + gg.TS - 1) / gg.TS;
        for (int d = 0; d < 3; ++d) gg.x0[d] = geo.x0[d] - p->pshift * geo.h;
    }
    CellGeo& cg = p->cg;
    cg.ncell = geo.ncell;
    for (int d = 0; d < 3; ++d) cg.lo[d] = params->box_lo[d];
    cg.L = params->L;
    cg.cell = geo.cell;
    cg.rc2 = params->rc * params->rc;
    cg.periodic = params->periodic != 0;
    cg.qcap = default_qcap(dtype == FSE_F32 ? 4 : 8, false);
    cg.qcap_grad = default_qcap(dtype == FSE_F32 ? 4 : 8, true);
    FftGeo& fg = p->fg;
    fg.n = geo.n_fft;
    fg.ns = 0;
    fg.lines_cap = 0;
    int L = fg.n;
    for (int s = 0; s < 8 && geo.radices[s]; ++s) {
        fg.rad[s] = geo.radices[s];
        fg.Ls[s] = L;
        L /= geo.radices[s];
        fg.ns = s + 1;
    }
    // y- and z-line strides of the intermediate spectra padded to 128 bytes, so the
    // 16 (FP32) or 8 (FP64) lines a pass moves together start on a cache line
    {
        const int aln = 128 / (dtype == FSE_F32 ? 8 : 16);
        fg.sy = fg.sz = (geo.Mt + aln - 1) / aln * aln;
    }
    // fuse adjacent stages greedily where the pair is supported
    for (int s = 0; s < MAX_RADICES; ++s) fg.pair[s] = 0;
    for (int s = 0; s + 1 < fg.ns;) {
        if (fft_pair_ok(fg.rad[s], fg.rad[s + 1], dtype == FSE_F32 ? 4 : 8)) {
            fg.pair[s] = 1;
            s += 2;
        } else {
            s += 1;
        }
    }
}

// Free-space solver (Section 4.1-4.3): u = G * f on the M^3 grid with the
// truncated kernel's transform (precompute of Section 4.3) and the zero-padded
// transforms of size 2M; f, u: ncomp fields of M^3, processed three at a time.
template <typename T> fse_status_t freespace_solve_t(fse_plan* p, int ncomp, const T* f, T* u) {
    using V = C2<T>;
    const int M = p->geo.Mt, n = p->geo.n_fft, groups = p->batch;
    const int64_t M3 = (int64_t)M * M * M, Mp = M + 1;
    TRY(p->alloc((T**)&p->grid, 3 * groups * M3));
    TRY(p->alloc((T**)&p->phi, 3 * groups * M3));
    TRY(p->alloc((V**)&p->A, 3 * groups * Mp * M * (size_t)p->fg.sy));
    TRY(p->alloc((V**)&p->B, 3 * groups * Mp * n * (size_t)p->fg.sz));
    TRY(p->alloc(&p->sig64, Mp * Mp * Mp));
    TRY(p->alloc((T**)&p->sig, Mp * Mp * Mp));
    TRY(p->alloc((T**)&p->tw, 2 * n));
    TRY(p->alloc(&p->rev, n));
    TRY(p->alloc(&p->revinv, n));
    TRY(upload_fft_tables<T>(p));
    TRY(precompute<T>(p));
    hipStream_t st = p->stream;
    HIPCHK(hipMemcpyAsync(p->grid, f, ncomp * M3 * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (3 * groups > ncomp)
        HIPCHK(hipMemsetAsync((T*)p->grid + ncomp * M3, 0, (3 * groups - ncomp) * M3 * sizeof(T), st));
    launch_fft_forward<T>(p->fg, p->gf, (const T*)p->grid, p->A, p->B, 3 * groups, (const T*)p->tw, p->rev,
                          p->revinv, st, 1);
    launch_fft_forward<T>(p->fg, p->gf, (const T*)p->grid, p->A, p->B, 3 * groups, (const T*)p->tw, p->rev,
                          p->revinv, st, 2);
    launch_fft_zscale<T>(p->fg, p->gf, KSCALAR, p->B, 3, groups, (const T*)p->sig, PI / p->geo.Lt, (const T*)p->tw,
                         p->rev, p->revinv, st);
    launch_fft_inverse<T>(p->fg, p->gf, p->B, p->A, (T*)p->phi, 3, groups, (const T*)p->tw, p->rev, p->revinv, st,
                          1);
    launch_fft_inverse<T>(p->fg, p->gf, p->B, p->A, (T*)p->phi, 3, groups, (const T*)p->tw, p->rev, p->revinv, st,
                          2);
    LAUNCHCHK();
    HIPCHK(hipMemcpyAsync(u, p->phi, ncomp * M3 * sizeof(T), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));  // the workspace is freed on return
    return FSE_OK;
}

// Launch-shape tuning (runtime knobs): bin side (tiles of spreading and
// quadrature), real-space queue depths and waves per work item.
fse_status_t apply_tuning(fse_plan* p, const fse_tuning_t& t) {
    if (t.bin_side < MIN_BIN_SIDE || t.bin_side > MAX_BIN_SIDE || t.real_waves < 1 || t.real_waves > 4) {
        set_err("tuning: bin_side in [%d, %d], real_waves in [1, 4]", MIN_BIN_SIDE, MAX_BIN_SIDE);
        return FSE_EINVAL;
    }
    for (int q : {t.real_queue, t.real_queue_grad})
        if (q < 16 || q > 96 || q % 8) { set_err("tuning: queue depths in [16, 96], multiples of 8"); return FSE_EINVAL; }
    if (t.fft_lines < 0 || t.fft_lines > 16 || (t.fft_lines & (t.fft_lines - 1))) {
        set_err("tuning: fft_lines 0 (default) or 1, 2, 4, 8, 16");
        return FSE_EINVAL;
    }
    HIPCHK(hipStreamSynchronize(p->stream));
    p->gg.TS = t.bin_side;
    p->gg.nt = (p->gg.Mt + t.bin_side - 1) / t.bin_side;
    p->ntiles3 = (int64_t)p->gg.nt * p->gg.nt * p->gg.nt;
    p->bits_s = key_bits(p->ntiles3);
    p->cg.qcap = t.real_queue;
    p->cg.qcap_grad = t.real_queue_grad;
    p->real_waves = t.real_waves;
    p->fg.lines_cap = t.fft_lines;
    p->n = 0;  // the points' bins and work items follow the tuning: set them again
    p->forward_valid = false;
    p->free_targets();
    return FSE_OK;
}

fse_tuning_t current_tuning(const fse_plan* p) {
    fse_tuning_t t;
    t.bin_side = p->gg.TS;
    t.real_queue = p->cg.qcap;
    t.real_queue_grad = p->cg.qcap_grad;
    t.real_waves = p->real_waves;
    t.fft_lines = p->fg.lines_cap;
    return t;
}

// One timed workload run (set_points + eval [+ adjoint]), in milliseconds.
template <typename T>
fse_status_t time_workload(fse_plan* p, int64_t n, const T* x, const T* a, const T* b, const T* w, T* u, T* ds,
                           T* dx, int repeats, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    fse_status_t rc = FSE_OK;
    for (int r = -1; r < repeats && rc == FSE_OK; ++r) {  // r = -1: warm-up
        if (r == 0) (void)hipEventRecord(e0, p->stream);
        rc = set_points_t<T>(p, n, x, 0);
        if (rc == FSE_OK && w && !p->periodic && p->kernel != FSE_STRESSLET) {
            rc = eval_with_adjoint_t<T>(p, a, w, u, ds, dx);  // the forward and adjoint in one call
        } else {
            if (rc == FSE_OK) rc = eval_t<T>(p, a, b, u, nullptr, true);
            if (rc == FSE_OK && w) rc = adjoint_t<T>(p, a, w, ds, dx, 0);
        }
    }
    if (rc == FSE_OK) {
        (void)hipEventRecord(e1, p->stream);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess) rc = FSE_EHIP;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

template <typename T>
fse_status_t autotune_t(fse_plan* p, int64_t n, const T* x, const T* a, const T* b, const T* w, int repeats,
                        fse_tuning_t* best_out) {
    const int64_t vec = (int64_t)p->batch * n * 3;
    T *u = nullptr, *ds = nullptr, *dx = nullptr;
    auto release = [&]() {
        if (u) (void)hipFree(u);
        if (ds) (void)hipFree(ds);
        if (dx) (void)hipFree(dx);
    };
    if (hipMalloc(&u, vec * sizeof(T)) != hipSuccess ||
        (w && (hipMalloc(&ds, vec * sizeof(T)) != hipSuccess || hipMalloc(&dx, n * 3 * sizeof(T)) != hipSuccess))) {
        release();
        set_err("autotune: out of device memory");
        return FSE_ENOMEM;
    }
    fse_tuning_t best = current_tuning(p);
    float best_ms = 0.f;
    fse_status_t rc = apply_tuning(p, best);
    if (rc == FSE_OK) rc = time_workload<T>(p, n, x, a, b, w, u, ds, dx, repeats, &best_ms);
    const bool f32 = sizeof(T) == 4;
    // a queue depth whose pass the timed workload never runs keeps its value (the
    // fused call for one source set runs only the gradient pass; without w only
    // value passes run)
    const bool grad_only = w && !p->periodic && p->kernel != FSE_STRESSLET && p->batch == 1;
    // each knob in turn, the others held at the best so far
    for (int knob = 0; knob < 5 && rc == FSE_OK; ++knob) {
        if ((knob == 2 && grad_only) || (knob == 3 && !w)) continue;
        std::vector<int> cand;
        if (knob == 0) cand = {5, 6, 7, 8};
        else if (knob == 1) cand = {1, 2, 3, 4};
        else if (knob == 2) cand = f32 ? std::vector<int>{24, 32, 48} : std::vector<int>{32, 48, 64};
        else if (knob == 3) cand = {32, 48, 64};
        else cand = f32 ? std::vector<int>{0, 8, 4} : std::vector<int>{0, 2, 1};
        for (int v : cand) {
            fse_tuning_t t = best;
            int* field = knob == 0 ? &t.bin_side : knob == 1 ? &t.real_waves : knob == 2 ? &t.real_queue
                                                   : knob == 3 ? &t.real_queue_grad : &t.fft_lines;
            if (*field == v) continue;
            *field = v;
            float ms = 0.f;
            rc = apply_tuning(p, t);
            if (rc == FSE_OK) rc = time_workload<T>(p, n, x, a, b, w, u, ds, dx, repeats, &ms);
            if (rc != FSE_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    }
    if (rc == FSE_OK) rc = apply_tuning(p, best);
    if (rc == FSE_OK) rc = set_points_t<T>(p, n, x, 0);
    if (rc == FSE_OK) {
        hipError_t e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) { set_err("autotune: %s", hipGetErrorString(e)); rc = FSE_EHIP; }
    }
    release();
    if (rc == FSE_OK && best_out) *best_out = best;
    return rc;
}

// Device scratch of the no-allocation entry point: one array per GPU, loaded
// with the library's code object and held until the process ends.  Host code
// never uses the array's name as an address: it takes each device's address
// once from hipGetSymbolAddress and passes that.
__device__ __align__(256) unsigned char scratch[FSE_NOALLOC_MAX_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Address of the current device's scratch array (looked up on first use).
fse_status_t scratch_ptr(void** out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) { set_err("device %d beyond the supported %d", dev, MAX_DEVICES); return FSE_EINVAL; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* q = nullptr;
        HIPCHK(hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)));
        if (!q) { set_err("hipGetSymbolAddress returned a null scratch address"); return FSE_EHIP; }
        g_scratch_ptr[dev] = q;
    }
    *out = g_scratch_ptr[dev];
    return FSE_OK;
}

template <typename T>
fse_status_t eval_noalloc_t(fse_plan* p, int64_t n, const T* x, const T* a, const T* b, T* u, int validate) {
    TRY(plan_init<T>(p));
    TRY(set_points_t<T>(p, n, x, validate));
    return eval_t<T>(p, a, b, u, nullptr, true);
}

}  // namespace

extern "C" {

const char* fse_last_error(void) { return g_err; }

const char* fse_status_string(fse_status_t s) {
    switch (s) {
        case FSE_OK: return "ok";
        case FSE_EINVAL: return "invalid argument";
        case FSE_ERANGE: return "point outside the box";
        case FSE_ENOMEM: return "out of device memory";
        case FSE_EHIP: return "HIP runtime error";
        case FSE_EUNSUPPORTED: return "unsupported";
        case FSE_ESTATE: return "call order violated";
    }
    return "unknown status";
}

fse_status_t fse_geometry(fse_kernel_t kernel, const fse_params_t* params, fse_geometry_t* out) {
    return compute_geometry(kernel, params, out);
}

fse_status_t fse_plan_create(fse_kernel_t kernel, fse_dtype_t dtype, const fse_params_t* params, int32_t batch,
                             int64_t nmax, void* stream, fse_plan_t** out) {
    if (!out) { set_err("null plan pointer"); return FSE_EINVAL; }
    *out = nullptr;
    fse_geometry_t geo;
    TRY(check_plan_args(kernel, dtype, params, batch, nmax, &geo));
    fse_plan* p = new (std::nothrow) fse_plan();
    if (!p) { set_err("host allocation failed"); return FSE_ENOMEM; }
    setup_plan(p, kernel, dtype, params, geo, batch, nmax, stream);
    fse_status_t rc = dtype == FSE_F32 ? plan_init<float>(p) : plan_init<double>(p);
    if (rc != FSE_OK) {
        delete p;
        return rc;
    }
    *out = p;
    return FSE_OK;
}

fse_status_t fse_plan_geometry(const fse_plan_t* plan, fse_geometry_t* out) {
    if (!plan || !out) { set_err("null argument"); return FSE_EINVAL; }
    *out = plan->geo;
    return FSE_OK;
}

fse_status_t fse_plan_set_stream(fse_plan_t* plan, void* stream) {
    if (!plan) { set_err("null plan"); return FSE_EINVAL; }
    plan->stream = (hipStream_t)stream;
    return FSE_OK;
}

fse_status_t fse_set_points(fse_plan_t* plan, int64_t n, const void* x, int32_t validate) {
    if (!plan || !x) { set_err("null argument"); return FSE_EINVAL; }
    if (n < 2 || n > plan->nmax) { set_err("n=%lld outside [2, nmax=%lld]", (long long)n, (long long)plan->nmax); return FSE_EINVAL; }
    return plan->dtype == FSE_F32 ? set_points_t<float>(plan, n, (const float*)x, validate)
                                  : set_points_t<double>(plan, n, (const double*)x, validate);
}

fse_status_t fse_eval(fse_plan_t* plan, const void* a, const void* b, void* u) {
    if (!plan || !a || !u) { set_err("null argument"); return FSE_EINVAL; }
    if (plan->kernel == FSE_STRESSLET && !b) { set_err("stresslet needs the normals (src_b)"); return FSE_EINVAL; }
    if (plan->n == 0) { set_err("fse_set_points must come first"); return FSE_ESTATE; }
    return plan->dtype == FSE_F32
               ? eval_t<float>(plan, (const float*)a, (const float*)b, (float*)u, nullptr, true)
               : eval_t<double>(plan, (const double*)a, (const double*)b, (double*)u, nullptr, true);
}

fse_status_t fse_eval_parts(fse_plan_t* plan, const void* a, const void* b, void* u_real, void* u_fourier) {
    if (!plan || !a) { set_err("null argument"); return FSE_EINVAL; }
    if (plan->kernel == FSE_STRESSLET && !b) { set_err("stresslet needs the normals (src_b)"); return FSE_EINVAL; }
    if (plan->n == 0) { set_err("fse_set_points must come first"); return FSE_ESTATE; }
    return plan->dtype == FSE_F32
               ? eval_t<float>(plan, (const float*)a, (const float*)b, (float*)u_real, (float*)u_fourier, false)
               : eval_t<double>(plan, (const double*)a, (const double*)b, (double*)u_real, (double*)u_fourier,
                                false);
}

fse_status_t fse_set_targets(fse_plan_t* plan, int64_t nt, const void* y, int32_t validate) {
    if (!plan || !y) { set_err("null argument"); return FSE_EINVAL; }
    if (plan->periodic) { set_err("not implemented for the periodic sum"); return FSE_EUNSUPPORTED; }
    if (nt < 1 || nt > (int64_t)1 << 30) { set_err("nt=%lld outside [1, 2^30]", (long long)nt); return FSE_EINVAL; }
    return plan->dtype == FSE_F32 ? set_targets_t<float>(plan, nt, (const float*)y, validate)
                                  : set_targets_t<double>(plan, nt, (const double*)y, validate);
}

fse_status_t fse_eval_targets(fse_plan_t* plan, const void* a, const void* b, void* u_real, void* u_fourier) {
    if (!plan || !a || (!u_real && !u_fourier)) { set_err("null argument"); return FSE_EINVAL; }
    if (plan->kernel == FSE_STRESSLET && !b) { set_err("stresslet needs the normals (src_b)"); return FSE_EINVAL; }
    if (plan->n == 0) { set_err("fse_set_points must come first"); return FSE_ESTATE; }
    if (plan->tg.n == 0) { set_err("fse_set_targets must come first"); return FSE_ESTATE; }
    return plan->dtype == FSE_F32
               ? eval_targets_t<float>(plan, (const float*)a, (const float*)b, (float*)u_real, (float*)u_fourier)
               : eval_targets_t<double>(plan, (const double*)a, (const double*)b, (double*)u_real,
                                        (double*)u_fourier);
}

fse_status_t fse_eval_adjoint(fse_plan_t* plan, const void* a, const void* w, void* dsrc, void* dx,
                              int32_t recompute) {
    if (!plan || !a || !w) { set_err("null argument"); return FSE_EINVAL; }
    if (plan->periodic) { set_err("not implemented for the periodic sum"); return FSE_EUNSUPPORTED; }
    if (plan->kernel == FSE_STRESSLET) { set_err("the stresslet adjoint is not implemented"); return FSE_EUNSUPPORTED; }
    if (plan->n == 0) { set_err("fse_set_points must come first"); return FSE_ESTATE; }
    if (!dsrc && !dx) return FSE_OK;
    return plan->dtype == FSE_F32
               ? adjoint_t<float>(plan, (const float*)a, (const float*)w, (float*)dsrc, (float*)dx, recompute)
               : adjoint_t<double>(plan, (const double*)a, (const double*)w, (double*)dsrc, (double*)dx,
                                   recompute);
}

fse_status_t fse_eval_with_adjoint(fse_plan_t* plan, const void* a, const void* w, void* u, void* dsrc, void* dx) {
    if (!plan || !a || !w || !u || !dsrc || !dx) { set_err("null argument"); return FSE_EINVAL; }
    if (plan->periodic) { set_err("not implemented for the periodic sum"); return FSE_EUNSUPPORTED; }
    if (plan->kernel == FSE_STRESSLET) {
        set_err("stokeslet and rotlet plans only (the stresslet adjoint is fse_eval_adjoint_stresslet)");
        return FSE_EUNSUPPORTED;
    }
    if (plan->n == 0) { set_err("fse_set_points must come first"); return FSE_ESTATE; }
    return plan->dtype == FSE_F32
               ? eval_with_adjoint_t<float>(plan, (const float*)a, (const float*)w, (float*)u, (float*)dsrc,
                                            (float*)dx)
               : eval_with_adjoint_t<double>(plan, (const double*)a, (const double*)w, (double*)u, (double*)dsrc,
                                             (double*)dx);
}

fse_status_t fse_eval_adjoint_stresslet(fse_plan_t* plan, const void* q, const void* nrm, const void* w, void* dq,
                                        void* dn) {
    if (!plan || !q || !nrm || !w || !dq || !dn) { set_err("null argument"); return FSE_EINVAL; }
    if (plan->kernel != FSE_STRESSLET) { set_err("not a stresslet plan"); return FSE_EINVAL; }
    if (plan->n == 0) { set_err("fse_set_points must come first"); return FSE_ESTATE; }
    return plan->dtype == FSE_F32
               ? adjoint_stresslet_t<float>(plan, (const float*)q, (const float*)nrm, (const float*)w, (float*)dq,
                                            (float*)dn)
               : adjoint_stresslet_t<double>(plan, (const double*)q, (const double*)nrm, (const double*)w,
                                             (double*)dq, (double*)dn);
}

fse_status_t fse_plan_multiplier(fse_plan_t* plan, double* out) {
    if (!plan || !out) { set_err("null argument"); return FSE_EINVAL; }
    const size_t Mp = plan->geo.Mt + 1;
    HIPCHK(hipMemcpyAsync(out, plan->sig64, Mp * Mp * Mp * sizeof(double), hipMemcpyDeviceToHost, plan->stream));
    HIPCHK(hipStreamSynchronize(plan->stream));
    return FSE_OK;
}

fse_status_t fse_plan_grid(fse_plan_t* plan, int32_t which, double* out) {
    if (!plan || !out || (which != 0 && which != 1)) { set_err("bad argument"); return FSE_EINVAL; }
    const size_t M3 = (size_t)plan->geo.Mt * plan->geo.Mt * plan->geo.Mt;
    const size_t cnt = (size_t)plan->batch * (which == 0 ? plan->c_in : 3) * M3;
    const void* src = which == 0 ? plan->grid : plan->phi;
    HIPCHK(hipStreamSynchronize(plan->stream));
    if (plan->dtype == FSE_F64) {
        HIPCHK(hipMemcpy(out, src, cnt * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::vector<float> tmp(cnt);
        HIPCHK(hipMemcpy(tmp.data(), src, cnt * sizeof(float), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < cnt; ++i) out[i] = tmp[i];
    }
    return FSE_OK;
}

fse_status_t fse_precompute_cache_stats(int64_t* hits, int64_t* misses, size_t* bytes, int32_t* entries) {
    std::lock_guard<std::mutex> lk(bt_mu);
    if (hits) *hits = bt_hits;
    if (misses) *misses = bt_misses;
    if (bytes) *bytes = bt_bytes;
    if (entries) *entries = (int32_t)bt_cache.size();
    return FSE_OK;
}

fse_status_t fse_plan_bins(fse_plan_t* plan, int32_t* nbins, int32_t* perm_s, int32_t* bpack_s, double* coff_s,
                           int32_t* tile_start, int32_t* perm_r, int32_t* cell_start) {
    if (!plan) { set_err("null plan"); return FSE_EINVAL; }
    if (plan->n == 0) { set_err("fse_set_points must come first"); return FSE_ESTATE; }
    if (nbins) *nbins = plan->gg.nt;
    const size_t n = (size_t)plan->n;
    HIPCHK(hipStreamSynchronize(plan->stream));
    auto get = [&](void* dst, const void* src, size_t bytes) -> fse_status_t {
        if (dst) HIPCHK(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
        return FSE_OK;
    };
    TRY(get(perm_s, plan->perm_s, n * sizeof(int)));
    TRY(get(bpack_s, plan->bpack_s, n * sizeof(int)));
    TRY(get(tile_start, plan->start_s, (size_t)(plan->ntiles3 + 1) * sizeof(int)));
    TRY(get(perm_r, plan->perm_r, n * sizeof(int)));
    TRY(get(cell_start, plan->start_r, (size_t)(plan->ncells3 + 1) * sizeof(int)));
    if (coff_s) {
        if (plan->dtype == FSE_F64) {
            TRY(get(coff_s, plan->coff_s, 3 * n * sizeof(double)));
        } else {
            std::vector<float> tmp(3 * n);
            TRY(get(tmp.data(), plan->coff_s, 3 * n * sizeof(float)));
            for (size_t i = 0; i < 3 * n; ++i) coff_s[i] = tmp[i];
        }
    }
    return FSE_OK;
}

fse_status_t fse_plan_set_timing(fse_plan_t* plan, int32_t enable) {
    if (!plan) { set_err("null plan"); return FSE_EINVAL; }
    plan->timer.on = enable != 0;
    return FSE_OK;
}

fse_status_t fse_plan_timings(fse_plan_t* plan, double* ms, int64_t* launches) {
    if (!plan || !ms) { set_err("null argument"); return FSE_EINVAL; }
    HIPCHK(hipStreamSynchronize(plan->stream));
    for (int s = 0; s < FSE_NSTAGES; ++s) {
        ms[s] = 0.0;
        if (launches) launches[s] = 0;
    }
    for (auto& r : plan->timer.recs) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.stage] += t;
        if (launches) launches[r.stage] += 1;
    }
    plan->timer.recs.clear();
    plan->timer.used = 0;
    return FSE_OK;
}

const char* fse_stage_name(int32_t stage) {
    return (stage >= 0 && stage < FSE_NSTAGES) ? STAGE_NAMES[stage] : "unknown";
}

fse_status_t fse_plan_get_tuning(const fse_plan_t* plan, fse_tuning_t* out) {
    if (!plan || !out) { set_err("null argument"); return FSE_EINVAL; }
    *out = current_tuning(plan);
    return FSE_OK;
}

fse_status_t fse_plan_set_tuning(fse_plan_t* plan, const fse_tuning_t* t) {
    if (!plan || !t) { set_err("null argument"); return FSE_EINVAL; }
    return apply_tuning(plan, *t);
}

fse_status_t fse_plan_autotune(fse_plan_t* plan, int64_t n, const void* x, const void* a, const void* b,
                               const void* w, int32_t repeats, fse_tuning_t* best) {
    if (!plan || !x || !a) { set_err("null argument"); return FSE_EINVAL; }
    if (n < 2 || n > plan->nmax) { set_err("n=%lld outside [2, nmax]", (long long)n); return FSE_EINVAL; }
    if (plan->kernel == FSE_STRESSLET && !b) { set_err("stresslet needs the normals (src_b)"); return FSE_EINVAL; }
    if (w && (plan->kernel == FSE_STRESSLET || plan->periodic)) {
        set_err("autotune: the adjoint is timed for free-space stokeslet and rotlet plans only");
        return FSE_EINVAL;
    }
    if (repeats < 1) repeats = 1;
    return plan->dtype == FSE_F32
               ? autotune_t<float>(plan, n, (const float*)x, (const float*)a, (const float*)b, (const float*)w,
                                   repeats, best)
               : autotune_t<double>(plan, n, (const double*)x, (const double*)a, (const double*)b, (const double*)w,
                                    repeats, best);
}

fse_status_t fse_plan_workspace(const fse_plan_t* plan, size_t* bytes) {
    if (!plan || !bytes) { set_err("null argument"); return FSE_EINVAL; }
    *bytes = plan->bytes;
    return FSE_OK;
}

fse_status_t fse_eval_noalloc(fse_kernel_t kernel, fse_dtype_t dtype, const fse_params_t* params, int32_t batch,
                              int64_t n, const void* x, const void* src_a, const void* src_b, void* u,
                              int32_t validate, void* stream) {
    if (!x || !src_a || !u) { set_err("null argument"); return FSE_EINVAL; }
    if (kernel == FSE_STRESSLET && !src_b) { set_err("stresslet needs the normals (src_b)"); return FSE_EINVAL; }
    fse_geometry_t geo;
    TRY(check_plan_args(kernel, dtype, params, batch, n, &geo));
    fse_plan p;  // host object only; every device buffer is carved from the scratch array
    setup_plan(&p, kernel, dtype, params, geo, batch, n, stream);
    size_t need = 0;
    TRY(dtype == FSE_F32 ? plan_bytes<float>(&p, &need) : plan_bytes<double>(&p, &need));
    if (need > FSE_NOALLOC_MAX_BYTES) {
        set_err("this evaluation needs %zu bytes of device workspace, above the %zu-byte static scratch of "
                "fse_eval_noalloc (use a plan)", need, (size_t)FSE_NOALLOC_MAX_BYTES);
        return FSE_EINVAL;
    }
    void* base = nullptr;
    TRY(scratch_ptr(&base));
    p.arena = (char*)base;
    p.arena_cap = FSE_NOALLOC_MAX_BYTES;
    return dtype == FSE_F32
               ? eval_noalloc_t<float>(&p, n, (const float*)x, (const float*)src_a, (const float*)src_b, (float*)u,
                                       validate)
               : eval_noalloc_t<double>(&p, n, (const double*)x, (const double*)src_a, (const double*)src_b,
                                        (double*)u, validate);
}

fse_status_t fse_freespace_solve(int32_t family, fse_dtype_t dtype, int32_t M, double h, int32_t ncomp, const void* f,
                                 void* u, void* stream) {
    if (!f || !u) { set_err("null argument"); return FSE_EINVAL; }
    if (family != 0 && family != 1) { set_err("family must be 0 (biharmonic) or 1 (harmonic)"); return FSE_EINVAL; }
    if (dtype != FSE_F32 && dtype != FSE_F64) { set_err("unknown dtype"); return FSE_EINVAL; }
    if (M < 2 || M > MAX_MT || !smooth7(2 * M)) {
        set_err("M=%d: need 2 <= M <= %d and 2M factoring into 2,3,5,7", M, MAX_MT);
        return FSE_EINVAL;
    }
    if (!(h > 0) || !isfinite(h) || ncomp < 1) { set_err("need h > 0 and ncomp >= 1"); return FSE_EINVAL; }
    fse_geometry_t geo;
    memset(&geo, 0, sizeof geo);
    geo.Mt = M;
    geo.n_fft = 2 * M;
    geo.h = h;
    geo.Lt = M * h;
    geo.R = sqrt(3.0) * geo.Lt;  // Section 4.1: the truncation radius covers the box diagonal
    int Mg = (int)floor((1.0 + sqrt(3.0)) * M) + 1;
    if (Mg % 2) ++Mg;
    geo.Mg = Mg;
    geo.kinf = PI / h;
    geo.ncell = 1;
    geo.cell = geo.Lt;
    int rad[MAX_RADICES];
    const int ns = factorize(geo.n_fft, rad);
    if (ns < 0 || ns > 7) { set_err("cannot factor n=%d", geo.n_fft); return FSE_EINVAL; }
    for (int s = 0; s < ns; ++s) geo.radices[s] = rad[s];
    fse_params_t prm;
    memset(&prm, 0, sizeof prm);
    prm.xi = 1.0;
    prm.rc = geo.Lt;
    prm.M = M;
    prm.P = 2;
    prm.L = geo.Lt;
    prm.Mt = M;
    fse_plan p;  // host object; its device buffers are freed on return
    setup_plan(&p, FSE_STOKESLET, dtype, &prm, geo, (ncomp + 2) / 3, 2, stream);
    p.solver = true;
    p.family = family;
    return dtype == FSE_F32 ? freespace_solve_t<float>(&p, ncomp, (const float*)f, (float*)u)
                            : freespace_solve_t<double>(&p, ncomp, (const double*)f, (double*)u);
}

void fse_plan_destroy(fse_plan_t* plan) {
    if (!plan) return;
    (void)hipStreamSynchronize(plan->stream);
    delete plan;
}

}  // extern "C"
