// Host runtime of the C ABI in include/hk.h: handles, argument validation,
// tiling and LDS layout, workspace, and the stream-ordered launch sequence
//   control-block reset -> persistent basis iteration -> small sketched
//   least squares -> x = L_k y.
#include "hk.h"
#include "hk_internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_set>
#include <cfloat>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace hk;

namespace {

thread_local std::string g_err;

// HK_LOG (environment, read once): 0 or unset: silent; 1: every refused call
// and failure is also written to stderr; 2: as 1, plus one line per solve
// plan (kernel, grid, tile, LDS, workspace) and per server admission.
int log_level()
{
    static const int lv = [] {
        const char* e = std::getenv("HK_LOG");
        return e ? std::atoi(e) : 0;
    }();
    return lv;
}

hk_status fail(hk_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    if (log_level() >= 1) std::fprintf(stderr, "hk: status %d: %s\n", (int)st, buf);
    return st;
}

void log_info(const char* fmt, ...)
{
    if (log_level() < 2) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "hk: %s\n", buf);
}

// Live handles: every context, operator, solve and server from its creation
// to its destruction.  Entry points refuse a handle that is not live (null,
// never created here, or already destroyed) with HK_EINVAL before touching
// its memory, so a second destroy is an error rather than a double free.
// (A destroyed handle whose address a new handle reuses is live again.)
std::mutex g_live_mu;
std::unordered_set<const void*> g_live;

void live_add(const void* h)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(h);
}

bool live_take(const void* h)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    return h && g_live.erase(h) == 1;
}

bool live(const void* h)
{
    if (!h) return false;
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.count(h) != 0;
}

#define HK_LIVE(h)                                                                         \
    do {                                                                                   \
        if (!live(h)) return fail(HK_EINVAL, (h) ? "unknown or destroyed handle " #h : "null handle " #h); \
    } while (0)

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(HK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

// Workspace of hk_solve_run_noalloc: a static device array, one copy per
// GPU, held until the process ends.  Host code never passes `scratch` itself
// to a kernel (in host code it names a host-side stand-in); it uses the
// device address hipGetSymbolAddress returns, taken once per device.
constexpr size_t NOALLOC_MAX_BYTES = HK_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_MAX_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};
bool g_scratch_done[MAX_DEVICES] = {};

// Device address of this device's scratch copy (the device must be current).
void scratch_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = (e == hipSuccess) ? ptr : nullptr;
    g_scratch_done[device] = true;
}
}  // namespace

struct hk_context {
    int device = 0;
    hipStream_t stream = nullptr;
    int ncu = 0;
    size_t lds_max = 65536;
    unsigned long long wall_rate_khz = 100000;
};

struct hk_op {
    hk_context* ctx = nullptr;
    int kind = OP_BLUR;
    int64_t m = 0, n = 0;
    int dtype = HK_F64;
    // blur
    int ny = 0, nx = 0, r = 0, bc = 0;
    double* d_taps = nullptr;          // taps_y then taps_x (separable PSF)
    int ntap = 0;                      // general PSF: its nonzero entries
    int* d_toff = nullptr;             // (a + r) << 16 | (b + r)
    double* d_tw = nullptr;            // p(a, b)
    // CSR
    int64_t nnz = 0;
    int64_t* d_rp = nullptr;
    int* d_ci = nullptr;
    void* d_cv = nullptr;
    int64_t* d_rpt = nullptr;
    int* d_cit = nullptr;
    void* d_cvt = nullptr;
    int lpr = 16, lprt = 16;
    double anorm = 0.0;                // ||A||_inf (max absolute row sum)
    double anorm_t = 0.0;              // ||A^T||_inf
    // row pointers of A and A^T on the host, for the tile ranges below
    std::vector<int64_t> h_rp, h_rpt;
    // tile ranges balanced by nonzeros, per grid size: d holds the starts of
    // the m-space (G + 1 ints), then of the n-space; d == nullptr records a
    // grid for which no balanced ranges fit the plan
    struct CsrPart { int G = 0; int ept = 0; int* d = nullptr; };
    std::vector<CsrPart> parts;
    std::mutex part_mu;
};

struct hk_solve {
    hk_op* op = nullptr;
    hk_params prm{};
    int tb = HK_F64;               // basis storage type
    int rect = 0;
    int sk = SK_GAUSS;
    int kernel = OP_BLUR;
    int ept = 1;
    int G = 0;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    KArgs ka{};
    LsArgs la{};
    CombineArgs ca{};
    static constexpr int NEV = 256;        // runs whose events are kept (at most)
    int nev = NEV;                         // event slots created
    hipEvent_t ev[NEV][3] = {};
    hipStream_t stream = nullptr;          // where runs are ordered
    bool own_ws = true;                    // the workspace was allocated here
    // Gaussian sketches formed at the end as block contractions:
    // T = S2 [basis of the data space], c = S2 b, T1 = S1 L_k, then Z, F
    bool zend = false;
    BskArgs bz{}, bc{}, bf{};
    int nrhs = 1;                          // right-hand sides advanced together
    int sel = 0;                           // the one the getters report
    double* call = nullptr;                // S2 b of the first right-hand side (the others follow)
    double* yp = nullptr;                  // prefix-solution coefficients (first right-hand side's region)
    const void* b_last = nullptr;          // right-hand side(s) of the last run (for the true residuals)
    size_t region = 0;                     // bytes between right-hand sides' regions
    double* T = nullptr;
    double* T1 = nullptr;
    long long runs = 0;                    // runs launched
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;   // of the last run
    bool ran = false;
    bool waited = false;
    hk_status last = HK_OK;
    int k_done = 0;
    int nt = 0, ng = 0;
    // per right-hand side, after a wait: status, basis columns, pivots found
    int rst[RMAX] = {}, rkd[RMAX] = {}, rnt[RMAX] = {}, rng[RMAX] = {};
    bool aborted = false;                  // the last run's grid barrier timed out
};

namespace {

size_t dsize(int dtype) { return dtype == HK_F64 ? 8 : (dtype == HK_F32 ? 4 : 2); }
// LDS pivot block entries: FP32 for 16-bit bases
size_t pdsize(int tb) { return tb == HK_F64 ? 8 : 4; }

int lanes_per_row(double avg_nnz)
{
    int l = 4;
    while (l < 64 && l * 4 < avg_nnz) l *= 2;
    return l;
}

// ---------------------------------------------------------------- tiling
struct Plan {
    Space spm{}, spn{};
    int kernel = OP_BLUR;   // OP_BLUR_ONEBAR, OP_BLUR (generic) or OP_CSR
    int nslot = 0, spx = 0;
    int G = 0;
    int ept = 1;
    int lds_total = 0;
    KArgs lds{};      // only the lds_* fields
    bool ok = false;
    std::string why;
};

int lds_layout(KArgs& a, int kp1, int s, int ept, int rect, int op, int TY, int TX, int r, int ntap, int dtype,
               int pmode, int rp_stage)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 16);
        return (int)o;
    };
    a.lds_h = take(sizeof(double) * (KMAX + 1));
    a.lds_w = take(sizeof(double) * NT * ept);
    a.lds_pl_m = take(sizeof(int) * kp1);
    a.lds_pc_m = take(sizeof(int) * kp1);
    a.lds_bm_m = take(sizeof(unsigned) * ((NT * ept + 31) / 32));
    if (rect) {
        a.lds_pl_n = take(sizeof(int) * kp1);
        a.lds_pc_n = take(sizeof(int) * kp1);
        a.lds_bm_n = take(sizeof(unsigned) * ((NT * ept + 31) / 32));
    } else {
        a.lds_pl_n = a.lds_pl_m;
        a.lds_pc_n = a.lds_pc_m;
        a.lds_bm_n = a.lds_bm_m;
    }
    const size_t ng = (size_t)(s + 3) / 4;
    a.lds_sk = take(sizeof(double) * std::max<size_t>((size_t)s, 4 * ng));
    if (op == OP_BLUR) {
        const int SW = TX + 2 * r, SH = TY + 2 * r;
        a.lds_stage = take(dsize(dtype) * (size_t)SW * SH);
        a.lds_vert = take(sizeof(double) * (size_t)TY * SW);
        a.lds_taps = take(psf_lds_bytes(r, ntap));
    } else {
        a.lds_stage = a.lds_vert = a.lds_taps = 0;
    }
    const size_t tri = dsize(dtype) * (size_t)packed_size(kp1 - 1);
    a.pmode = pmode;
    a.lds_pD = take(tri);
    a.lds_pL = (rect && pmode == 0) ? take(tri) : a.lds_pD;
    a.lds_rp_m = a.lds_rp_n = -1;
    if (op == OP_CSR && rp_stage) {
        a.lds_rp_m = take(sizeof(int) * ((size_t)NT * ept + 1));
        a.lds_rp_n = rect ? take(sizeof(int) * ((size_t)NT * ept + 1)) : a.lds_rp_m;
    }
    a.lds_total = (int)off;
    return a.lds_total;
}

int kp1_of(const hk_params* p) { return p->k + 1; }

// slots per pivot of the window partial sums: tiles a (2r+1)-wide window spans
int spx_of(int r, int TX) { return (2 * r + 1 + TX - 1) / TX + 1; }
int nslot_of(int r, int TY, int TX) { return spx_of(r, TX) * ((2 * r + 1 + TY - 1) / TY + 1); }

// LDS of the single-barrier blur kernel; 0 if it does not fit.  zeta > 0:
// the per-step sparse-sign row lists; nrhs: right-hand sides, each with its
// own block of what it keeps across steps.
int lds_layout_onebar(KArgs& a, int k, int s, int ept, int TY, int TX, int r, int ntap, int tb, int zeta,
                      int nrhs, size_t lds_max)
{
    a.lds_rp_m = a.lds_rp_n = -1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 16);
        return (int)o;
    };
    const int kp1 = k + 1;
    a.lds_h = take(sizeof(double) * (KMAX + 1));
    a.lds_hs = take(sizeof(double) * (KMAX + 1));
    a.lds_w = take(sizeof(double) * NT * ept);
    const size_t ng = (size_t)(s + 3) / 4;
    a.lds_sk = take(sizeof(double) * std::max<size_t>((size_t)s, 4 * ng));
    const int SW = TX + 2 * r, SH = TY + 2 * r;
    a.lds_stage = take(dsize(tb) * (size_t)SW * SH);
    a.lds_vert = take(sizeof(double) * (size_t)TY * SW);
    a.lds_taps = take(psf_lds_bytes(r, ntap));
    a.lds_wred = take(sizeof(double) * (size_t)kp1 * (size_t)std::max(NWAVE, 1 + nslot_of(r, TY, TX)));
    a.pmode = 0;
    a.lds_skt = 0;
    if (zeta > 0) {
        // sparse-sign row lists of S2 and S1: offsets (s + 1 each, 32 bits) and
        // entries (16 bits per nonzero); the kernel needs them
        const size_t tabs = sizeof(unsigned) * 2 * (size_t)(s + 1) + sizeof(unsigned short) * 2 * (size_t)TY * TX * (size_t)zeta;
        a.lds_skt = take(tabs);
    }
    // what each right-hand side keeps across steps, one block per right-hand
    // side: the scales s_j and f_j scales, this tile's pivots, all pivots,
    // the window list and the pivot block P
    const size_t rb = off;
    a.lds_scale = take(sizeof(double) * 2 * (size_t)kp1);
    a.lds_pl_m = take(sizeof(int) * kp1);
    a.lds_pc_m = take(sizeof(int) * kp1);
    a.lds_bm_m = take(sizeof(unsigned) * ((NT * ept + 31) / 32));
    a.lds_pl_n = take(sizeof(int) * kp1);      // all pivots
    a.lds_pc_n = take(sizeof(int) * kp1);      // window list
    a.lds_bm_n = a.lds_bm_m;
    a.lds_pD = take(pdsize(tb) * (size_t)packed_size(k));
    a.lds_pL = a.lds_pD;
    a.lds_rhs = (int)(off - rb);
    off = rb + (size_t)std::max(1, nrhs) * (size_t)a.lds_rhs;
    if (off > lds_max) return 0;
    a.lds_total = (int)off;
    return a.lds_total;
}

// Right-hand sides a solve advances together (0 in the parameters means 1).
int nrhs_of(const hk_params* p) { return p->nrhs > 1 ? p->nrhs : 1; }

Space range_space(int64_t len, int G)
{
    Space sp{};
    sp.kind = 1;
    sp.len = (int)len;
    sp.ntile = G;
    return sp;
}

Plan plan_solve(const hk_op* op, const hk_params* p, int rect, int max_blocks, size_t lds_max)
{
    Plan pl;
    const int tb = p->basis_dtype;
    // pivot blocks: a persistent LDS copy of each if they fit, else one
    // buffer loaded before each substitution
    // (CSR row pointers are staged in LDS too when they fit)
    auto layout = [&](int ept, int TY, int TX, int r, int opk) {
        for (int pmode = 0; pmode < 2; ++pmode) {
            for (int rps = 1; rps >= 0; --rps) {
                lds_layout(pl.lds, kp1_of(p), p->s, ept, rect, opk, TY, TX, r, op->ntap, tb, pmode, rps);
                if ((size_t)pl.lds.lds_total <= lds_max) {
                    pl.lds_total = pl.lds.lds_total;
                    return;
                }
            }
        }
        pl.lds_total = pl.lds.lds_total;
    };
    const int kp1 = p->k + 1;
    const int G_cap = std::max(1, std::min(max_blocks, MAXG));
    if (op->kind == OP_BLUR) {
        // 2-D tiles: area ~ n / #CU rounded to a power of two, >= 64
        const int64_t n = op->n;
        int64_t area = 64;
        while (area * G_cap < n) area *= 2;
        for (; area <= (int64_t)NT * MAX_EPT; area *= 2) {
            int lg = 0;
            while ((int64_t(1) << (lg + 1)) <= area) ++lg;
            int TX = 1 << ((lg + 1) / 2), TY = 1 << (lg / 2);
            TX = std::min<int>(TX, std::max(1, op->nx));
            while ((int64_t)TX * TY < area && TY < op->ny) TY *= 2;
            const int ntx = (op->nx + TX - 1) / TX, nty = (op->ny + TY - 1) / TY;
            const int G = ntx * nty;
            if (G > G_cap) continue;
            Space sp{};
            sp.kind = 0; sp.len = (int)n; sp.ntile = G;
            sp.ny = op->ny; sp.nx = op->nx; sp.TY = TY; sp.TX = TX; sp.ntx = ntx;
            pl.spm = pl.spn = sp;
            pl.G = G;
            pl.ept = (TY * TX + NT - 1) / NT;
            if (pl.ept > 2) pl.ept = 4;
            const int tabs = p->sketch == HK_SKETCH_SPARSE_SIGN ? p->zeta : 0;   // sparse-sign row lists
            if (lds_layout_onebar(pl.lds, p->k, p->s, pl.ept, TY, TX, op->r, op->ntap, tb, tabs, nrhs_of(p),
                                  lds_max)) {
                pl.kernel = OP_BLUR_ONEBAR;
                pl.lds_total = pl.lds.lds_total;
                pl.spx = spx_of(op->r, TX);
                pl.nslot = nslot_of(op->r, TY, TX);
            } else if (tb == HK_BF16 || tb == HK_F16) {
                pl.why = "16-bit bases need the single-barrier blur kernel, whose LDS plan does not fit";
                return pl;
            } else if (nrhs_of(p) > 1) {
                pl.why = "the right-hand sides' state does not fit the single-barrier kernel's LDS "
                         "(fewer right-hand sides or a smaller k)";
                return pl;
            } else {
                pl.kernel = OP_BLUR;
                layout(pl.ept, TY, TX, op->r, OP_BLUR);
            }
            pl.ok = true;
            return pl;
        }
        pl.why = "image too large for one tile per compute unit";
        return pl;
    }
    // CSR: contiguous row ranges; both spaces share the workgroup count
    const int64_t lmax = rect ? std::max(op->m, op->n) : op->m;
    const int64_t lmin = rect ? std::min(op->m, op->n) : op->m;
    int G = (int)std::min<int64_t>(G_cap, lmin);
    if (G >= 8) G -= G % 8;
    const int64_t per = (lmax + G - 1) / G;
    if (per > (int64_t)NT * MAX_EPT) {
        pl.why = "operator too large for one tile per compute unit";
        return pl;
    }
    pl.G = G;
    pl.kernel = OP_CSR;
    pl.spm = range_space(op->m, G);
    pl.spn = rect ? range_space(op->n, G) : pl.spm;
    pl.ept = (int)((per + NT - 1) / NT);
    if (pl.ept > 2) pl.ept = 4;
    layout(pl.ept, 0, 0, 0, OP_CSR);
    pl.ok = true;
    return pl;
}

hk_status validate(const hk_op* op, const hk_params* p, int* rect)
{
    if (!op || !p) return fail(HK_EINVAL, "null operator or parameters");
    if (p->flags & ~(uint32_t)HK_FLAG_TRACE) return fail(HK_EINVAL, "unknown flags 0x%x", p->flags);
    if (p->k < 1) return fail(HK_EINVAL, "k must be >= 1 (got %d)", p->k);
    if (p->k > KMAX) return fail(HK_EUNSUPPORTED, "k = %d exceeds the supported maximum %d", p->k, KMAX);
    if (p->k > std::min(op->m, op->n)) return fail(HK_EINVAL, "k = %d exceeds min(m, n)", p->k);
    if (p->sketch != HK_SKETCH_NONE && p->s < p->k + 1)
        return fail(HK_EINVAL, "sketch size s = %d must be >= k + 1 = %d", p->s, p->k + 1);
    if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return fail(HK_EINVAL, "lambda must be finite and >= 0");
    if (p->sketch != HK_SKETCH_GAUSSIAN && p->sketch != HK_SKETCH_SPARSE_SIGN && p->sketch != HK_SKETCH_NONE)
        return fail(HK_EINVAL, "unknown sketch type %d", p->sketch);
    if (p->sketch == HK_SKETCH_SPARSE_SIGN && (p->zeta < 1 || p->zeta > p->s))
        return fail(HK_EINVAL, "zeta = %d must be in [1, s]", p->zeta);
    if (p->max_workgroups < 0) return fail(HK_EINVAL, "max_workgroups must be >= 0");
    if (p->pivot_sample < 0 || p->pivot_sample > SAMPLE_MAX)
        return fail(HK_EINVAL, "pivot_sample = %d must be in [0, %d]", p->pivot_sample, SAMPLE_MAX);
    if (p->nrhs < 0 || p->nrhs > RMAX) return fail(HK_EINVAL, "nrhs = %d must be in [0, %d]", p->nrhs, RMAX);
    if (p->nrhs > 1) {
        if (op->kind != OP_BLUR)
            return fail(HK_EUNSUPPORTED, "several right-hand sides are implemented for blur operators");
        if (p->pivot_sample > 0)
            return fail(HK_EUNSUPPORTED, "several right-hand sides take full partial pivoting");
        if (p->basis_dtype != HK_F64 && p->basis_dtype != HK_F32)
            return fail(HK_EUNSUPPORTED, "several right-hand sides need FP64 or FP32 bases");
    }
    if (p->sketch != HK_SKETCH_NONE && p->s > 16384)
        return fail(HK_EUNSUPPORTED, "sketch size s = %d exceeds 16384", p->s);
    if (p->basis_dtype < HK_F64 || p->basis_dtype > HK_F16)
        return fail(HK_EINVAL, "unknown basis dtype %d", p->basis_dtype);
    if (p->basis_dtype == HK_F32 && op->dtype == HK_F64)
        return fail(HK_EUNSUPPORTED, "FP32 bases need an FP32 operator");
    if ((p->basis_dtype == HK_BF16 || p->basis_dtype == HK_F16) && (op->dtype != HK_F32 || op->kind != OP_BLUR))
        return fail(HK_EUNSUPPORTED, "16-bit bases are implemented for FP32 blur operators");
    int r = 0;
    if (p->method == HK_METHOD_AUTO) r = (op->m != op->n);
    else if (p->method == HK_METHOD_HESSENBERG) r = 0;
    else if (p->method == HK_METHOD_CHANGING_HESSENBERG) r = 1;
    else return fail(HK_EINVAL, "unknown method %d", p->method);
    if (!r && op->m != op->n) return fail(HK_EINVAL, "the Hessenberg method needs a square operator");
    if (r && op->kind != OP_CSR)
        return fail(HK_EUNSUPPORTED, "the generalized Hessenberg method needs A^T: use a CSR operator");
    *rect = r;
    return HK_OK;
}

// Workgroups the basis kernel may use: the compute units, or fewer when the
// caller caps the grid (so that several solves can run side by side).
int grid_cap(const hk_context* ctx, const hk_params* p)
{
    return p->max_workgroups > 0 ? std::min(ctx->ncu, p->max_workgroups) : ctx->ncu;
}

// Block sketch of `ncol` columns of length `len` by s rows: 64 x 64 output
// tiles times chunks of the contraction, about 1024 workgroups in all for
// `ncol_ref` columns (0: ncol).  The chunks fix the order in which each
// entry's sum is formed, so several right-hand sides' columns (ncol_ref =
// one right-hand side's) are summed exactly as a single one's.
BskArgs bsk_plan(int64_t len, int ncol, int s, int ncol_ref = 0)
{
    BskArgs b{};
    b.len = (int)len;
    b.ncol = ncol;
    b.s = s;
    b.rt = (s + 63) / 64;
    b.ct = (ncol + 63) / 64;
    const int ct_ref = ((ncol_ref > 0 ? ncol_ref : ncol) + 63) / 64;
    const int64_t kc0 = std::max<int64_t>(1, (1024 + b.rt * ct_ref - 1) / (b.rt * ct_ref));
    const int64_t per = (len + kc0 - 1) / kc0;
    b.chunk = (int)std::max<int64_t>(16, (per + 15) / 16 * 16);
    b.kc = (int)((len + b.chunk - 1) / b.chunk);
    b.ldo = s;
    b.scale = 1.0 / std::sqrt((double)s);
    return b;
}

size_t bsk_tiles(int64_t len, int ncol, int s, int ncol_ref = 0)
{
    const BskArgs b = bsk_plan(len, ncol, s, ncol_ref);
    return (size_t)b.rt * b.ct * b.kc;
}

// The parameters a solve runs with: without a sketch the small problem has
// the k + 1 rows of H_{k+1,k}, so s = k + 1 (and no sparse-sign columns).
hk_params effective_params(const hk_params& p)
{
    hk_params e = p;
    if (e.sketch == HK_SKETCH_NONE) {
        e.s = e.k + 1;
        e.zeta = 0;
    }
    return e;
}

struct WsLayout {
    size_t ctl, L, D, H, W, tp, gp, PD, PL, pvD, pvL, amv, ami, zpart, fpart, cpart, Z, F, c;
    size_t Q, R, r, y, yp, res, d, xpart, trace, scale, wpart, sval, sidx, T, T1, call, part, total;
    size_t region;          // bytes of one right-hand side's region (regions first, side by side)
    int trace_cap;
    int64_t ldl, ldd;
};

WsLayout ws_layout(const hk_op* op, const hk_params* p, int rect, int G, int nslot)
{
    WsLayout w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const int k = p->k, kp1 = k + 1, s = p->s;
    const size_t es = dsize(p->basis_dtype);
    w.ldl = (int64_t)align_up((size_t)op->n, 64);
    w.ldd = (int64_t)align_up((size_t)op->m, 64);
    const int rows = p->lambda > 0.0 ? 2 * s : s;
    w.ctl = take(sizeof(Ctl));
    w.H = take(sizeof(double) * (size_t)kp1 * k);
    w.W = take(sizeof(double) * (size_t)k * k);
    w.tp = take(sizeof(int) * kp1);
    w.gp = take(sizeof(int) * kp1);
    w.PD = rect ? take(es * (size_t)kp1 * kp1) : 0;
    w.PL = take(es * (size_t)kp1 * kp1);
    w.pvD = take(sizeof(double) * kp1);
    w.pvL = take(sizeof(double) * kp1);
    w.amv = take(sizeof(double) * 2 * G);
    w.ami = take(sizeof(int) * 2 * G);
    w.zpart = take(sizeof(long long) * 2 * (size_t)G * s);     // two parities
    w.fpart = take(sizeof(long long) * 2 * (size_t)G * s);
    w.cpart = take(sizeof(long long) * (size_t)G * s);
    w.Z = take(sizeof(double) * (size_t)s * k);
    w.F = take(sizeof(double) * (size_t)s * k);
    w.c = take(sizeof(double) * s);
    w.Q = take(sizeof(double) * (size_t)rows * k);
    w.R = take(sizeof(double) * (size_t)k * k);
    w.r = take(sizeof(double) * rows);
    w.y = take(sizeof(double) * k);
    w.yp = take(sizeof(double) * k);
    w.res = take(sizeof(double) * k);
    w.d = take(sizeof(double) * k);
    w.xpart = take(sizeof(double) * 2 * (size_t)small_ls_wgs(s, p->lambda) * ls_xcap(k));
    w.trace_cap = (p->flags & HK_FLAG_TRACE) ? 2 * (6 * kp1 + 8) + 16 * (kp1 + 1) : 0;
    w.trace = take(sizeof(unsigned long long) * (size_t)std::max(1, w.trace_cap + (w.trace_cap ? ARR_SLOTS + LS_TRACE : 0)));
    w.scale = take(sizeof(double) * kp1);
    w.wpart = take(sizeof(double) * 2 * (size_t)kp1 * std::max(1, nslot));
    w.sval = take(sizeof(double) * 4 * SAMPLE_SLOTS);
    w.sidx = take(sizeof(int) * 4 * SAMPLE_SLOTS);
    // one region per right-hand side, then what they share: the
    // end-of-solve block sketches of all their bases and b's, and the bases
    const int nr = nrhs_of(p);
    w.region = off;
    off = w.region * (size_t)nr;
    if (p->sketch == HK_SKETCH_GAUSSIAN && (p->basis_dtype == HK_F64 || p->basis_dtype == HK_F32)) {   // end-of-solve block sketches
        const int nc = nr * kp1;
        w.T = take(sizeof(double) * (size_t)s * nc);
        w.T1 = take(sizeof(double) * (size_t)s * nc);
        w.call = take(sizeof(double) * (size_t)s * nr);
        const int64_t lz = rect ? op->m : op->n;
        const size_t tiles = std::max(std::max(bsk_tiles(lz, nc, s, kp1), bsk_tiles(op->m, nr, s, 1)),
                                      bsk_tiles(op->n, nc, s, kp1));
        w.part = take(sizeof(double) * 4096 * tiles);
    }
    // the bases last: every column a run reads it has written first, so a
    // reused workspace needs only [0, L) cleared
    w.L = take(es * (size_t)w.ldl * kp1 * nr);
    w.D = rect ? take(es * (size_t)w.ldd * kp1) : 0;
    w.total = off;
    return w;
}

hk_status current_device(hk_context* ctx)
{
    HIP_TRY(hipSetDevice(ctx->device));
    return HK_OK;
}

}  // namespace

static hk_status op_apply_on(hk_op* op, int transpose, const void* x_dev, void* y_dev, hipStream_t st);

// ====================================================================== ABI
extern "C" {

int32_t hk_abi_version(void) { return HK_ABI_VERSION; }

const char* hk_last_error(void) { return g_err.c_str(); }

hk_status hk_context_create(int32_t device, void* stream, hk_context** out)
{
    if (!out) return fail(HK_EINVAL, "null output handle");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(HK_EINVAL, "device %d out of range (%d devices)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    auto* c = new (std::nothrow) hk_context;
    if (!c) return fail(HK_ENOMEM, "host allocation failed");
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->ncu = prop.multiProcessorCount;
    c->lds_max = prop.sharedMemPerBlock;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) == hipSuccess && rate > 0)
        c->wall_rate_khz = (unsigned long long)rate;
    scratch_setup(device);    // the no-alloc entry point's workspace on this device
    live_add(c);
    *out = c;
    return HK_OK;
}

hk_status hk_context_destroy(hk_context* ctx)
{
    if (!live_take(ctx)) return fail(HK_EINVAL, ctx ? "unknown or destroyed context" : "null context");
    delete ctx;
    return HK_OK;
}

static void op_free(hk_op* op)
{
    if (!op) return;
    hipFree(op->d_taps);
    hipFree(op->d_toff);
    hipFree(op->d_tw);
    hipFree(op->d_rp);
    hipFree(op->d_ci);
    hipFree(op->d_cv);
    hipFree(op->d_rpt);
    hipFree(op->d_cit);
    hipFree(op->d_cvt);
    for (auto& pt : op->parts) hipFree(pt.d);
    delete op;
}

// Row ranges of G tiles of about equal weight nnz_i + alpha per row, alpha =
// beta times the mean row length (at least 1), every tile non-empty: tile t
// holds [st[t], st[t + 1]).  With C(i) = rp[i] + alpha i and the cut st[t] =
// the first i with C(i) >= t W / G (W = C(len)), a tile [a, b) has
// C(b - 1) - C(a) < W / G, so fewer than (nnz / alpha + len) / G + 1 rows
// (about twice the mean for beta = 1); the clamps that keep every tile
// non-empty can only matter for a few huge rows, and the caller checks the
// largest tile against the plan.
static bool balanced_ranges(const std::vector<int64_t>& rp, int G, double beta, std::vector<int>& st, int& maxrows)
{
    const int64_t len = (int64_t)rp.size() - 1;
    if (G < 1 || len < G) return false;
    const double alpha = std::max(1.0, beta * (double)rp[len] / (double)len);
    const double W = (double)rp[len] + alpha * (double)len;
    st.assign((size_t)G + 1, 0);
    st[G] = (int)len;
    int64_t lo = 0;
    for (int t = 1; t < G; ++t) {
        const double target = W * t / G;
        // the smallest i in [lo + 1, len - (G - t)] with rp[i] + alpha i >= target
        int64_t a = lo + 1, b = len - (G - t);
        while (a < b) {
            const int64_t mid = (a + b) / 2;
            if ((double)rp[mid] + alpha * (double)mid >= target) b = mid;
            else a = mid + 1;
        }
        st[t] = (int)a;
        lo = a;
    }
    maxrows = 0;
    for (int t = 0; t < G; ++t) maxrows = std::max(maxrows, st[t + 1] - st[t]);
    return true;
}

// Balanced tile ranges of a CSR operator for a plan of G tiles of at most
// NT * ept rows, cached on the operator.  Computed, and their device copy
// allocated, only when may_alloc; nullptr when there are none (the plan then
// keeps equal row ranges).
static const int* csr_partition(hk_op* op, int G, int ept, int rect, bool may_alloc)
{
    std::lock_guard<std::mutex> lk(op->part_mu);
    for (const auto& pt : op->parts)
        if (pt.G == G && pt.ept == ept) return pt.d;
    if (!may_alloc) return nullptr;
    hk_op::CsrPart cp;
    cp.G = G;
    cp.ept = ept;
    const int cap = NT * ept;
    std::vector<int> sm, sn;
    for (double beta : {1.0, 2.0, 4.0}) {
        int mm = 0, mn = 0;
        if (!balanced_ranges(op->h_rp, G, beta, sm, mm)) break;
        if (rect && !balanced_ranges(op->h_rpt, G, beta, sn, mn)) break;
        if (mm > cap || (rect && mn > cap)) continue;
        if (!rect) sn = sm;
        int* d = nullptr;
        if (hipMalloc(&d, sizeof(int) * 2 * ((size_t)G + 1)) != hipSuccess) break;
        if (hipMemcpy(d, sm.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d + G + 1, sn.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice) != hipSuccess) {
            hipFree(d);
            break;
        }
        cp.d = d;
        break;
    }
    op->parts.push_back(cp);
    return cp.d;
}

hk_status hk_op_create_blur(hk_context* ctx, int64_t ny, int64_t nx, const double* taps_y,
                            const double* taps_x, int32_t radius, hk_bc bc, hk_dtype dt, hk_op** out)
{
    HK_LIVE(ctx);
    if (!out) return fail(HK_EINVAL, "null output handle");
    *out = nullptr;
    if (!ctx || !taps_y || !taps_x) return fail(HK_EINVAL, "null argument");
    if (ny < 1 || nx < 1 || ny * nx > (int64_t)1 << 30) return fail(HK_EINVAL, "bad image size %lld x %lld", (long long)ny, (long long)nx);
    if (radius < 0 || radius > 64) return fail(HK_EINVAL, "radius %d outside [0, 64]", radius);
    if (bc != HK_BC_ZERO && bc != HK_BC_REFLECT) return fail(HK_EINVAL, "unknown boundary condition %d", bc);
    if (dt != HK_F64 && dt != HK_F32) return fail(HK_EINVAL, "unknown dtype %d", dt);
    if (bc == HK_BC_REFLECT && (radius > ny || radius > nx))
        return fail(HK_EINVAL, "reflective boundary needs radius <= image size");
    double sy = 0.0, sx = 0.0;
    for (int i = 0; i <= 2 * radius; ++i) {
        if (!std::isfinite(taps_y[i]) || !std::isfinite(taps_x[i])) return fail(HK_ENUMERIC, "non-finite PSF tap");
        sy += std::fabs(taps_y[i]);
        sx += std::fabs(taps_x[i]);
    }
    hk_status st = current_device(ctx);
    if (st) return st;
    auto* op = new (std::nothrow) hk_op;
    if (!op) return fail(HK_ENOMEM, "host allocation failed");
    op->ctx = ctx;
    op->kind = OP_BLUR;
    op->m = op->n = ny * nx;
    op->dtype = dt;
    op->ny = (int)ny; op->nx = (int)nx; op->r = radius; op->bc = bc;
    op->anorm = op->anorm_t = sy * sx;
    const size_t nt = 2 * (size_t)radius + 1;
    if (hipMalloc(&op->d_taps, sizeof(double) * 2 * nt) != hipSuccess) { op_free(op); return fail(HK_ENOMEM, "hipMalloc failed"); }
    std::vector<double> taps(2 * nt);
    std::copy(taps_y, taps_y + nt, taps.begin());
    std::copy(taps_x, taps_x + nt, taps.begin() + nt);
    if (hipMemcpy(op->d_taps, taps.data(), sizeof(double) * 2 * nt, hipMemcpyHostToDevice) != hipSuccess) {
        op_free(op);
        return fail(HK_EDEVICE, "hipMemcpy failed");
    }
    live_add(op);
    *out = op;
    return HK_OK;
}

hk_status hk_op_create_gaussian_blur(hk_context* ctx, int64_t ny, int64_t nx, double sigma,
                                     int32_t radius, hk_bc bc, hk_dtype dt, hk_op** out)
{
    HK_LIVE(ctx);
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(HK_EINVAL, "sigma must be positive");
    if (radius < 0 || radius > 64) return fail(HK_EINVAL, "radius %d outside [0, 64]", radius);
    std::vector<double> g(2 * (size_t)radius + 1);
    double sum = 0.0;
    for (int a = -radius; a <= radius; ++a) {
        g[a + radius] = std::exp(-(double)a * a / (2.0 * sigma * sigma));
        sum += g[a + radius];
    }
    for (double& v : g) v /= sum;
    return hk_op_create_blur(ctx, ny, nx, g.data(), g.data(), radius, bc, dt, out);
}

hk_status hk_op_create_blur_psf(hk_context* ctx, int64_t ny, int64_t nx, const double* psf, int32_t radius,
                                hk_bc bc, hk_dtype dt, hk_op** out)
{
    HK_LIVE(ctx);
    if (!out) return fail(HK_EINVAL, "null output handle");
    *out = nullptr;
    if (!ctx || !psf) return fail(HK_EINVAL, "null argument");
    if (radius < 0 || radius > 64) return fail(HK_EINVAL, "radius %d outside [0, 64]", radius);
    const int w = 2 * radius + 1;
    double pmax = 0.0;
    int a0 = 0, b0 = 0;
    for (int a = 0; a < w; ++a)
        for (int b = 0; b < w; ++b) {
            const double v = psf[(size_t)a * w + b];
            if (!std::isfinite(v)) return fail(HK_ENUMERIC, "non-finite PSF entry at (%d, %d)", a, b);
            if (std::fabs(v) > pmax) { pmax = std::fabs(v); a0 = a; b0 = b; }
        }
    // A PSF of rank one, p(a, b) = ty(a) tx(b) to rounding, takes the
    // separable path: ty(a) = p(a, b0) / p(a0, b0), tx(b) = p(a0, b)
    if (pmax > 0.0) {
        std::vector<double> ty(w), tx(w);
        for (int a = 0; a < w; ++a) ty[a] = psf[(size_t)a * w + b0] / psf[(size_t)a0 * w + b0];
        for (int b = 0; b < w; ++b) tx[b] = psf[(size_t)a0 * w + b];
        bool sep = true;
        for (int a = 0; a < w && sep; ++a)
            for (int b = 0; b < w; ++b)
                if (std::fabs(ty[a] * tx[b] - psf[(size_t)a * w + b]) > 4.0 * DBL_EPSILON * pmax) { sep = false; break; }
        if (sep) return hk_op_create_blur(ctx, ny, nx, ty.data(), tx.data(), radius, bc, dt, out);
    }
    // the nonzero entries as a tap list
    std::vector<int> toff;
    std::vector<double> tw;
    double asum = 0.0;
    for (int a = 0; a < w; ++a)
        for (int b = 0; b < w; ++b) {
            const double v = psf[(size_t)a * w + b];
            if (v == 0.0) continue;
            toff.push_back((a << 16) | b);
            tw.push_back(v);
            asum += std::fabs(v);
        }
    if ((int)toff.size() > HK_PSF_MAX_TAPS)
        return fail(HK_EUNSUPPORTED, "the PSF has %zu nonzero entries; at most %d are supported", toff.size(),
                    HK_PSF_MAX_TAPS);
    if (toff.empty()) {   // the zero operator: one zero tap keeps the list nonempty
        toff.push_back((radius << 16) | radius);
        tw.push_back(0.0);
    }
    // the separable creation checks the image, boundary and dtype; then the
    // taps are replaced by the list
    std::vector<double> unit(w, 0.0);
    unit[radius] = 1.0;
    hk_op* op = nullptr;
    hk_status st = hk_op_create_blur(ctx, ny, nx, unit.data(), unit.data(), radius, bc, dt, &op);
    if (st) return st;
    op->ntap = (int)toff.size();
    op->anorm = op->anorm_t = asum;
    bool ok = hipMalloc(&op->d_toff, sizeof(int) * toff.size()) == hipSuccess &&
              hipMalloc(&op->d_tw, sizeof(double) * tw.size()) == hipSuccess;
    if (!ok) { live_take(op); op_free(op); return fail(HK_ENOMEM, "hipMalloc failed"); }
    ok = hipMemcpy(op->d_toff, toff.data(), sizeof(int) * toff.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(op->d_tw, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) { live_take(op); op_free(op); return fail(HK_EDEVICE, "hipMemcpy failed"); }
    live_add(op);
    *out = op;
    return HK_OK;
}

hk_status hk_op_create_csr(hk_context* ctx, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                           const int32_t* col, const void* val, hk_dtype dt, hk_op** out)
{
    HK_LIVE(ctx);
    if (!out) return fail(HK_EINVAL, "null output handle");
    *out = nullptr;
    if (!ctx || !rowptr || (nnz > 0 && (!col || !val))) return fail(HK_EINVAL, "null argument");
    if (m < 1 || n < 1 || m >= ((int64_t)1 << 31) || n >= ((int64_t)1 << 31) || nnz < 0)
        return fail(HK_EINVAL, "bad CSR shape m=%lld n=%lld nnz=%lld", (long long)m, (long long)n, (long long)nnz);
    if (dt != HK_F64 && dt != HK_F32) return fail(HK_EINVAL, "unknown dtype %d", dt);
    if (rowptr[0] != 0 || rowptr[m] != nnz) return fail(HK_EINVAL, "rowptr must start at 0 and end at nnz");
    for (int64_t i = 0; i < m; ++i)
        if (rowptr[i + 1] < rowptr[i]) return fail(HK_EINVAL, "rowptr decreases at row %lld", (long long)i);
    for (int64_t p = 0; p < nnz; ++p)
        if (col[p] < 0 || col[p] >= n) return fail(HK_EINVAL, "column index out of range at %lld", (long long)p);
    const size_t es = dsize(dt);
    auto valat = [&](int64_t p) -> double {
        return dt == HK_F64 ? ((const double*)val)[p] : (double)((const float*)val)[p];
    };
    // A^T by counting sort (stable: row order within each column)
    std::vector<int64_t> rpt(n + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) rpt[col[p] + 1]++;
    for (int64_t c = 0; c < n; ++c) rpt[c + 1] += rpt[c];
    std::vector<int32_t> cit(nnz);
    std::vector<unsigned char> cvt(es * (size_t)nnz);
    std::vector<int64_t> fill(rpt.begin(), rpt.end() - 1);
    double anorm = 0.0;
    std::vector<double> colsum(n, 0.0);
    for (int64_t i = 0; i < m; ++i) {
        double rs = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const double v = valat(p);
            if (!std::isfinite(v)) return fail(HK_ENUMERIC, "non-finite matrix entry at %lld", (long long)p);
            rs += std::fabs(v);
            colsum[col[p]] += std::fabs(v);
            const int64_t q = fill[col[p]]++;
            cit[q] = (int32_t)i;
            std::memcpy(&cvt[es * q], (const unsigned char*)val + es * p, es);
        }
        anorm = std::max(anorm, rs);
    }
    double anorm_t = 0.0;
    for (double v : colsum) anorm_t = std::max(anorm_t, v);

    hk_status st = current_device(ctx);
    if (st) return st;
    auto* op = new (std::nothrow) hk_op;
    if (!op) return fail(HK_ENOMEM, "host allocation failed");
    op->ctx = ctx;
    op->kind = OP_CSR;
    op->m = m; op->n = n; op->nnz = nnz; op->dtype = dt;
    op->anorm = anorm; op->anorm_t = anorm_t;
    op->lpr = lanes_per_row((double)nnz / (double)m);
    op->lprt = lanes_per_row((double)nnz / (double)n);
    op->h_rp.assign(rowptr, rowptr + m + 1);
    op->h_rpt = rpt;
    const size_t nb = std::max<int64_t>(nnz, 1);
    bool ok = hipMalloc(&op->d_rp, sizeof(int64_t) * (m + 1)) == hipSuccess &&
              hipMalloc(&op->d_ci, sizeof(int32_t) * nb) == hipSuccess &&
              hipMalloc(&op->d_cv, es * nb) == hipSuccess &&
              hipMalloc(&op->d_rpt, sizeof(int64_t) * (n + 1)) == hipSuccess &&
              hipMalloc(&op->d_cit, sizeof(int32_t) * nb) == hipSuccess &&
              hipMalloc(&op->d_cvt, es * nb) == hipSuccess;
    if (!ok) { op_free(op); return fail(HK_ENOMEM, "hipMalloc failed for the CSR arrays"); }
    ok = hipMemcpy(op->d_rp, rowptr, sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(op->d_rpt, rpt.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice) == hipSuccess;
    if (ok && nnz > 0)
        ok = hipMemcpy(op->d_ci, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(op->d_cv, val, es * nnz, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(op->d_cit, cit.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(op->d_cvt, cvt.data(), es * nnz, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) { op_free(op); return fail(HK_EDEVICE, "hipMemcpy failed for the CSR arrays"); }
    live_add(op);
    *out = op;
    return HK_OK;
}

hk_status hk_op_shape(const hk_op* op, int64_t* m, int64_t* n)
{
    HK_LIVE(op);
    if (!op) return fail(HK_EINVAL, "null operator");
    if (m) *m = op->m;
    if (n) *n = op->n;
    return HK_OK;
}

hk_status hk_op_apply(hk_op* op, int32_t transpose, const void* x_dev, void* y_dev)
{
    HK_LIVE(op);
    if (!op || !x_dev || !y_dev) return fail(HK_EINVAL, "null argument");
    if (transpose && op->kind != OP_CSR) return fail(HK_EUNSUPPORTED, "A^T products are provided for CSR operators");
    hk_status st = current_device(op->ctx);
    if (st) return st;
    return op_apply_on(op, transpose, x_dev, y_dev, op->ctx->stream);
}

}  // extern "C"

// y = A x (or A^T x) on stream st, in the operator's own product kernel.
static hk_status op_apply_on(hk_op* op, int transpose, const void* x_dev, void* y_dev, hipStream_t st)
{
    ApplyArgs a{};
    a.transpose = transpose;
    a.x = x_dev;
    a.y = y_dev;
    int ept = 1;
    if (op->kind == OP_BLUR) {
        Space sp{};
        sp.kind = 0; sp.len = (int)op->n; sp.ny = op->ny; sp.nx = op->nx;
        sp.TX = std::min(32, op->nx);
        sp.TY = 16;
        sp.ntx = (op->nx + sp.TX - 1) / sp.TX;
        sp.ntile = sp.ntx * ((op->ny + sp.TY - 1) / sp.TY);
        a.sp = sp;
        a.ny = op->ny; a.nx = op->nx; a.r = op->r; a.bc = op->bc;
        a.taps_y = op->d_taps;
        a.taps_x = op->d_taps ? op->d_taps + 2 * op->r + 1 : nullptr;
        a.toff = op->d_toff;
        a.tw = op->d_tw;
        a.ntap = op->ntap;
        size_t off = 0;
        auto take = [&](size_t b) { size_t o = off; off = align_up(off + b, 16); return (int)o; };
        const int SW = sp.TX + 2 * op->r, SH = sp.TY + 2 * op->r;
        a.lds_w = take(sizeof(double) * sp.TY * sp.TX);
        a.lds_stage = take(dsize(op->dtype) * (size_t)SW * SH);
        a.lds_vert = take(sizeof(double) * (size_t)sp.TY * SW);
        a.lds_taps = take(psf_lds_bytes(op->r, op->ntap));
        a.lds_total = (int)off;
        if ((size_t)a.lds_total > op->ctx->lds_max) return fail(HK_EUNSUPPORTED, "blur radius too large for LDS");
    } else {
        const int64_t len = transpose ? op->n : op->m;
        const int per = 256;
        Space sp = range_space(len, (int)((len + per - 1) / per));
        a.sp = sp;
        a.rp = transpose ? op->d_rpt : op->d_rp;
        a.ci = transpose ? op->d_cit : op->d_ci;
        a.cv = transpose ? op->d_cvt : op->d_cv;
        a.lpr = transpose ? op->lprt : op->lpr;
        a.lds_w = 0;
        a.lds_total = (int)(sizeof(double) * per);
    }
    HIP_TRY(launch_apply(op->dtype, op->kind, ept, a, st));
    return HK_OK;
}

extern "C" {

hk_status hk_op_destroy(hk_op* op)
{
    if (!live_take(op)) return fail(HK_EINVAL, op ? "unknown or destroyed operator" : "null operator");
    hipSetDevice(op->ctx->device);
    op_free(op);
    return HK_OK;
}

static hk_status max_blocks(const hk_op* op, const hk_params* p, int rect, Plan* out)
{
    // probe occupancy with the LDS of the plan at #CU blocks; shrink if needed
    const hk_context* ctx = op->ctx;
    Plan pl = plan_solve(op, p, rect, grid_cap(ctx, p), ctx->lds_max - 1024);   // 1 KB: static LDS of the kernels
    if (!pl.ok) return fail(HK_EUNSUPPORTED, "%s", pl.why.c_str());
    if ((size_t)pl.lds_total > ctx->lds_max)
        return fail(HK_EUNSUPPORTED, "LDS need %d B exceeds the device limit %zu B", pl.lds_total, ctx->lds_max);
    int per_cu = 0;
    hipError_t e = iterate_occupancy(p->basis_dtype, op->dtype, pl.kernel,
                                     p->sketch == HK_SKETCH_SPARSE_SIGN ? SK_SPARSE : SK_GAUSS, pl.ept,
                                     p->pivot_sample > 0 ? 1 : 0, pl.lds_total, &per_cu);
    if (e != hipSuccess) return fail(HK_EDEVICE, "occupancy query failed: %s", hipGetErrorString(e));
    if (per_cu < 1) return fail(HK_EUNSUPPORTED, "the basis kernel does not fit on a compute unit");
    if (pl.G > per_cu * ctx->ncu) return fail(HK_EUNSUPPORTED, "grid of %d exceeds co-resident capacity", pl.G);
    *out = pl;
    return HK_OK;
}

hk_status hk_solve_workspace_bytes(const hk_op* op, const hk_params* p_in, size_t* bytes)
{
    HK_LIVE(op);
    if (!bytes) return fail(HK_EINVAL, "null output");
    int rect = 0;
    hk_status st = validate(op, p_in, &rect);
    if (st) return st;
    const hk_params pe = effective_params(*p_in);
    const hk_params* p = &pe;
    Plan pl = plan_solve(op, p, rect, grid_cap(op->ctx, p), op->ctx->lds_max - 1024);
    if (!pl.ok) return fail(HK_EUNSUPPORTED, "%s", pl.why.c_str());
    *bytes = ws_layout(op, p, rect, pl.G, pl.nslot).total;
    return HK_OK;
}

}  // extern "C"

// Plan a solve: validated effective parameters, tiling and workspace size.
static hk_status solve_plan(hk_op* op, const hk_params* p_in, hk_params* pe, int* rect, Plan* pl, size_t* bytes)
{
    hk_status st = validate(op, p_in, rect);
    if (st) return st;
    *pe = effective_params(*p_in);
    st = current_device(op->ctx);
    if (st) return st;
    st = max_blocks(op, pe, *rect, pl);
    if (st) return st;
    *bytes = ws_layout(op, pe, *rect, pl->G, pl->nslot).total;
    return HK_OK;
}

// Fill a solve's arguments for the workspace at `base` (laid out as `w`).
static hk_status solve_bind(hk_solve* sv, hk_op* op, const hk_params* p, int rect, const Plan& pl,
                            const WsLayout& w, unsigned char* base, hipStream_t stream, bool may_alloc)
{
    sv->op = op;
    sv->prm = *p;
    sv->tb = p->basis_dtype;
    sv->rect = rect;
    sv->sk = p->sketch == HK_SKETCH_SPARSE_SIGN ? SK_SPARSE : SK_GAUSS;
    sv->ept = pl.ept;
    sv->kernel = pl.kernel;
    sv->G = pl.G;
    sv->stream = stream;
    sv->ws_bytes = w.total;
    KArgs& a = sv->ka;
    a = pl.lds;    // lds_* offsets
    a.m = (int)op->m; a.n = (int)op->n; a.k = p->k; a.s = p->s; a.zeta = p->zeta;
    a.lam = p->lambda;
    a.seed_lo = (uint32_t)(p->seed & 0xffffffffu);
    a.seed_hi = (uint32_t)(p->seed >> 32);
    a.rect = rect;
    a.nosk = (p->sketch == HK_SKETCH_NONE) ? 1 : 0;
    a.coop = p->max_workgroups > 0 ? 0 : 1;
    // The block sketch reads Z through the Hessenberg relation A L_k =
    // L_{k+1} H, which a stored basis satisfies to its rounding: FP64 and
    // FP32 bases use it; 16-bit bases keep the exact per-step z_j = S2 A l_j.
    sv->zend = (p->sketch == HK_SKETCH_GAUSSIAN) && (p->basis_dtype == HK_F64 || p->basis_dtype == HK_F32);
    a.stepsk = (p->sketch == HK_SKETCH_NONE || sv->zend) ? 0 : 1;
    a.psamp = p->pivot_sample;
    a.pnc = (p->pivot_sample + 3) / 4 + 2;
    a.sval = (double*)(base + w.sval);
    a.sidx = (int*)(base + w.sidx);
    a.G = pl.G;
    a.xcd_map = (pl.G % 8 == 0) ? 1 : 0;
    a.spm = pl.spm;
    a.spn = pl.spn;
    if (pl.kernel == OP_CSR) {
        // CSR tiles balanced by nonzeros (plus a row term for the bases),
        // when the operator has (or may compute) ranges that fit the plan
        if (const int* st = csr_partition(op, pl.G, pl.ept, rect, may_alloc)) {
            a.spm.kind = 2;
            a.spm.st = st;
            a.spn.kind = 2;
            a.spn.st = rect ? st + pl.G + 1 : st;
        }
    }
    a.ny = op->ny; a.nx = op->nx; a.r = op->r; a.bc = op->bc;
    a.taps_y = op->d_taps;
    a.taps_x = op->d_taps ? op->d_taps + 2 * op->r + 1 : nullptr;
    a.toff = op->d_toff;
    a.tw = op->d_tw;
    a.ntap = op->ntap;
    a.rp = op->d_rp; a.ci = op->d_ci; a.cv = op->d_cv;
    a.rpt = op->d_rpt; a.cit = op->d_cit; a.cvt = op->d_cvt;
    a.lpr = op->lpr; a.lprt = op->lprt;
    a.scz = fx_scale((double)op->m * op->anorm * 1.000001);
    a.scf = fx_scale((double)op->n * 1.000001);
    a.L = base + w.L; a.ldl = w.ldl;
    a.D = rect ? base + w.D : nullptr; a.ldd = w.ldd;
    a.H = (double*)(base + w.H);
    a.W = (double*)(base + w.W);
    a.tp = (int*)(base + w.tp);
    a.gp = (int*)(base + w.gp);
    a.PD = rect ? base + w.PD : nullptr;
    a.PL = base + w.PL;
    a.pvD = (double*)(base + w.pvD);
    a.pvL = (double*)(base + w.pvL);
    a.amv = (double*)(base + w.amv);
    a.ami = (int*)(base + w.ami);
    a.zpart = (long long*)(base + w.zpart);
    a.fpart = (long long*)(base + w.fpart);
    a.cpart = (long long*)(base + w.cpart);
    a.Z = (double*)(base + w.Z);
    a.F = (double*)(base + w.F);
    a.c = (double*)(base + w.c);
    a.ctl = (Ctl*)(base + w.ctl);
    a.timeout_ticks = op->ctx->wall_rate_khz * 1000ull * 5ull;   // 5 s per barrier wait
    a.scale = (double*)(base + w.scale);
    a.wpart = (double*)(base + w.wpart);
    a.nslot = pl.nslot;
    a.spx = pl.spx;
    a.trace_cap = w.trace_cap;
    a.trace = w.trace_cap ? (unsigned long long*)(base + w.trace) : nullptr;
    const int nr = nrhs_of(p);
    sv->nrhs = nr;
    a.nrhs = nr;
    a.rhs_stride = (long long)w.region;
    a.lds_rhs = pl.lds.lds_rhs;
    sv->region = w.region;
    sv->call = a.c;
    if (sv->zend) {
        // one block contraction per sketch over every right-hand side's
        // basis (side by side in L) or b: S is generated once per 64
        // columns of the block, whatever the number of right-hand sides
        const uint32_t k0 = a.seed_lo, k1 = a.seed_hi;
        const int nc = nr * (p->k + 1);
        sv->T = (double*)(base + w.T);
        sv->T1 = (double*)(base + w.T1);
        sv->call = (double*)(base + w.call);
        double* part = (double*)(base + w.part);
        // T = S2 [d_1 .. d_{k+1}] (the data-space basis) of each right-hand side
        sv->bz = bsk_plan(rect ? op->m : op->n, nc, p->s, p->k + 1);
        sv->bz.q = rect ? a.D : a.L;
        sv->bz.ldq = rect ? a.ldd : a.ldl;
        sv->bz.stream = 2u; sv->bz.k0 = k0; sv->bz.k1 = k1;
        sv->bz.part = part;
        sv->bz.out = sv->T;
        // c = S2 b of each right-hand side (b is set per run)
        sv->bc = bsk_plan(op->m, nr, p->s, 1);
        sv->bc.ldq = op->m;
        sv->bc.stream = 2u; sv->bc.k0 = k0; sv->bc.k1 = k1;
        sv->bc.part = part;
        sv->bc.out = sv->call;
        // T1 = S1 [l_1 .. l_{k+1}] of each right-hand side (its first k
        // columns are F)
        sv->bf = bsk_plan(op->n, nc, p->s, p->k + 1);
        sv->bf.q = a.L;
        sv->bf.ldq = a.ldl;
        sv->bf.stream = 1u; sv->bf.k0 = k0; sv->bf.k1 = k1;
        sv->bf.part = part;
        sv->bf.out = sv->T1;
    }
    LsArgs& l = sv->la;
    l.s = p->s; l.k = p->k; l.lam = p->lambda;
    // unsketched: Z is H_{k+1,k} itself (column-major, leading dimension
    // k + 1 = s); F = [I; 0] and c = beta e_1 are written before the solve
    l.Z = a.nosk ? a.H : a.Z; l.F = a.F; l.c = a.c;
    l.Q = (double*)(base + w.Q);
    l.R = (double*)(base + w.R);
    l.r = (double*)(base + w.r);
    l.y = (double*)(base + w.y);
    sv->yp = (double*)(base + w.yp);
    l.res = (double*)(base + w.res);
    l.d = (double*)(base + w.d);
    l.ctl = a.ctl;
    l.trace = w.trace_cap ? a.trace + w.trace_cap + ARR_SLOTS : nullptr;
    l.nrhs = nr;
    l.rhs_stride = (long long)w.region;
    l.c = sv->call;                               // S2 b of right-hand side b: c_stride doubles further on
    l.c_stride = sv->zend ? p->s : (long long)(w.region / sizeof(double));
    CombineArgs& c = sv->ca;
    c.n = (int)op->n; c.k = p->k; c.L = a.L; c.ldl = a.ldl; c.y = l.y; c.ctl = a.ctl;
    c.rhs_stride = (long long)w.region;
    c.scale = (pl.kernel == OP_BLUR_ONEBAR) ? a.scale : nullptr;
    // the row-split least-squares kernel spreads the rows of [Z; lambda F]
    // over several workgroups; a capped grid (a share of the device, as in
    // the serving loop) keeps one workgroup per right-hand side
    l.xpart = (double*)(base + w.xpart);
    l.timeout = a.timeout_ticks;
    l.nwg = p->max_workgroups > 0 ? 1 : small_ls_wgs(p->s, p->lambda);
    l.nb = small_ls_panel(p->s, p->k, p->lambda, l.nwg, op->ctx->lds_max);
    if (l.nb == 0) l.nwg = 1;
    if (l.nb == 0 && (size_t)small_ls_lds_bytes(p->s, p->k, p->lambda) > op->ctx->lds_max)
        return fail(HK_EUNSUPPORTED, "sketch size too large for the least-squares kernel's LDS");
    return HK_OK;
}

// Frees a solve's events, its own workspace and the handle (no registry
// check: also for a solve whose creation failed).
static void solve_free(hk_solve* sv)
{
    hipSetDevice(sv->op->ctx->device);
    for (int i = 0; i < hk_solve::NEV; ++i)
        for (int q = 0; q < 3; ++q)
            if (sv->ev[i][q]) hipEventDestroy(sv->ev[i][q]);
    if (sv->own_ws) hipFree(sv->ws);
    delete sv;
}

// Create a solve.  ws: a device buffer of at least the planned size to use
// as workspace (zeroed on `stream`), or null to allocate one; nev: runs whose
// timing events are kept; stream: where runs are ordered.
static hk_status solve_create(hk_op* op, const hk_params* p_in, void* ws, size_t ws_cap, int nev,
                              hipStream_t stream, hk_solve** out)
{
    if (!out) return fail(HK_EINVAL, "null output handle");
    *out = nullptr;
    int rect = 0;
    hk_params pe{};
    Plan pl;
    size_t need = 0;
    hk_status st = solve_plan(op, p_in, &pe, &rect, &pl, &need);
    if (st) return st;
    const hk_params* p = &pe;
    const WsLayout w = ws_layout(op, p, rect, pl.G, pl.nslot);
    if (ws && ws_cap < w.total) return fail(HK_ENOMEM, "workspace of %zu bytes is smaller than %zu", ws_cap, w.total);
    auto* sv = new (std::nothrow) hk_solve;
    if (!sv) return fail(HK_ENOMEM, "host allocation failed");
    sv->op = op;
    sv->nev = std::max(1, std::min(nev, (int)hk_solve::NEV));
    if (ws) {
        sv->ws = ws;
        sv->own_ws = false;
    } else if (hipMalloc(&sv->ws, w.total) != hipSuccess) {
        delete sv;
        return fail(HK_ENOMEM, "hipMalloc of %zu workspace bytes failed", w.total);
    }
    for (int i = 0; i < sv->nev; ++i)
        for (int q = 0; q < 3; ++q)
            if (hipEventCreate(&sv->ev[i][q]) != hipSuccess) {
                solve_free(sv);
                return fail(HK_EDEVICE, "hipEventCreate failed");
            }
    // zero the workspace once (H, W, pivots read back even when unused)
    const hipError_t ze = sv->own_ws ? hipMemset(sv->ws, 0, w.total) : launch_fill_zero(sv->ws, w.total, stream);
    if (ze != hipSuccess) {
        solve_free(sv);
        return fail(HK_EDEVICE, "zeroing the workspace failed");
    }
    st = solve_bind(sv, op, p, rect, pl, w, (unsigned char*)sv->ws, stream, true);
    if (st) {
        solve_free(sv);
        return st;
    }
    {
        static const char* kname[] = {"blur (generic)", "csr (generic)", "blur (single barrier)"};
        char tile[64];
        if (pl.kernel == OP_CSR)
            std::snprintf(tile, sizeof tile, "about %lld rows", (long long)((op->m + pl.G - 1) / pl.G));
        else
            std::snprintf(tile, sizeof tile, "%dx%d pixels", pl.spm.TY, pl.spm.TX);
        log_info("solve: %s kernel, %d workgroups, tiles of %s, %d elements per thread, LDS %d B, "
                 "workspace %zu B, k = %d, s = %d, %d right-hand side(s), least squares on %d workgroup(s)",
                 kname[pl.kernel], pl.G, tile, pl.ept, pl.lds_total, w.total, p->k, p->s,
                 std::max(1, p->nrhs), std::max(1, sv->la.nwg));
    }
    live_add(sv);
    *out = sv;
    return HK_OK;
}

// Enqueue one run on `s`: control reset, basis kernel, sketches at the end,
// small least squares, x = L_k y.  Events (optional) bracket the basis
// kernel and the run.
static hk_status solve_enqueue(hk_solve* sv, const void* b_dev, void* x_dev, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1, hipEvent_t e2)
{
    KArgs a = sv->ka;
    a.b = b_dev;
    const int nr = sv->nrhs;
    // right-hand side b's region: the same layout, b * region bytes further on
    auto at = [&](auto* q, int b) { return (decltype(q))((char*)q + (size_t)b * sv->region); };
    for (int b = 0; b < nr; ++b) HIP_TRY(launch_ctl_init(at(a.ctl, b), s));
    if (e0) HIP_TRY(hipEventRecord(e0, s));
    HIP_TRY(launch_iterate(sv->tb, sv->op->dtype, sv->kernel, sv->sk, sv->ept, a, s));
    if (e1) HIP_TRY(hipEventRecord(e1, s));
    if (a.nosk)
        for (int b = 0; b < nr; ++b)
            HIP_TRY(launch_hess_rhs(at(a.F, b), at(a.c, b), sv->prm.s, sv->prm.k, sv->prm.lambda, at(a.ctl, b), s));
    if (sv->zend) {
        // Gaussian sketches of the whole basis: Z = (S2 D_{k+1}) H_{k+1,k},
        // F = S1 L_k, c = S2 b (the Gaussian entries in the data's precision)
        const int tg = sv->op->dtype == HK_F64 ? 0 : 1;
        const bool fz = sv->prm.lambda > 0.0;
        HIP_TRY(launch_block_sketch(sv->tb, tg, sv->bz, s));
        BskArgs bc = sv->bc;
        bc.q = b_dev;
        HIP_TRY(launch_block_sketch(sv->op->dtype == HK_F64 ? 0 : 1, tg, bc, s));
        if (fz) HIP_TRY(launch_block_sketch(sv->tb, tg, sv->bf, s));
        const long long cs = (long long)sv->prm.s * (sv->prm.k + 1);   // one right-hand side's columns of T
        for (int b = 0; b < nr; ++b)
            HIP_TRY(launch_sketch_finish(sv->T + b * cs, fz ? sv->T1 + b * cs : nullptr, at(a.H, b),
                                         sv->kernel == OP_BLUR_ONEBAR ? at(a.scale, b) : nullptr, sv->prm.s,
                                         sv->prm.k, at(a.Z, b), at(a.F, b), s));
    }
    HIP_TRY(launch_small_ls(sv->la, s));
    CombineArgs c = sv->ca;
    c.x = x_dev;
    HIP_TRY(launch_combine(sv->tb, sv->op->dtype, c, nr, s));
    if (e2) HIP_TRY(hipEventRecord(e2, s));
    return HK_OK;
}

extern "C" {

hk_status hk_solve_create(hk_op* op, const hk_params* p, hk_solve** out)
{
    HK_LIVE(op);
    if (!op) return fail(HK_EINVAL, "null operator");
    return solve_create(op, p, nullptr, 0, hk_solve::NEV, op->ctx->stream, out);
}

hk_status hk_solve_create_with_workspace(hk_op* op, const hk_params* p, void* ws_dev, size_t ws_bytes,
                                         hk_solve** out)
{
    HK_LIVE(op);
    if (!op) return fail(HK_EINVAL, "null operator");
    if (ws_dev && ((uintptr_t)ws_dev & 255)) return fail(HK_EINVAL, "workspace pointer is not 256-byte aligned");
    if (ws_dev && ws_bytes == 0) return fail(HK_ENOMEM, "workspace of 0 bytes");
    return solve_create(op, p, ws_dev, ws_bytes, hk_solve::NEV, op->ctx->stream, out);
}

hk_status hk_solve_run(hk_solve* sv, const void* b_dev, void* x_dev)
{
    HK_LIVE(sv);
    if (!sv || !b_dev || !x_dev) return fail(HK_EINVAL, "null argument");
    hk_status st = current_device(sv->op->ctx);
    if (st) return st;
    const int slot = (int)(sv->runs % sv->nev);
    sv->ev0 = sv->ev[slot][0];
    sv->ev1 = sv->ev[slot][1];
    sv->ev2 = sv->ev[slot][2];
    st = solve_enqueue(sv, b_dev, x_dev, sv->stream, sv->ev0, sv->ev1, sv->ev2);
    if (st) return st;
    sv->b_last = b_dev;
    sv->runs++;
    sv->ran = true;
    sv->waited = false;
    return HK_OK;
}

hk_status hk_solve_run_noalloc(hk_op* op, const hk_params* p_in, const void* b_dev, void* x_dev, int32_t* info_dev)
{
    HK_LIVE(op);
    if (!op || !p_in || !b_dev || !x_dev) return fail(HK_EINVAL, "null argument");
    hk_context* ctx = op->ctx;
    int rect = 0;
    hk_params pe{};
    Plan pl;
    size_t need = 0;
    hk_status st = solve_plan(op, p_in, &pe, &rect, &pl, &need);
    if (st) return st;
    if (need > NOALLOC_MAX_BYTES)
        return fail(HK_ENOMEM, "the solve needs %zu workspace bytes; the static workspace holds %zu", need,
                    NOALLOC_MAX_BYTES);
    const int dev = ctx->device;
    unsigned char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (dev < 0 || dev >= MAX_DEVICES || !g_scratch_done[dev])
            return fail(HK_EDEVICE, "no static workspace was set up for device %d", dev);
        if (!g_scratch_ptr[dev])
            return fail(HK_EDEVICE, "hipGetSymbolAddress of the static workspace failed: %s",
                        hipGetErrorString(g_scratch_err[dev]));
        base = (unsigned char*)g_scratch_ptr[dev];
    }
    const WsLayout w = ws_layout(op, &pe, rect, pl.G, pl.nslot);
    hk_solve sv;                       // launch arguments only: no events, no workspace of its own
    st = solve_bind(&sv, op, &pe, rect, pl, w, base, ctx->stream, false);
    if (st) return st;
    // the previous call's contents: clear everything before the bases (each
    // basis column is written before it is read)
    HIP_TRY(launch_fill_zero(base, w.L, ctx->stream));
    st = solve_enqueue(&sv, b_dev, x_dev, ctx->stream, nullptr, nullptr, nullptr);
    if (st) return st;
    if (info_dev) HIP_TRY(launch_solve_info(sv.ka.ctl, info_dev, ctx->stream));
    return HK_OK;
}

hk_status hk_solve_wait(hk_solve* sv)
{
    HK_LIVE(sv);
    if (!sv) return fail(HK_EINVAL, "null solve");
    if (!sv->ran) return fail(HK_EINVAL, "the solve has not been run");
    if (sv->waited) return sv->last;
    hk_status st = current_device(sv->op->ctx);
    if (st) return st;
    HIP_TRY(hipEventSynchronize(sv->ev2));
    // every right-hand side's control block (the first also holds the
    // barrier's abort flag); the run's status is the worst of them
    bool abort = false;
    int worst = HK_OK, bad = -1;
    for (int b = 0; b < sv->nrhs; ++b) {
        Ctl ctl;
        HIP_TRY(hipMemcpy(&ctl, (const char*)sv->ka.ctl + (size_t)b * sv->region, sizeof(Ctl), hipMemcpyDeviceToHost));
        if (b == 0) abort = ctl.abort != 0;
        sv->rst[b] = ctl.status;
        sv->rkd[b] = ctl.k_done;
        sv->rnt[b] = ctl.nt;
        sv->rng[b] = ctl.ng;
        if (ctl.status < 0 && bad < 0) bad = b;
        if (ctl.status == HK_BREAKDOWN && worst == HK_OK) worst = HK_BREAKDOWN;
    }
    sv->waited = true;
    sv->aborted = abort;
    sv->k_done = sv->rkd[sv->sel];
    sv->nt = sv->rnt[sv->sel];
    sv->ng = sv->rng[sv->sel];
    if (abort) {
        sv->last = fail(HK_EDEVICE, "grid barrier timed out: the basis kernel was aborted");
    } else if (bad >= 0) {
        const int st = sv->rst[bad];
        sv->last = fail(st, st == HK_ENUMERIC ? "right-hand side %d: non-finite values or a rank-deficient sketched problem"
                                              : "right-hand side %d: device error %d", bad, st);
    } else {
        sv->last = worst;
    }
    return sv->last;
}

hk_status hk_solve_select_rhs(hk_solve* sv, int32_t rhs)
{
    HK_LIVE(sv);
    if (!sv) return fail(HK_EINVAL, "null solve");
    if (rhs < 0 || rhs >= sv->nrhs) return fail(HK_EINVAL, "right-hand side %d outside [0, %d)", rhs, sv->nrhs);
    sv->sel = rhs;
    sv->k_done = sv->rkd[rhs];
    sv->nt = sv->rnt[rhs];
    sv->ng = sv->rng[rhs];
    return HK_OK;
}

// The last run has finished and the selected right-hand side's results are
// valid: an error of another right-hand side does not hide them.
static hk_status ensure_done(hk_solve* sv)
{
    if (!sv) return fail(HK_EINVAL, "null solve");
    hk_status st = hk_solve_wait(sv);
    if (st >= 0) return HK_OK;
    if (sv->nrhs > 1 && !sv->aborted && sv->rst[sv->sel] >= 0) return HK_OK;
    if (sv->nrhs > 1 && !sv->aborted)
        return fail(sv->rst[sv->sel], "right-hand side %d: status %d", sv->sel, sv->rst[sv->sel]);
    return st;
}

hk_status hk_solve_info(hk_solve* sv, int32_t* k_done)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    if (k_done) *k_done = sv->k_done;
    return sv->nrhs > 1 ? sv->rst[sv->sel] : sv->last;
}

hk_status hk_solve_get_hessenberg(hk_solve* sv, double* H, double* W)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    const int k = sv->prm.k;
    const size_t ro = (size_t)sv->sel * sv->region;     // the selected right-hand side's region
    if (H) HIP_TRY(hipMemcpy(H, (const char*)sv->ka.H + ro, sizeof(double) * (size_t)(k + 1) * k, hipMemcpyDeviceToHost));
    if (W) {
        if (!sv->rect) return fail(HK_EINVAL, "W exists for the generalized Hessenberg method only");
        HIP_TRY(hipMemcpy(W, sv->ka.W, sizeof(double) * (size_t)k * k, hipMemcpyDeviceToHost));
    }
    return HK_OK;
}

hk_status hk_solve_get_pivots(hk_solve* sv, int64_t* t, int64_t* g)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    const int k = sv->prm.k;
    std::vector<int> buf(k + 1);
    const size_t ro = (size_t)sv->sel * sv->region;
    if (t) {
        HIP_TRY(hipMemcpy(buf.data(), (const char*)sv->ka.tp + ro, sizeof(int) * (k + 1), hipMemcpyDeviceToHost));
        for (int i = 0; i <= k; ++i) t[i] = i < sv->nt ? buf[i] : -1;
    }
    if (g) {
        if (!sv->rect) return fail(HK_EINVAL, "g exists for the generalized Hessenberg method only");
        HIP_TRY(hipMemcpy(buf.data(), sv->ka.gp, sizeof(int) * (k + 1), hipMemcpyDeviceToHost));
        for (int i = 0; i < k; ++i) g[i] = i < sv->ng ? buf[i] : -1;
    }
    return HK_OK;
}

hk_status hk_solve_get_residuals(hk_solve* sv, double* res)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    if (!res) return fail(HK_EINVAL, "null output");
    HIP_TRY(hipMemcpy(res, (const char*)sv->la.res + (size_t)sv->sel * sv->region, sizeof(double) * sv->prm.k,
                      hipMemcpyDeviceToHost));
    for (int i = sv->k_done; i < sv->prm.k; ++i) res[i] = 0.0;
    return HK_OK;
}

hk_status hk_solve_get_prefix_solution(hk_solve* sv, int32_t kp, void* x_dev)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    if (!x_dev) return fail(HK_EINVAL, "null output");
    if (kp < 1 || kp > sv->k_done) return fail(HK_EINVAL, "prefix length %d outside [1, %d]", kp, sv->k_done);
    HIP_TRY(hipSetDevice(sv->op->ctx->device));
    const hipStream_t s = sv->op->ctx->stream;
    const size_t ro = (size_t)sv->sel * sv->region;
    auto at = [&](auto* q) { return (decltype(q))((char*)q + ro); };
    double* yp = at(sv->yp);
    HIP_TRY(launch_prefix_y(at(sv->la.R), at(sv->la.d), sv->prm.k, kp, 1, yp, s));
    CombineArgs c = sv->ca;
    c.L = (const char*)c.L + (size_t)sv->sel * (sv->prm.k + 1) * c.ldl * dsize(sv->prm.basis_dtype);
    c.ctl = at(c.ctl);
    c.y = yp;
    c.scale = c.scale ? at(c.scale) : nullptr;
    c.x = x_dev;
    c.kcap = kp;
    HIP_TRY(launch_combine(sv->tb, sv->op->dtype, c, 1, s));
    HIP_TRY(hipStreamSynchronize(s));
    return HK_OK;
}

hk_status hk_solve_get_true_residuals(hk_solve* sv, double* res)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    if (!res) return fail(HK_EINVAL, "null output");
    if (!sv->b_last) return fail(HK_EINVAL, "no run of this solve with a right-hand side to compare against");
    hk_op* op = sv->op;
    HIP_TRY(hipSetDevice(op->ctx->device));
    const hipStream_t s = op->ctx->stream;
    const int kd = sv->k_done, k = sv->prm.k;
    const size_t es = dsize(op->dtype);
    void* xt = nullptr;
    void* ax = nullptr;
    double* dres = nullptr;
    auto cleanup = [&]() { hipFree(xt); hipFree(ax); hipFree(dres); };
    if (hipMalloc(&xt, es * (size_t)op->n) != hipSuccess || hipMalloc(&ax, es * (size_t)op->m) != hipSuccess ||
        hipMalloc(&dres, sizeof(double) * (size_t)std::max(1, k)) != hipSuccess) {
        cleanup();
        return fail(HK_ENOMEM, "hipMalloc of the residual buffers failed");
    }
    const size_t ro = (size_t)sv->sel * sv->region;
    auto at = [&](auto* q) { return (decltype(q))((char*)q + ro); };
    const void* b = (const char*)sv->b_last + (size_t)sv->sel * (size_t)op->m * es;
    CombineArgs c = sv->ca;
    c.L = (const char*)c.L + (size_t)sv->sel * (sv->prm.k + 1) * c.ldl * dsize(sv->prm.basis_dtype);
    c.ctl = at(c.ctl);
    c.y = at(sv->yp);
    c.scale = c.scale ? at(c.scale) : nullptr;
    c.x = xt;
    hk_status out = HK_OK;
    for (int kp = 1; kp <= kd && out == HK_OK; ++kp) {
        // x_kp = L_kp y_kp, then ||b - A x_kp|| with the operator's own product
        hipError_t e = launch_prefix_y(at(sv->la.R), at(sv->la.d), k, kp, 1, at(sv->yp), s);
        if (e == hipSuccess) {
            c.kcap = kp;
            e = launch_combine(sv->tb, op->dtype, c, 1, s);
        }
        if (e != hipSuccess) { out = fail(HK_EDEVICE, "%s", hipGetErrorString(e)); break; }
        out = op_apply_on(op, 0, xt, ax, s);
        if (out == HK_OK) {
            e = launch_resid_norm(op->dtype == HK_F64 ? 0 : 1, b, ax, (long long)op->m, dres + (kp - 1), s);
            if (e != hipSuccess) out = fail(HK_EDEVICE, "%s", hipGetErrorString(e));
        }
    }
    if (out == HK_OK && kd > 0 &&
        (hipMemcpyAsync(res, dres, sizeof(double) * kd, hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
        out = fail(HK_EDEVICE, "copying the residuals failed");
    cleanup();
    if (out != HK_OK) return out;
    for (int i = kd; i < k; ++i) res[i] = 0.0;
    return HK_OK;
}

hk_status hk_solve_get_sketches(hk_solve* sv, double* Z, double* F, double* c)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    // the small problem's inputs (for the unsketched method H, [I; 0], beta e_1)
    const size_t sk = (size_t)sv->prm.s * sv->prm.k;
    const size_t ro = (size_t)sv->sel * sv->region;
    if (Z) HIP_TRY(hipMemcpy(Z, (const char*)sv->la.Z + ro, sizeof(double) * sk, hipMemcpyDeviceToHost));
    if (F) HIP_TRY(hipMemcpy(F, (const char*)sv->la.F + ro, sizeof(double) * sk, hipMemcpyDeviceToHost));
    if (c) HIP_TRY(hipMemcpy(c, sv->la.c + (size_t)sv->sel * sv->la.c_stride, sizeof(double) * sv->prm.s,
                             hipMemcpyDeviceToHost));
    return HK_OK;
}

hk_status hk_solve_get_basis(hk_solve* sv, int32_t which, void* dst_dev)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    if (!dst_dev) return fail(HK_EINVAL, "null output");
    const size_t es = dsize(sv->tb);
    const int kp1 = sv->prm.k + 1;
    // the selected right-hand side's basis and scales
    const void* Lb = (const char*)sv->ka.L + es * (size_t)sv->sel * kp1 * (size_t)sv->ka.ldl;
    const double* scb = (const double*)((const char*)sv->ka.scale + (size_t)sv->sel * sv->region);
    if (which == 2 || (which == 0 && sv->kernel != OP_BLUR_ONEBAR)) {
        // the columns as stored (unnormalised v_j for the single-barrier kernel)
        HIP_TRY(hipMemcpy2D(dst_dev, es * sv->op->n, Lb, es * sv->ka.ldl, es * sv->op->n, kp1,
                            hipMemcpyDeviceToDevice));
    } else if (which == 0) {
        // stored unnormalised with per-column scales: copy l_j = s_j v_j
        HIP_TRY(launch_scale_basis(sv->tb, Lb, sv->ka.ldl, scb, sv->op->n, kp1, dst_dev, sv->stream));
        HIP_TRY(hipStreamSynchronize(sv->stream));
    } else if (which == 1) {
        if (!sv->rect) return fail(HK_EINVAL, "D exists for the generalized Hessenberg method only");
        HIP_TRY(hipMemcpy2D(dst_dev, es * sv->op->m, sv->ka.D, es * sv->ka.ldd, es * sv->op->m, kp1,
                            hipMemcpyDeviceToDevice));
    } else {
        return fail(HK_EINVAL, "which must be 0 (L), 1 (D) or 2 (stored L)");
    }
    return HK_OK;
}

hk_status hk_solve_grid(const hk_solve* sv, int32_t* workgroups)
{
    HK_LIVE(sv);
    if (!sv || !workgroups) return fail(HK_EINVAL, "null argument");
    *workgroups = sv->G;
    return HK_OK;
}

hk_status hk_solve_timing(hk_solve* sv, double* iterate_ms, double* total_ms)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    float a = 0.f, b = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, sv->ev0, sv->ev1));
    HIP_TRY(hipEventElapsedTime(&b, sv->ev0, sv->ev2));
    if (iterate_ms) *iterate_ms = a;
    if (total_ms) *total_ms = b;
    return HK_OK;
}

hk_status hk_solve_timing_history(hk_solve* sv, int32_t max_runs, double* iterate_ms,
                                  double* total_ms, int32_t* n)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    if (max_runs < 0 || !n) return fail(HK_EINVAL, "bad arguments");
    const long long kept = std::min<long long>(sv->runs, sv->nev);
    const int cnt = (int)std::min<long long>(kept, max_runs);
    for (int i = 0; i < cnt; ++i) {
        const long long run = sv->runs - cnt + i;
        const int slot = (int)(run % sv->nev);
        float a = 0.f, b = 0.f;
        HIP_TRY(hipEventElapsedTime(&a, sv->ev[slot][0], sv->ev[slot][1]));
        HIP_TRY(hipEventElapsedTime(&b, sv->ev[slot][0], sv->ev[slot][2]));
        if (iterate_ms) iterate_ms[i] = a;
        if (total_ms) total_ms[i] = b;
    }
    *n = cnt;
    return HK_OK;
}

hk_status hk_solve_get_trace(hk_solve* sv, int32_t max, uint64_t* ticks, int32_t* n, double* tick_ns)
{
    HK_LIVE(sv);
    hk_status st = ensure_done(sv);
    if (st) return st;
    if (!n || max < 0 || (max > 0 && !ticks)) return fail(HK_EINVAL, "bad arguments");
    if (!sv->ka.trace) return fail(HK_EINVAL, "the solve was created without HK_FLAG_TRACE");
    Ctl ctl;
    HIP_TRY(hipMemcpy(&ctl, sv->ka.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    // barrier pairs, then sub-step marks (blur kernel), per-workgroup arrivals,
    // then the LS kernel's marks
    const int rec = sv->ka.trace_cap + ARR_SLOTS + LS_TRACE;
    const int cnt = std::min(rec, (int)max);
    if (cnt > 0) HIP_TRY(hipMemcpy(ticks, sv->ka.trace, sizeof(uint64_t) * cnt, hipMemcpyDeviceToHost));
    *n = cnt;
    if (tick_ns) *tick_ns = 1e6 / (double)sv->op->ctx->wall_rate_khz;
    return HK_OK;
}

hk_status hk_solve_destroy(hk_solve* sv)
{
    if (!live_take(sv)) return fail(HK_EINVAL, sv ? "unknown or destroyed solve" : "null solve");
    solve_free(sv);
    return HK_OK;
}

}  // extern "C"

// ====================================================================== serving
// Continuous batching on one device.  Requests are queued on arrival and
// admitted in arrival order whenever a slot, the workspace they need within
// the device-memory budget and the compute units of their basis kernel are
// free.  Each admitted solve runs on its slot's stream with an ordinary
// (non-cooperative) launch, so the basis kernels of up to `slots` requests
// run side by side; the sum of their grids never exceeds the compute units
// given to the server, which keeps every grid co-resident.  Retired
// workspaces are pooled for reuse instead of freed, because freeing device
// memory would wait for the solves still running.
struct hk_server {
    hk_context* ctx = nullptr;
    size_t budget = 0;              // device bytes of workspace the server may hold
    size_t held = 0;                // allocated (in use or pooled)
    int wg_total = 0, wg_used = 0;  // compute units for basis kernels
    struct Slot {
        hipStream_t st = nullptr;
        hk_solve* sv = nullptr;
        int64_t ticket = -1;
        void* buf = nullptr;
        size_t cap = 0;
    };
    std::vector<Slot> slots;
    struct Req {
        int64_t ticket;
        hk_op* op;
        hk_params p;
        const void* b;
        void* x;
        hipEvent_t ready;           // the context stream at submission (b and x produced)
    };
    std::deque<Req> queue;
    struct Res {
        hk_status status = HK_OK;
        int k_done = 0, grid = 0;
        double t_submit = 0.0, t_start = 0.0, t_finish = 0.0;
        bool done = false;
    };
    std::vector<Res> res;
    std::vector<std::pair<void*, size_t>> pool;   // idle workspaces
    std::vector<hipEvent_t> evpool;               // idle submission events
    int64_t completed = 0;
    int running = 0;
};

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void finish_request(hk_server* s, int64_t t, hk_status st, int k_done)
{
    auto& r = s->res[(size_t)t];
    r.status = st;
    r.k_done = k_done;
    r.t_finish = now_s();
    if (r.t_start == 0.0) r.t_start = r.t_finish;
    r.done = true;
    s->completed++;
}

// Retire finished solves, then admit queued requests while they fit.
hk_status server_pump(hk_server* s)
{
    for (auto& sl : s->slots) {
        if (!sl.sv) continue;
        const hipError_t q = hipEventQuery(sl.sv->ev2);
        if (q == hipErrorNotReady) continue;
        const hk_status st = (q == hipSuccess) ? hk_solve_wait(sl.sv) : fail(HK_EDEVICE, "%s", hipGetErrorString(q));
        finish_request(s, sl.ticket, st, sl.sv->k_done);
        s->wg_used -= sl.sv->G;
        s->running--;
        hk_solve_destroy(sl.sv);           // the workspace is the server's
        s->pool.emplace_back(sl.buf, sl.cap);
        sl.sv = nullptr;
        sl.ticket = -1;
        sl.buf = nullptr;
        sl.cap = 0;
    }
    while (!s->queue.empty()) {
        hk_server::Slot* slot = nullptr;
        for (auto& sl : s->slots)
            if (!sl.sv) { slot = &sl; break; }
        if (!slot) break;
        const hk_server::Req rq = s->queue.front();
        // grid: a fair share of the compute units, or as many as the
        // problem needs when its tiles do not fit in a share
        const int share = std::max(1, s->wg_total / (int)s->slots.size());
        hk_params p = rq.p;
        p.max_workgroups = rq.p.max_workgroups > 0 ? std::min(rq.p.max_workgroups, s->wg_total) : share;
        hk_params pe{};
        int rect = 0;
        Plan pl;
        size_t need = 0;
        hk_status st = solve_plan(rq.op, &p, &pe, &rect, &pl, &need);
        // a problem with more tiles than a share: the fewest extra shares
        for (int cap = 2 * share; st == HK_EUNSUPPORTED && rq.p.max_workgroups == 0 && p.max_workgroups < s->wg_total;
             cap += share) {
            p.max_workgroups = std::min(cap, s->wg_total);
            st = solve_plan(rq.op, &p, &pe, &rect, &pl, &need);
        }
        if (st < 0) {
            s->queue.pop_front();
            s->evpool.push_back(rq.ready);
            finish_request(s, rq.ticket, st, 0);
            continue;
        }
        if (pl.G > s->wg_total - s->wg_used) break;          // wait for compute units
        // workspace: the smallest pooled buffer that fits, else a new one
        int pick = -1;
        for (int i = 0; i < (int)s->pool.size(); ++i)
            if (s->pool[i].second >= need && (pick < 0 || s->pool[i].second < s->pool[pick].second)) pick = i;
        void* buf = nullptr;
        size_t cap = 0;
        if (pick >= 0) {
            buf = s->pool[pick].first;
            cap = s->pool[pick].second;
            s->pool.erase(s->pool.begin() + pick);
        } else {
            if (s->held + need > s->budget && s->running == 0) {
                // nothing runs: the idle buffers can be released cheaply
                for (auto& b : s->pool) {
                    hipFree(b.first);
                    s->held -= b.second;
                }
                s->pool.clear();
            }
            if (s->held + need > s->budget) {
                if (s->running > 0) break;                      // wait for memory
                s->queue.pop_front();
                s->evpool.push_back(rq.ready);
                finish_request(s, rq.ticket, fail(HK_ENOMEM, "workspace of %zu bytes exceeds the budget", need), 0);
                continue;
            }
            if (hipMalloc(&buf, need) != hipSuccess) {
                if (s->running > 0) break;
                s->queue.pop_front();
                s->evpool.push_back(rq.ready);
                finish_request(s, rq.ticket, fail(HK_ENOMEM, "hipMalloc of %zu bytes failed", need), 0);
                continue;
            }
            cap = need;
            s->held += need;
        }
        // the slot stream starts after everything the caller's stream held
        // at submission (whatever produced b and x)
        const hipError_t we = hipStreamWaitEvent(slot->st, rq.ready, 0);
        s->evpool.push_back(rq.ready);
        hk_solve* sv = nullptr;
        st = we == hipSuccess ? solve_create(rq.op, &p, buf, cap, 1, slot->st, &sv)
                              : fail(HK_EDEVICE, "hipStreamWaitEvent failed: %s", hipGetErrorString(we));
        if (st == HK_OK) {
            st = hk_solve_run(sv, rq.b, rq.x);
            if (st != HK_OK) {
                hk_solve_destroy(sv);
                sv = nullptr;
            }
        }
        s->queue.pop_front();
        if (st != HK_OK) {
            s->pool.emplace_back(buf, cap);
            finish_request(s, rq.ticket, st, 0);
            continue;
        }
        log_info("server: request %lld admitted on slot %d, %d workgroups, %zu B of workspace",
                 (long long)rq.ticket, (int)(slot - s->slots.data()), sv->G, cap);
        slot->sv = sv;
        slot->ticket = rq.ticket;
        slot->buf = buf;
        slot->cap = cap;
        s->wg_used += sv->G;
        s->running++;
        auto& r = s->res[(size_t)rq.ticket];
        r.t_start = now_s();
        r.grid = sv->G;
    }
    return HK_OK;
}

}  // namespace

extern "C" {

static void server_free(hk_server* s);

hk_status hk_server_create(hk_context* ctx, int32_t slots, size_t budget_bytes, int32_t workgroups,
                           hk_server** out)
{
    HK_LIVE(ctx);
    if (!ctx || !out) return fail(HK_EINVAL, "null argument");
    *out = nullptr;
    if (slots < 1 || slots > 16) return fail(HK_EINVAL, "slots = %d must be in [1, 16]", slots);
    if (workgroups < 0) return fail(HK_EINVAL, "workgroups must be >= 0");
    hk_status st = current_device(ctx);
    if (st) return st;
    auto* s = new (std::nothrow) hk_server;
    if (!s) return fail(HK_ENOMEM, "host allocation failed");
    s->ctx = ctx;
    if (budget_bytes == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete s; return fail(HK_EDEVICE, "hipMemGetInfo failed"); }
        budget_bytes = fr / 10 * 8;
    }
    s->budget = budget_bytes;
    // a few compute units stay free for the short kernels of finishing solves
    s->wg_total = workgroups > 0 ? std::min(workgroups, ctx->ncu) : std::max(1, ctx->ncu - 8);
    s->slots.resize((size_t)slots);
    for (auto& sl : s->slots)
        if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess) {
            server_free(s);
            return fail(HK_EDEVICE, "hipStreamCreateWithFlags failed");
        }
    live_add(s);
    *out = s;
    return HK_OK;
}

hk_status hk_server_destroy(hk_server* s)
{
    if (!live_take(s)) return fail(HK_EINVAL, s ? "unknown or destroyed server" : "null server");
    server_free(s);
    return HK_OK;
}

// Waits for the running solves and frees everything the server holds (no
// registry check: also for a server whose creation failed).
static void server_free(hk_server* s)
{
    hipSetDevice(s->ctx->device);
    for (auto& sl : s->slots) {
        if (sl.st) hipStreamSynchronize(sl.st);
        if (sl.sv) hk_solve_destroy(sl.sv);
        if (sl.buf) hipFree(sl.buf);
        if (sl.st) hipStreamDestroy(sl.st);
    }
    for (auto& b : s->pool) hipFree(b.first);
    for (auto& rq : s->queue) hipEventDestroy(rq.ready);
    for (hipEvent_t e : s->evpool) hipEventDestroy(e);
    delete s;
}

hk_status hk_server_submit(hk_server* s, hk_op* op, const hk_params* params, const void* b_dev, void* x_dev,
                           int64_t* ticket)
{
    HK_LIVE(s);
    HK_LIVE(op);
    if (!s || !op || !params || !b_dev || !x_dev || !ticket) return fail(HK_EINVAL, "null argument");
    if (op->ctx->device != s->ctx->device) return fail(HK_EINVAL, "the operator lives on another device");
    hk_status st = current_device(s->ctx);
    if (st) return st;
    // an event on the context stream marks what the solve must follow
    hipEvent_t ev = nullptr;
    if (!s->evpool.empty()) {
        ev = s->evpool.back();
        s->evpool.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        return fail(HK_EDEVICE, "hipEventCreateWithFlags failed");
    }
    if (hipEventRecord(ev, s->ctx->stream) != hipSuccess) {
        s->evpool.push_back(ev);
        return fail(HK_EDEVICE, "hipEventRecord on the context stream failed");
    }
    const int64_t t = (int64_t)s->res.size();
    s->res.emplace_back();
    s->res.back().t_submit = now_s();
    s->queue.push_back({t, op, *params, b_dev, x_dev, ev});
    *ticket = t;
    return server_pump(s);
}

hk_status hk_server_poll(hk_server* s, int64_t* completed)
{
    HK_LIVE(s);
    if (!s) return fail(HK_EINVAL, "null server");
    hk_status st = current_device(s->ctx);
    if (st) return st;
    st = server_pump(s);
    if (completed) *completed = s->completed;
    return st;
}

hk_status hk_server_wait(hk_server* s, int64_t ticket)
{
    HK_LIVE(s);
    if (!s || ticket < 0 || ticket >= (int64_t)s->res.size()) return fail(HK_EINVAL, "bad ticket");
    hk_status st = current_device(s->ctx);
    if (st) return st;
    while (!s->res[(size_t)ticket].done) {
        st = server_pump(s);
        if (st) return st;
        if (s->res[(size_t)ticket].done) break;
        if (s->running == 0 && !s->queue.empty() && s->queue.front().ticket <= ticket)
            return fail(HK_EDEVICE, "request %lld cannot be admitted", (long long)ticket);
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    return s->res[(size_t)ticket].status;
}

hk_status hk_server_result(hk_server* s, int64_t ticket, hk_status* status, int32_t* k_done, int32_t* workgroups,
                           double* t_submit, double* t_start, double* t_finish)
{
    HK_LIVE(s);
    if (!s || ticket < 0 || ticket >= (int64_t)s->res.size()) return fail(HK_EINVAL, "bad ticket");
    const auto& r = s->res[(size_t)ticket];
    if (!r.done) return fail(HK_EINVAL, "request %lld has not finished", (long long)ticket);
    if (status) *status = r.status;
    if (k_done) *k_done = r.k_done;
    if (workgroups) *workgroups = r.grid;
    if (t_submit) *t_submit = r.t_submit;
    if (t_start) *t_start = r.t_start;
    if (t_finish) *t_finish = r.t_finish;
    return HK_OK;
}

}  // extern "C"
