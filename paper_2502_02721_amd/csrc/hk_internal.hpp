// Internal definitions shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hk {

constexpr int NT = 512;             // threads per workgroup (8 wave64s)
constexpr int NWAVE = NT / 64;
constexpr int KMAX = 255;           // largest k: k+1 pivot slots fit 4 per lane of one wave
constexpr int KSLOT = 4;            // (KMAX+1)/64
constexpr int MAX_EPT = 4;          // elements per thread of a tile (tile <= 2048 elements)
constexpr int MAXG = 256;           // workgroups of the persistent kernel (one per CU)
constexpr int SAMPLE_MAX = 64;      // largest pivot sample
constexpr int RMAX = 8;             // right-hand sides a solve advances together
constexpr int SAMPLE_SLOTS = 4 * ((SAMPLE_MAX + 3) / 4 + 2);   // candidate slots per search
// a whole basis (at most NT * MAX_EPT * MAXG elements per column, KMAX + 1
// FP64 columns) is addressed by 32-bit byte offsets of one buffer resource
static_assert((long long)NT * MAX_EPT * MAXG * 8 * (KMAX + 1) < (1LL << 31), "basis exceeds 2 GiB");

enum OpKind { OP_BLUR = 0, OP_CSR = 1, OP_BLUR_ONEBAR = 2 };

// Fixed-point scale 2^e such that terms whose magnitudes sum to at most
// `bound` accumulate below 2^61 in int64 (exact, order-independent sums).
__host__ __device__ inline double fx_scale(double bound)
{
    int ex = 0;
    if (!(bound > 0.0)) return 1.0;
    frexp(bound, &ex);
    return ldexp(1.0, 61 - ex);
}
enum SketchKind { SK_GAUSS = 0, SK_SPARSE = 1 };

// How the elements of one space (length m or n) are split into tiles, one
// tile per workgroup.  kind 0: 2-D image tiles TY x TX (row-major image of
// nx columns); kind 1: contiguous ranges [t*len/ntile, (t+1)*len/ntile).
struct Space {
    int kind;                    // 0: 2-D image tiles; 1: equal row ranges; 2: row ranges at st[]
    int len;
    int ntile;
    int ny, nx, TY, TX, ntx;
    const int* st;               // kind 2: tile t holds [st[t], st[t + 1]), st[ntile] = len (device)
};

// Device control block at the start of the workspace: status words, then
// the grid-barrier counters, each on its own 256-byte line.
struct alignas(256) CtlLine {
    unsigned v;
    unsigned pad[63];
};

struct Ctl {
    unsigned bar;        // flat arrivals (start-up barrier)
    unsigned abort;      // set when a barrier wait times out
    int k_done;          // basis columns built
    int status;          // 0 ok, 1 breakdown, <0 error (hk_status)
    int ls_status;       // small least-squares status
    int nt;              // pivots found in the data-space basis (t)
    int ng;              // pivots found in the unknowns' basis (g, sLSLU)
    int nbar;            // grid barriers passed (trace length / 2)
    double beta;         // first pivot entry b(t_1) (the unsketched right-hand side beta e_1)
    int pad[54];
    CtlLine gcnt;        // XCD-leader arrivals
    CtlLine xcnt[16];    // arrivals per XCD
    CtlLine xflag[16];   // release epoch per XCD
    CtlLine pop[16];     // workgroups per XCD
    CtlLine lsb;         // arrivals at the least-squares kernel's barrier (row-split form)
};

// Everything the persistent Hessenberg kernel needs (passed by value).
struct KArgs {
    int m, n, k, s, zeta;
    double lam;
    uint32_t seed_lo, seed_hi;
    int rect;                   // 1: generalized Hessenberg (sLSLU)
    int nosk;                   // 1: no sketches (the unsketched CMRH / LSLU projected problem)
    int coop;                   // 1: cooperative launch (whole-device grid)
    int stepsk;                 // 1: sketch partials every step (0: none, or a block sketch at the end)
    int psamp, pnc;             // sampled pivoting: sample size (0: full argmax), Philox calls
    double* sval;               // published sample values, 4 x SAMPLE_SLOTS
    int* sidx;                  // their rows (-1: a pivot row), 4 x SAMPLE_SLOTS
    int xcd_map;                // XCD-aware tile numbering
    int G;                      // workgroups = tiles
    const void* b;
    Space spm, spn;             // tiling of the data space (m) and unknowns (n)
    // blur: separable taps, or (ntap > 0) the tap list of a general PSF,
    // offsets (a + r) << 16 | (b + r) and weights
    int ny, nx, r, bc;
    const double* taps_y;
    const double* taps_x;
    const int* toff;
    const double* tw;
    int ntap;
    // CSR of A (m rows) and of A^T (n rows)
    const int64_t* rp;  const int* ci;  const void* cv;
    const int64_t* rpt; const int* cit; const void* cvt;
    int lpr, lprt;              // lanes per row for the two CSR products
    // fixed-point scales 2^sc for the sparse-sign partial sums
    double scz, scf;            // w = A l (|w| <= ||A||_inf), l (|l| <= 1)
    // workspace
    void* L; int64_t ldl;       // basis L: n x (k+1), column stride ldl
    void* D; int64_t ldd;       // basis D: m x (k+1) (sLSLU)
    double* H; double* W;       // (k+1) x k, k x k
    int* tp; int* gp;           // pivots of D (or of L for sCMRH) and of L (sLSLU)
    void* PD; void* PL;         // pivot blocks (k+1)^2, column-major, storage type
    double* pvD; double* pvL;   // operator output at the pivot rows
    double* amv; int* ami;      // argmax partials [2G]
    long long* zpart;           // sketch partial sums [G*s] (int64 fixed point or FP64 bits)
    long long* fpart;
    long long* cpart;
    double* Z; double* F; double* c;
    Ctl* ctl;
    unsigned long long timeout_ticks;
    // optional per-barrier timestamps of workgroup 0 (wall clock ticks):
    // trace[2e] before arriving at barrier e, trace[2e+1] after it released
    unsigned long long* trace;
    int trace_cap;
    // pivot blocks in LDS: pmode 0 keeps a packed copy of every block for the
    // whole solve (one row appended per step), pmode 1 bulk-loads the needed
    // triangle into one LDS buffer before each substitution
    int pmode;
    // LDS layout (byte offsets into the dynamic shared buffer)
    int lds_h, lds_w, lds_pl_m, lds_pc_m, lds_bm_m, lds_pl_n, lds_pc_n, lds_bm_n;
    int lds_sk, lds_stage, lds_vert, lds_taps, lds_pD, lds_pL, lds_total;
    // single-barrier blur kernel: FP64 scales 1/eta of the stored (unnormalised)
    // basis vectors, window partial sums of A v at the pivots, layout
    double* scale;              // k+1
    double* wpart;              // (k+1) * nslot
    int nslot, spx;             // slots per pivot, slots per row of the window box
    int lds_scale, lds_hs, lds_wred;
    int lds_skt;                // sparse-sign tables (0: built on the fly)
    // right-hand sides advanced together (single-barrier blur kernel): each
    // has a workspace region rhs_stride bytes after the previous one (its
    // basis: (k + 1) columns after the previous one's in L; its b: m
    // elements further on) and an LDS block lds_rhs bytes further on
    int nrhs;
    long long rhs_stride;
    int lds_rhs;
    // CSR operators: the row pointers of the workgroup's m-tile and n-tile
    // rows, relative to the tile's first entry (int32), staged once per solve
    // (-1: not staged, read from global memory)
    int lds_rp_m, lds_rp_n;
};

// LDS bytes of a blur's PSF: 2 (2r + 1) separable taps, or ntap weights and
// offsets of a general PSF
__host__ __device__ inline int psf_lds_bytes(int r, int ntap)
{
    return ntap > 0 ? ((ntap * 8 + 15) / 16) * 16 + ntap * 4 : 2 * (2 * r + 1) * 8;
}

// Column-packed strict lower triangle of a (k+1) x (k+1) pivot block:
// column c holds rows c+1..k.
__host__ __device__ inline int packed_col(int c, int k) { return c * k - (c * (c - 1)) / 2; }
__host__ __device__ inline long long packed_size(int k) { return (long long)k * (k + 1) / 2; }

struct LsArgs {
    int s, k;
    int nb;                      // panel width of the blocked kernel (0: column-by-column kernel)
    double lam;
    const double* Z; const double* F; const double* c;
    double* Q; double* R; double* r; double* y; double* res; double* d;
    Ctl* ctl;
    unsigned long long* trace;   // LS_TRACE timestamps, or null
    // several right-hand sides: workgroup b solves the problem whose Z, F,
    // Q, R, r, y, res, d and ctl lie b * rhs_stride bytes further on, with
    // c b * c_stride doubles further on
    int nrhs;
    long long rhs_stride;
    long long c_stride;
    // row-split form: nwg workgroups per right-hand side, each holding a
    // slice of the rows; sums over rows meet in xpart (2 x nwg x ls_xcap(k)
    // doubles, in the right-hand side's region) behind a bounded barrier
    int nwg;
    double* xpart;
    unsigned long long timeout;
};

// The small problem of right-hand side b (the workgroup's).
__device__ __forceinline__ LsArgs ls_rebase(const LsArgs& a0, int b)
{
    LsArgs a = a0;
    if (b == 0) return a;
    const long long st = (long long)b * a0.rhs_stride;
    auto sh = [&](auto* q) { return q ? (decltype(q))((const char*)q + st) : q; };
    a.Z = sh(a0.Z); a.F = sh(a0.F); a.Q = sh(a0.Q); a.R = sh(a0.R); a.r = sh(a0.r);
    a.y = sh(a0.y); a.res = sh(a0.res); a.d = sh(a0.d); a.ctl = sh(a0.ctl); a.xpart = sh(a0.xpart);
    a.c = a0.c + (long long)b * a0.c_stride;
    a.trace = nullptr;
    return a;
}
constexpr int LS_TRACE = 256;    // timestamp slots of the least-squares kernel
// per-workgroup barrier arrival / release timestamps of the blur kernel at
// steps j = 8 q + 4 (q < ARR_SAMPLES): ARR_SAMPLES x 2 x MAXG slots after the
// basis kernel's own trace
constexpr int ARR_SAMPLES = 32;
constexpr int ARR_SLOTS = ARR_SAMPLES * 2 * MAXG;

struct CombineArgs {
    int n, k;
    const void* L; int64_t ldl;
    const double* y;
    const double* scale;         // per-column scale of the stored basis, or null
    void* x;
    const Ctl* ctl;
    // right-hand side blockIdx.y: its basis (k + 1) columns further on, x n
    // elements further on, y, scale and ctl rhs_stride bytes further on
    long long rhs_stride;
    int kcap;                    // > 0: use at most kcap columns (a prefix solution)
};

struct ApplyArgs {
    int transpose;
    Space sp;                    // output-space tiling
    int ny, nx, r, bc;
    const double* taps_y; const double* taps_x;
    const int* toff; const double* tw; int ntap;   // general PSF (ntap > 0)
    const int64_t* rp; const int* ci; const void* cv;
    int lpr;
    const void* x; void* y;
    int lds_w, lds_stage, lds_vert, lds_taps, lds_total;
};

// Host-side launchers (defined in hk_kernels.hip).  Types: 0 f64, 1 f32;
// tb = basis storage, to = operator / vector storage.
hipError_t launch_iterate(int tb, int to, int op, int sketch, int ept, const KArgs& a, hipStream_t st);
hipError_t launch_ctl_init(Ctl* ctl, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);   // p, bytes: multiples of 16
hipError_t launch_solve_info(const Ctl* ctl, int32_t* info, hipStream_t st);
hipError_t launch_small_ls(const LsArgs& a, hipStream_t st);
hipError_t launch_combine(int tb, int to, const CombineArgs& a, int nrhs, hipStream_t st);
// y' = R(1:kp, 1:kp)^{-1} d(1:kp) (R column-major with leading dimension k),
// by the same column-oriented substitution as the least-squares kernels
// (recip: multiply by the reciprocal of the diagonal, as the least-squares kernels do)
// out = ||b - y||_2 (m entries of type dtype: 0 FP64, 1 FP32), FP64 sums in a fixed order
hipError_t launch_resid_norm(int dtype, const void* b, const void* y, long long m, double* out, hipStream_t st);
hipError_t launch_prefix_y(const double* R, const double* d, int k, int kp, int recip, double* yp,
                           hipStream_t st);
// block sketch C = S B with S generated (hk_bsk.hip)
struct BskArgs {
    const void* q;              // B: len x ncol, column-major, leading dimension ldq
    long long ldq;
    int len, ncol;
    int s;                      // rows of S
    int rt, ct, kc, chunk;      // row tiles, column tiles (64), contraction chunks and their length
    uint32_t stream, k0, k1;    // Philox stream and key of S
    double* part;               // rt * ct * kc tiles of 64 x 64
    double* out;                // s x ncol, leading dimension ldo
    int ldo;
    double scale;               // 1 / sqrt(s)
};
hipError_t launch_block_sketch(int tq, int tg, const BskArgs& a, hipStream_t st);
hipError_t launch_sketch_finish(const double* T, const double* T1, const double* H, const double* sc, int s, int k,
                                double* Z, double* F, hipStream_t st);
hipError_t launch_hess_rhs(double* F, double* c, int s, int k, double lam, const Ctl* ctl, hipStream_t st);
hipError_t launch_apply(int dtype, int op, int ept, const ApplyArgs& a, hipStream_t st);
hipError_t launch_scale_basis(int tb, const void* src, int64_t ld, const double* scale, int64_t len,
                              int ncols, void* dst, hipStream_t st);
hipError_t iterate_occupancy(int tb, int to, int op, int sketch, int ept, int samp, int lds_bytes,
                             int* blocks_per_cu);
size_t small_ls_lds_bytes(int s, int k, double lam);
constexpr int LS_MWG_MAX = 32;   // workgroups of the row-split least-squares kernel
// doubles per workgroup of one cross-workgroup sum: a projection block
// ((k + 1) x 16) or a 16 x 16 Gram matrix
__host__ __device__ inline int ls_xcap(int k) { return (k + 1) * 16 > 256 ? (k + 1) * 16 : 256; }
int small_ls_wgs(int s, double lam);
int small_ls_panel(int s, int k, double lam, int nwg, size_t lds_max);
hipError_t launch_small_ls_blocked(int nb, const LsArgs& a, hipStream_t st);

}  // namespace hk
