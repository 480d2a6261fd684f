// gfx950 kernels for the sketched inner-product-free Krylov methods.
//
// One persistent cooperative kernel runs the whole basis iteration of a solve
// (Sec. 3.1: Hessenberg process with partial pivoting, eq. (Hessenberg_s);
// generalized Hessenberg process, eq. (Hessenberg_r), Algorithm 1).  Each
// workgroup owns one tile of the data space (and, for sLSLU, one tile of the
// unknowns) for the whole solve, so the new basis vector it produces stays in
// registers across the grid-wide argmax and is written to HBM exactly once.
// Per step (square case) the phases are
//   A: u = A l_j on the tile (FP64), S2-sketch partials of u, u at own pivots
//   B: coefficients h = P^{-1} u(pivots) (forward substitution on the pivot
//      block), v = u - L_j h streamed over the tile's basis rows, exact zeros
//      at pivot rows, per-tile argmax |v|
//   C: global argmax -> new pivot, l_{j+1} = v / v(pivot), S1-sketch partials
// separated by grid barriers (bounded spin, abort flag: every wave exits).
// No inner product is formed anywhere in the iteration.
#pragma once
#include "hk_internal.hpp"

#include <climits>

namespace hk {

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds, multipliers 0xD2511F53
// and 0xCD9E8D57, key schedule advanced by 0x9E3779B9 / 0xBB67AE85.
// ------------------------------------------------------------------------
struct Words { uint32_t w[4]; };

__device__ __forceinline__ Words philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                          uint32_t key0, uint32_t key1)
{
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint32_t a_hi = __umulhi(0xD2511F53u, x0), a_lo = 0xD2511F53u * x0;
        const uint32_t b_hi = __umulhi(0xCD9E8D57u, x2), b_lo = 0xCD9E8D57u * x2;
        const uint32_t y0 = b_hi ^ x1 ^ key0;
        const uint32_t y2 = a_hi ^ x3 ^ key1;
        x0 = y0; x1 = b_lo; x2 = y2; x3 = a_lo;
        key0 += 0x9E3779B9u;
        key1 += 0xBB67AE85u;
    }
    Words r;
    r.w[0] = x0; r.w[1] = x1; r.w[2] = x2; r.w[3] = x3;
    return r;
}

// Four standard normals of rows 4*grp .. 4*grp+3, column `col` of the Gaussian
// embedding: Box-Muller on the uniforms (2*(w>>9)+1) 2^-24 of one Philox
// block (counter (col, grp, stream, 0)).  FP32 storage generates in FP32.
template <typename TS>
__device__ __forceinline__ void gauss4(uint32_t col, uint32_t grp, uint32_t stream, uint32_t k0,
                                       uint32_t k1, double g[4]);

template <>
__device__ __forceinline__ void gauss4<double>(uint32_t col, uint32_t grp, uint32_t stream,
                                               uint32_t k0, uint32_t k1, double g[4])
{
    Words w = philox10(col, grp, stream, 0u, k0, k1);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const double ua = (double)(2u * (w.w[2 * p] >> 9) + 1u) * 0x1p-24;
        const double ub = (double)(2u * (w.w[2 * p + 1] >> 9) + 1u) * 0x1p-24;
        const double rad = sqrt(-2.0 * log(ua));
        double sn, cs;
        sincospi(2.0 * ub, &sn, &cs);
        g[2 * p] = rad * cs;
        g[2 * p + 1] = rad * sn;
    }
}

template <>
__device__ __forceinline__ void gauss4<float>(uint32_t col, uint32_t grp, uint32_t stream,
                                              uint32_t k0, uint32_t k1, double g[4])
{
    Words w = philox10(col, grp, stream, 0u, k0, k1);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float ua = (float)(2u * (w.w[2 * p] >> 9) + 1u) * 0x1p-24f;
        const float ub = (float)(2u * (w.w[2 * p + 1] >> 9) + 1u) * 0x1p-24f;
        const float rad = sqrtf(-2.0f * logf(ua));
        float sn, cs;
        sincospif(2.0f * ub, &sn, &cs);
        g[2 * p] = (double)(rad * cs);
        g[2 * p + 1] = (double)(rad * sn);
    }
}

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------
__device__ __forceinline__ double readlane_d(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// DPP move of a 64-bit value (two 32-bit moves); lanes the control does not
// write get 0.
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ long long dpp64(long long v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffLL), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, ROW_MASK, 0xF, false);
    return ((long long)hi << 32) | (unsigned int)lo;
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double v)
{
    return __longlong_as_double(dpp64<CTRL, ROW_MASK>(__double_as_longlong(v)));
}

// Sum over the wave left in lane 63 (other lanes hold partial sums).
__device__ __forceinline__ double wave_sum_to63(double v)
{
    v += dpp_d<0xB1>(v);          // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);          // quad_perm [2,3,0,1]
    v += dpp_d<0x124>(v);         // row_ror:4
    v += dpp_d<0x128>(v);         // row_ror:8
    v += dpp_d<0x142, 0xA>(v);    // row_bcast:15 into rows 1, 3
    v += dpp_d<0x143, 0xC>(v);    // row_bcast:31 into rows 2, 3
    return v;
}

// Sum over the wave, returned to every lane.  DPP steps: quad xor 1 and 2,
// rotations by 4 and 8 inside each row of 16, then row 0 -> 1, 2 -> 3 and
// lane 31 -> rows 2, 3; lane 63 ends with the total.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_d<0xB1>(v);          // quad_perm [1,0,3,2]
    v += dpp_d<0x4E>(v);          // quad_perm [2,3,0,1]
    v += dpp_d<0x124>(v);         // row_ror:4
    v += dpp_d<0x128>(v);         // row_ror:8
    v += dpp_d<0x142, 0xA>(v);    // row_bcast:15 into rows 1, 3
    v += dpp_d<0x143, 0xC>(v);    // row_bcast:31 into rows 2, 3
    return readlane_d(v, 63);
}

__device__ __forceinline__ long long wave_sum_ll(long long v)
{
    v += dpp64<0xB1>(v);
    v += dpp64<0x4E>(v);
    v += dpp64<0x124>(v);
    v += dpp64<0x128>(v);
    v += dpp64<0x142, 0xA>(v);
    v += dpp64<0x143, 0xC>(v);
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), 63);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), 63);
    return ((long long)hi << 32) | (unsigned int)lo;
}

// (|v|, index) ordering: larger magnitude wins, ties go to the smaller index.
__device__ __forceinline__ bool am_better(double a1, int i1, double a2, int i2)
{
    return a1 > a2 || (a1 == a2 && i1 < i2);
}

__device__ __forceinline__ void wave_argmax(double& best, int& idx, double& val)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(idx, o);
        const double ov = __shfl_xor(val, o);
        if (am_better(ob, oi, best, idx)) { best = ob; idx = oi; val = ov; }
    }
}

__device__ __forceinline__ int bc_map(int i, int N, int bc)
{
    if (i >= 0 && i < N) return i;
    if (bc == 0) return -1;
    if (i < 0) i = -i - 1;
    if (i >= N) i = 2 * N - i - 1;
    return (i >= 0 && i < N) ? i : -1;
}

// ------------------------------------------------------------------------
// tiles
// ------------------------------------------------------------------------
struct Tile {
    int start;   // 1-D: first global index
    int E;       // elements (2-D: TY*TX slots, some may lie outside the image)
    int y0, x0;  // 2-D origin
};

__device__ __forceinline__ int range_start(int t, int len, int ntile)
{
    return (int)(((long long)t * len) / ntile);
}

__device__ __forceinline__ Tile tile_info(const Space& sp, int t)
{
    Tile ti;
    if (sp.kind == 0) {
        ti.y0 = (t / sp.ntx) * sp.TY;
        ti.x0 = (t % sp.ntx) * sp.TX;
        ti.E = sp.TY * sp.TX;
        ti.start = 0;
    } else if (sp.kind == 2) {
        ti.start = sp.st[t];
        ti.E = sp.st[t + 1] - ti.start;
        ti.y0 = ti.x0 = 0;
    } else {
        ti.start = range_start(t, sp.len, sp.ntile);
        ti.E = range_start(t + 1, sp.len, sp.ntile) - ti.start;
        ti.y0 = ti.x0 = 0;
    }
    return ti;
}

__device__ __forceinline__ bool elem_global(const Space& sp, const Tile& ti, int e, int& gi)
{
    if (e >= ti.E) return false;
    if (sp.kind == 0) {
        const int y = ti.y0 + e / sp.TX, x = ti.x0 + e % sp.TX;
        gi = y * sp.nx + x;
        return y < sp.ny && x < sp.nx;
    }
    gi = ti.start + e;
    return true;
}

// tile and local element that own global index gi
__device__ __forceinline__ void owner_of(const Space& sp, int gi, int& t, int& e)
{
    if (sp.kind == 0) {
        const int y = gi / sp.nx, x = gi % sp.nx;
        t = (y / sp.TY) * sp.ntx + x / sp.TX;
        e = (y % sp.TY) * sp.TX + (x % sp.TX);
    } else if (sp.kind == 2) {
        // the last tile whose start is <= gi (starts increase strictly)
        int lo = 0, hi = sp.ntile - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sp.st[mid] <= gi) lo = mid;
            else hi = mid - 1;
        }
        t = lo;
        e = gi - sp.st[lo];
    } else {
        int c = (int)(((long long)gi * sp.ntile) / sp.len);
        while (c + 1 < sp.ntile && range_start(c + 1, sp.len, sp.ntile) <= gi) ++c;
        while (c > 0 && range_start(c, sp.len, sp.ntile) > gi) --c;
        t = c;
        e = gi - range_start(c, sp.len, sp.ntile);
    }
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of tiles so stencil halos are shared inside one L2.
__device__ __forceinline__ int tile_of_block(int G, int xcd_map)
{
    const int b = blockIdx.x;
    if (!xcd_map) return b;
    return (b % 8) * (G / 8) + b / 8;
}

// ------------------------------------------------------------------------
// Grid barrier, hierarchical over the XCDs (each has its own L2).
//  - every wave drains its stores (s_waitcnt 0): they are in its XCD's L2;
//  - one thread per workgroup counts the arrival on its XCD's counter;
//  - the last arriver of an XCD writes that L2 back (agent release), counts
//    the XCD on the global counter, spins (bounded) until all XCDs arrived,
//    acquires, and publishes the epoch on its XCD's release flag;
//  - the other workgroups of the XCD spin on that flag and acquire (L1/L2
//    invalidate), so reads after the barrier see every workgroup's writes.
// One atomic per workgroup goes to its XCD line and one per XCD to the
// global line.  Every wait is bounded: on timeout the abort flag is raised
// and every waiter returns false.
// ------------------------------------------------------------------------
struct BarState {
    unsigned xcd, pop, nxcd, gbase, epoch;
};

__device__ __forceinline__ unsigned hw_xcc_id()
{
    // hardware register XCC_ID (id 20), bits [3:0]: the XCD this wave runs on
    return __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((16 - 1) << 11)) & 0xfu;
}

__device__ __forceinline__ bool spin_until(unsigned* p, unsigned target, Ctl* ctl,
                                           unsigned long long timeout)
{
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() - t0 > timeout) {
            __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Start-up: count the workgroups of each XCD (one flat barrier).
__device__ __forceinline__ bool hbar_init(Ctl* ctl, BarState& bs, unsigned G, unsigned long long timeout)
{
    __shared__ int s_ok;
    __shared__ unsigned s_xcd, s_pop, s_nx;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned x = hw_xcc_id();
        __hip_atomic_fetch_add(&ctl->pop[x].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&ctl->gcnt.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool ok = spin_until(&ctl->gcnt.v, G, ctl, timeout);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        unsigned nx = 0;
        for (int i = 0; i < 16; ++i)
            nx += __hip_atomic_load(&ctl->pop[i].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1u : 0u;
        s_xcd = x;
        s_pop = __hip_atomic_load(&ctl->pop[x].v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_nx = nx;
        s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    bs.xcd = s_xcd;
    bs.pop = s_pop;
    bs.nxcd = s_nx;
    bs.gbase = G;
    bs.epoch = 0;
    return s_ok != 0;
}

__device__ __forceinline__ bool hbar_sync(Ctl* ctl, BarState& bs, unsigned long long timeout,
                          unsigned long long* trace = nullptr, int trace_cap = 0)
{
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const unsigned ep = ++bs.epoch;
    if (threadIdx.x == 0) {
        const bool tr = trace && blockIdx.x == 0 && (int)(2 * ep) <= trace_cap;
        if (tr) trace[2 * (ep - 1)] = wall_clock64();
        bool ok;
        const unsigned old = __hip_atomic_fetch_add(&ctl->xcnt[bs.xcd].v, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        if (old == ep * bs.pop - 1) {           // last workgroup of this XCD
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(&ctl->gcnt.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = spin_until(&ctl->gcnt.v, bs.gbase + ep * bs.nxcd, ctl, timeout);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(&ctl->xflag[bs.xcd].v, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = spin_until(&ctl->xflag[bs.xcd].v, ep, ctl, timeout);
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        if (tr) trace[2 * (ep - 1) + 1] = wall_clock64();
        if (blockIdx.x == 0) ctl->nbar = (int)ep;
        s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    return s_ok != 0;
}

// ------------------------------------------------------------------------
// operator products on one tile -> wt[e] (FP64, LDS)
// ------------------------------------------------------------------------
// Separable blur: stage the tile plus an r-pixel halo (boundary condition
// applied while staging), vertical pass into FP64, horizontal pass.
constexpr int BLUR_SB = 8;                       // halo loads in flight per thread

// First block of the halo loads of a tile (staged region element q of the
// block is q0 + u * NT + thread, q0 = 0); `in` flags the loads that hit the
// image.  Issued early, they overlap other latency.
template <typename TS>
__device__ __forceinline__ void blur_stage_issue(const TS* __restrict__ x, int ny, int nx, int r, int bc,
                                                 const Tile& ti, int TY, int TX, TS (&v)[BLUR_SB], unsigned& in)
{
    const int SW = TX + 2 * r, SH = TY + 2 * r;
    in = 0u;
#pragma unroll
    for (int u = 0; u < BLUR_SB; ++u) {
        const int q = u * NT + (int)threadIdx.x;
        const int yy = q / SW, xx = q - yy * SW;
        const int y = bc_map(ti.y0 - r + yy, ny, bc);
        const int xg = bc_map(ti.x0 - r + xx, nx, bc);
        const bool ok = (q < SH * SW) && y >= 0 && xg >= 0;
        if (ok) in |= 1u << u;
        v[u] = x[ok ? y * nx + xg : 0];
    }
}

// The PSF as the kernels read it from LDS: separable taps tyl (x) txl
// (ntap == 0), or a list of ntap entries of a general PSF, each an offset
// (a + r, b + r) packed as (a + r) << 16 | (b + r) and its weight
// p(a, b) (the correlation (A u)(y, x) = sum p(a, b) u(y + a, x + b)).
struct PsfL {
    const double* tyl;
    const double* txl;
    const int* toff;
    const double* tw;
    int ntap;
};

// Copy the PSF into LDS at `taps` (no barrier: the caller synchronises).
__device__ __forceinline__ PsfL psf_stage(unsigned char* taps, int r, const double* taps_y, const double* taps_x,
                                          const int* toff, const double* tw, int ntap)
{
    PsfL ps;
    ps.ntap = ntap;
    double* td = (double*)taps;
    if (ntap > 0) {
        int* to = (int*)(taps + ((ntap * 8 + 15) / 16) * 16);
        for (int q = threadIdx.x; q < ntap; q += NT) {
            td[q] = tw[q];
            to[q] = toff[q];
        }
        ps.tw = td;
        ps.toff = to;
        ps.tyl = ps.txl = nullptr;
    } else {
        const int w = 2 * r + 1;
        for (int q = threadIdx.x; q < w; q += NT) {
            td[q] = taps_y[q];
            td[w + q] = taps_x[q];
        }
        ps.tyl = td;
        ps.txl = td + w;
        ps.toff = nullptr;
        ps.tw = nullptr;
    }
    return ps;
}

// Separable blur of one tile: wt = A x on the tile's pixels, with the halo
// staged in LDS; v / in are the first block from blur_stage_issue.  A
// general PSF (ps.ntap > 0) takes one pass over its tap list instead of the
// two 1-D passes.
template <typename TS>
__device__ __forceinline__ void blur_tile_staged(const TS* __restrict__ x, int ny, int nx, int r, int bc,
                                                 const Tile& ti, int TY, int TX, const PsfL& ps,
                                                 TS* stage, double* vert, double* wt,
                                                 const TS (&v0)[BLUR_SB], unsigned in0,
                                                 unsigned long long* tmk = nullptr)
{
    const double* tyl = ps.tyl;
    const double* txl = ps.txl;
    const int SW = TX + 2 * r, SH = TY + 2 * r;
    constexpr int SB = BLUR_SB;
#pragma unroll
    for (int u = 0; u < SB; ++u) {
        const int q = u * NT + (int)threadIdx.x;
        if (q < SH * SW) stage[q] = ((in0 >> u) & 1u) ? v0[u] : TS(0);
    }
    for (int q0 = SB * NT; q0 < SH * SW; q0 += SB * NT) {
        TS v[SB];
        bool in[SB];
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int q = q0 + u * NT + (int)threadIdx.x;
            const int yy = q / SW, xx = q - yy * SW;
            const int y = bc_map(ti.y0 - r + yy, ny, bc);
            const int xg = bc_map(ti.x0 - r + xx, nx, bc);
            in[u] = (q < SH * SW) && y >= 0 && xg >= 0;
            v[u] = x[in[u] ? y * nx + xg : 0];
        }
#pragma unroll
        for (int u = 0; u < SB; ++u) {
            const int q = q0 + u * NT + (int)threadIdx.x;
            if (q < SH * SW) stage[q] = in[u] ? v[u] : TS(0);
        }
    }
    __syncthreads();
    if (tmk && threadIdx.x == 0) tmk[0] = wall_clock64();
    if (ps.ntap > 0) {
        // general PSF: each thread forms 4 consecutive rows of one column,
        // one weight and offset (LDS broadcast) and 4 staged values per tap
        const int ngy = (TY + 3) / 4;
        for (int it = threadIdx.x; it < ngy * TX; it += NT) {
            const int g = it / TX, xx = it - g * TX;
            const int y0 = 4 * g;
            const int y1 = min(y0 + 1, TY - 1), y2 = min(y0 + 2, TY - 1), y3 = min(y0 + 3, TY - 1);
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll 4
            for (int t = 0; t < ps.ntap; ++t) {
                const int o = ps.toff[t];
                const double w = ps.tw[t];
                const TS* src = stage + (o >> 16) * SW + xx + (o & 0xffff);
                a0 = fma(w, (double)src[y0 * SW], a0);
                a1 = fma(w, (double)src[y1 * SW], a1);
                a2 = fma(w, (double)src[y2 * SW], a2);
                a3 = fma(w, (double)src[y3 * SW], a3);
            }
            double* wo = wt + y0 * TX + xx;
            wo[0] = a0;
            if (y0 + 1 < TY) wo[TX] = a1;
            if (y0 + 2 < TY) wo[2 * TX] = a2;
            if (y0 + 3 < TY) wo[3 * TX] = a3;
        }
        __syncthreads();
        if (tmk && threadIdx.x == 0) tmk[1] = wall_clock64();
        return;
    }
    const int taps = 2 * r + 1;
    // vertical pass: each thread computes 4 consecutive rows of one column
    // from a sliding window of 4 staged values (one LDS read, 4 independent
    // FMAs per tap)
    // (TY need not be a multiple of 4: the last group clamps its reads to
    // the staged rows and stores only the rows that exist)
    const int ngy = (TY + 3) / 4;
    for (int it = threadIdx.x; it < ngy * SW; it += NT) {
        const int g = it / SW, xx = it - g * SW;
        const int y0 = 4 * g;
        const TS* col = stage + xx;
        double s0 = (double)col[y0 * SW], s1 = (double)col[min(y0 + 1, SH - 1) * SW],
               s2 = (double)col[min(y0 + 2, SH - 1) * SW];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        // unrolled so that several taps' LDS reads are in flight together;
        // with TY a multiple of 4 no read needs the clamp
        if ((TY & 3) == 0) {
            const TS* src = col + (y0 + 3) * SW;
#pragma unroll 8
            for (int b = 0; b < taps; ++b) {
                const double s3 = (double)src[b * SW];
                const double w = tyl[b];
                a0 = fma(w, s0, a0); a1 = fma(w, s1, a1); a2 = fma(w, s2, a2); a3 = fma(w, s3, a3);
                s0 = s1; s1 = s2; s2 = s3;
            }
        } else {
#pragma unroll 8
            for (int b = 0; b < taps; ++b) {
                const double s3 = (double)col[min(y0 + b + 3, SH - 1) * SW];
                const double w = tyl[b];
                a0 = fma(w, s0, a0); a1 = fma(w, s1, a1); a2 = fma(w, s2, a2); a3 = fma(w, s3, a3);
                s0 = s1; s1 = s2; s2 = s3;
            }
        }
        double* vo = vert + y0 * SW + xx;
        vo[0] = a0;
        if (y0 + 1 < TY) vo[SW] = a1;
        if (y0 + 2 < TY) vo[2 * SW] = a2;
        if (y0 + 3 < TY) vo[3 * SW] = a3;
    }
    __syncthreads();
    if (tmk && threadIdx.x == 0) tmk[1] = wall_clock64();
    // horizontal pass: 2 consecutive outputs of one row per thread (an odd
    // TX clamps the last pair's extra read and drops its second output)
    const int ngx = (TX + 1) / 2;
    for (int it = threadIdx.x; it < TY * ngx; it += NT) {
        const int yy = it / ngx, x0 = 2 * (it - yy * ngx);
        const double* row = vert + yy * SW;
        double s0 = row[x0];
        double a0 = 0.0, a1 = 0.0;
        if ((TX & 1) == 0) {                       // no read needs the clamp
#pragma unroll 8
            for (int b = 0; b < taps; ++b) {
                const double s1 = row[x0 + b + 1];
                const double w = txl[b];
                a0 = fma(w, s0, a0); a1 = fma(w, s1, a1);
                s0 = s1;
            }
        } else {
#pragma unroll 8
            for (int b = 0; b < taps; ++b) {
                const double s1 = row[min(x0 + b + 1, SW - 1)];
                const double w = txl[b];
                a0 = fma(w, s0, a0); a1 = fma(w, s1, a1);
                s0 = s1;
            }
        }
        wt[yy * TX + x0] = a0;
        if (x0 + 1 < TX) wt[yy * TX + x0 + 1] = a1;
    }
    __syncthreads();
}

template <typename TS>
__device__ __forceinline__ void blur_tile(const TS* __restrict__ x, int ny, int nx, int r, int bc, const Tile& ti,
                                          int TY, int TX, const PsfL& ps, TS* stage,
                                          double* vert, double* wt, unsigned long long* tmk = nullptr)
{
    TS v[BLUR_SB];
    unsigned in;
    blur_stage_issue<TS>(x, ny, nx, r, bc, ti, TY, TX, v, in);
    blur_tile_staged<TS>(x, ny, nx, r, bc, ti, TY, TX, ps, stage, vert, wt, v, in, tmk);
}

// Long rows (a wave per row): each wave takes two rows at a time and issues
// the loads of up to 8 entries per lane of both rows before any gather, so a
// pair of rows costs three dependent memory round trips (row pointers,
// entries, gathers) rather than about five per row.  Per lane the entries
// are accumulated in increasing position, then summed over the wave.
template <typename TV, typename TX>
__device__ void csr_tile_wave2(const int64_t* __restrict__ rp, const int* __restrict__ ci,
                               const TV* __restrict__ cv, const TX* __restrict__ x, const Tile& ti,
                               double* wt, const int* rpl, long long rbase)
{
    constexpr int B = 8;                           // entries per lane per row and batch
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // row pointers from the LDS copy when staged (one LDS read instead of a
    // global round trip per row pair)
    auto rowp = [&](int e) -> long long { return rpl ? rbase + rpl[e] : rp[ti.start + e]; };
    for (int e0 = 2 * wave; e0 < ti.E; e0 += 2 * NWAVE) {
        const bool two = e0 + 1 < ti.E;
        const long long pa = rowp(e0), pm = rowp(e0 + 1);
        const long long pb = two ? rowp(e0 + 2) : pm;
        const long long na = pm - pa, nb = pb - pm;      // entries of row e0 and e0+1
        double acca = 0.0, accb = 0.0;
        for (long long b0 = 0; b0 < na || b0 < nb; b0 += 64 * B) {
            int ca[B], cb[B];
            TV va[B], vb[B];
            // loads are unconditional at clamped positions (a row with no
            // entries is skipped as a whole); values past the row are masked
            if (na > 0) {
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const long long q = b0 + lane + 64 * u;
                    const long long qa = pa + (q < na ? q : na - 1);
                    ca[u] = ci[qa];
                    const TV t = cv[qa];
                    va[u] = q < na ? t : TV(0);
                }
            } else {
#pragma unroll
                for (int u = 0; u < B; ++u) { ca[u] = 0; va[u] = TV(0); }
            }
            if (nb > 0) {
#pragma unroll
                for (int u = 0; u < B; ++u) {
                    const long long q = b0 + lane + 64 * u;
                    const long long qb = pm + (q < nb ? q : nb - 1);
                    cb[u] = ci[qb];
                    const TV t = cv[qb];
                    vb[u] = q < nb ? t : TV(0);
                }
            } else {
#pragma unroll
                for (int u = 0; u < B; ++u) { cb[u] = 0; vb[u] = TV(0); }
            }
            TX xa[B], xb[B];
#pragma unroll
            for (int u = 0; u < B; ++u) { xa[u] = x[ca[u]]; xb[u] = x[cb[u]]; }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                acca = fma((double)va[u], (double)xa[u], acca);
                accb = fma((double)vb[u], (double)xb[u], accb);
            }
        }
        acca = wave_sum(acca);
        accb = wave_sum(accb);
        if (lane == 0) {
            wt[e0] = acca;
            if (two) wt[e0 + 1] = accb;
        }
    }
    __syncthreads();
}

// CSR rows [start, start+E): groups of `lpr` lanes per row, FP64 accumulation.
// rpl (optional): the tile's row pointers in LDS, relative to rbase.
template <typename TV, typename TX>
__device__ __forceinline__ void csr_tile(const int64_t* __restrict__ rp, const int* __restrict__ ci,
                         const TV* __restrict__ cv, const TX* __restrict__ x, const Tile& ti,
                         int lpr, double* wt, const int* rpl = nullptr, long long rbase = 0)
{
    if (lpr == 64) {
        csr_tile_wave2<TV, TX>(rp, ci, cv, x, ti, wt, rpl, rbase);
        return;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rpw = 64 / lpr;
    const int sub = lane / lpr, sl = lane - sub * lpr;
    for (int base = wave * rpw; base < ti.E; base += NWAVE * rpw) {
        const int e = base + sub;
        double acc = 0.0;
        if (e < ti.E) {
            const long long p0 = rpl ? rbase + rpl[e] : rp[ti.start + e];
            const long long p1 = rpl ? rbase + rpl[e + 1] : rp[ti.start + e + 1];
            long long p = p0 + sl;
            // batches of 4 entries per lane: indices and values, then the
            // gathers, then the FMAs (in entry order)
            for (; p + 3 * lpr < p1; p += 4 * lpr) {
                int c4[4];
                TV v4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) { c4[u] = ci[p + u * lpr]; v4[u] = cv[p + u * lpr]; }
                TX x4[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) x4[u] = x[c4[u]];
#pragma unroll
                for (int u = 0; u < 4; ++u) acc = fma((double)v4[u], (double)x4[u], acc);
            }
            for (; p < p1; p += lpr) acc = fma((double)cv[p], (double)x[ci[p]], acc);
        }
        for (int o = lpr >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (sl == 0 && e < ti.E) wt[e] = acc;
    }
    __syncthreads();
}

// ------------------------------------------------------------------------
// sketch partial sums of a tile vector vals[e] (FP64, LDS)
// ------------------------------------------------------------------------
// Sparse sign (zeta nonzeros +-1/sqrt(zeta) per column, one per row block
// [b s/zeta, (b+1) s/zeta), block b from word b%4 of Philox (col, b/4,
// stream, 1)).  Terms are accumulated as int64 fixed point: exact, so the
// sum does not depend on the order of the LDS atomics.  out[r] holds sum of
// sign * round(v * scale) over the tile.
__device__ void sketch_sparse_partial(const double* vals, const Space& sp, const Tile& ti, int s,
                                      int zeta, uint32_t stream, uint32_t k0, uint32_t k1,
                                      double scale, long long* acc, long long* out)
{
    for (int r = threadIdx.x; r < s; r += NT) acc[r] = 0;
    __syncthreads();
    for (int e = threadIdx.x; e < ti.E; e += NT) {
        int gi;
        if (!elem_global(sp, ti, e, gi)) continue;
        const long long q = __double2ll_rn(vals[e] * scale);
        if (q == 0) continue;
        for (int b4 = 0; b4 < zeta; b4 += 4) {
            const Words w = philox10((uint32_t)gi, (uint32_t)(b4 >> 2), stream, 1u, k0, k1);
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                const int b = b4 + qq;
                if (b >= zeta) break;
                // block boundaries floor(b s / zeta): b s < 2^31 for s < 2^15
                const int st = (int)((unsigned)(b * s) / (unsigned)zeta);
                const int en = (int)((unsigned)((b + 1) * s) / (unsigned)zeta);
                const uint32_t word = w.w[qq];
                const int row = st + (int)(((unsigned long long)(word >> 1) * (unsigned)(en - st)) >> 31);
                atomicAdd((unsigned long long*)&acc[row], (unsigned long long)((word & 1u) ? -q : q));
            }
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < s; r += NT) out[r] = acc[r];
}

// Gaussian: out[r] = sum_e g(r, col(e)) * vals[e] (unscaled normals).  Each
// thread owns one row group (4 rows) and a strided subset of the elements,
// summed in element order; the nsub subsets of a row group sit in adjacent
// lanes and are added by a fixed xor-shuffle tree: deterministic.
template <typename TS>
__device__ void sketch_gauss_partial(const double* vals, const Space& sp, const Tile& ti, int s,
                                     uint32_t stream, uint32_t k0, uint32_t k1, double* red,
                                     double* out)
{
    const int NG = (s + 3) >> 2;
    int nsub = 1;
    while (nsub * 2 <= 64 && nsub * 2 * NG <= NT) nsub *= 2;
    for (int base = 0; base < NG * nsub; base += NT) {
        const int t = base + threadIdx.x;
        const int rg = t / nsub, es = t - rg * nsub;
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        if (rg < NG) {
            for (int e = es; e < ti.E; e += nsub) {
                int gi;
                if (!elem_global(sp, ti, e, gi)) continue;
                const double v = vals[e];
                double g[4];
                gauss4<TS>((uint32_t)gi, (uint32_t)rg, stream, k0, k1, g);
                a0 = fma(g[0], v, a0); a1 = fma(g[1], v, a1); a2 = fma(g[2], v, a2); a3 = fma(g[3], v, a3);
            }
        }
        for (int o = nsub >> 1; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o); a1 += __shfl_xor(a1, o);
            a2 += __shfl_xor(a2, o); a3 += __shfl_xor(a3, o);
        }
        if (rg < NG && es == 0) {
            red[4 * rg] = a0; red[4 * rg + 1] = a1; red[4 * rg + 2] = a2; red[4 * rg + 3] = a3;
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < s; r += NT) out[r] = red[r];
    __syncthreads();
}

// Sparse-sign rows of one tile, built once per solve.  For every sketch row
// r, ents[offs[r] .. offs[r+1]) lists the tile elements e whose column of S
// has a nonzero in row r, as e | (negative << 15), in increasing e.  A step's
// partial S x over the tile is then a gather per row with no atomics, summed
// in a fixed order.
struct SkRows {
    unsigned* offs;          // s + 1
    unsigned short* ents;    // E * zeta
};

__device__ void sketch_rows_build(const Space& sp, const Tile& ti, int s, int zeta, uint32_t stream,
                                  uint32_t k0, uint32_t k1, SkRows t, unsigned* cur)
{
    // row counts in offs[r + 1]
    for (int r = threadIdx.x; r <= s; r += NT) t.offs[r] = 0u;
    __syncthreads();
    auto each = [&](auto&& fn) {
        for (int e = threadIdx.x; e < ti.E; e += NT) {
            int gi;
            if (!elem_global(sp, ti, e, gi)) continue;
            for (int b4 = 0; b4 < zeta; b4 += 4) {
                const Words w = philox10((uint32_t)gi, (uint32_t)(b4 >> 2), stream, 1u, k0, k1);
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const int b = b4 + qq;
                    if (b >= zeta) break;
                    const int st = (int)((unsigned)(b * s) / (unsigned)zeta);
                    const int en = (int)((unsigned)((b + 1) * s) / (unsigned)zeta);
                    const uint32_t word = w.w[qq];
                    const int row = st + (int)(((unsigned long long)(word >> 1) * (unsigned)(en - st)) >> 31);
                    fn(e, row, (int)(word & 1u));
                }
            }
        }
    };
    each([&](int, int row, int) { atomicAdd(&t.offs[row + 1], 1u); });
    __syncthreads();
    // inclusive scan of offs[1 .. s] by wave 0: lane-contiguous chunks
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int C = (s + 63) / 64;
        const int r0 = min(s, lane * C), r1 = min(s, r0 + C);
        unsigned loc = 0u;
        for (int r = r0; r < r1; ++r) loc += t.offs[r + 1];
        unsigned incl = loc;                    // inclusive scan over lanes
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned up = __shfl_up(incl, o);
            if (lane >= o) incl += up;
        }
        unsigned run = incl - loc;
        for (int r = r0; r < r1; ++r) {
            run += t.offs[r + 1];
            t.offs[r + 1] = run;
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < s; r += NT) cur[r] = t.offs[r];
    __syncthreads();
    each([&](int e, int row, int neg) {
        const unsigned pos = atomicAdd(&cur[row], 1u);
        t.ents[pos] = (unsigned short)(e | (neg << 15));
    });
    __syncthreads();
    // the slot order above depends on timing: sort each row by element
    for (int r = threadIdx.x; r < s; r += NT) {
        const unsigned b = t.offs[r], en = t.offs[r + 1];
        for (unsigned q = b + 1; q < en; ++q) {
            const unsigned short x = t.ents[q];
            unsigned p = q;
            while (p > b && (t.ents[p - 1] & 0x7fffu) > (x & 0x7fffu)) {
                t.ents[p] = t.ents[p - 1];
                --p;
            }
            t.ents[p] = x;
        }
    }
    __syncthreads();
}

// out[r] = sum over the row's entries of +-vals[e], in list order (FP64),
// rows t0, t0 + nt, ... (no barrier: callable by a subset of the waves).
__device__ __forceinline__ void sketch_rows_sum(const double* vals, SkRows t, int s, double* out, int t0, int nt)
{
    for (int r = t0; r < s; r += nt) {
        const unsigned b = t.offs[r], en = t.offs[r + 1];
        double acc = 0.0;
        unsigned q = b;
        for (; q + 4 <= en; q += 4) {
            unsigned short x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = t.ents[q + u];
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = vals[x[u] & 0x7fffu];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += (x[u] & 0x8000u) ? -v[u] : v[u];
        }
        for (; q < en; ++q) {
            const unsigned short x = t.ents[q];
            const double v = vals[x & 0x7fffu];
            acc += (x & 0x8000u) ? -v : v;
        }
        out[r] = acc;
    }
}

// All rows by the whole workgroup; ends with a workgroup barrier.
__device__ void sketch_rows_partial(const double* vals, SkRows t, int s, double* out)
{
    sketch_rows_sum(vals, t, s, out, (int)threadIdx.x, NT);
    __syncthreads();                            // vals may be overwritten next
}

template <typename TS, int SK>
__device__ __forceinline__ void sketch_partial(const KArgs& a, const double* vals, const Space& sp,
                                               const Tile& ti, uint32_t stream, double scale,
                                               unsigned char* sk, long long* part, int tile)
{
    if constexpr (SK == SK_SPARSE) {
        sketch_sparse_partial(vals, sp, ti, a.s, a.zeta, stream, a.seed_lo, a.seed_hi, scale,
                              (long long*)sk, part + (long long)tile * a.s);
    } else {
        sketch_gauss_partial<TS>(vals, sp, ti, a.s, stream, a.seed_lo, a.seed_hi, (double*)sk,
                                 (double*)(part + (long long)tile * a.s));
    }
}

// Reduce the G partials of this workgroup's slice of sketch rows into out[]
// (one wave per row, fixed order).
// Row r of the sketch: out[r] = inv * sum over the G workgroup partials, by
// one wave in a fixed order.
template <int SK>
__device__ __forceinline__ void reduce_row(const long long* part, int G, int s, int r, double inv, double* out)
{
    const int lane = threadIdx.x & 63;
    if constexpr (SK == SK_SPARSE) {
        long long v[MAXG / 64];
#pragma unroll
        for (int u = 0; u < MAXG / 64; ++u) {
            const int q = lane + 64 * u;
            v[u] = part[(long long)(q < G ? q : 0) * s + r];
        }
        long long acc = 0;
#pragma unroll
        for (int u = 0; u < MAXG / 64; ++u)
            if (lane + 64 * u < G) acc += v[u];
        acc = wave_sum_ll(acc);
        if (lane == 0) out[r] = (double)acc * inv;
    } else {
        const double* pd = (const double*)part;
        double v[MAXG / 64];
#pragma unroll
        for (int u = 0; u < MAXG / 64; ++u) {
            const int q = lane + 64 * u;
            v[u] = pd[(long long)(q < G ? q : 0) * s + r];
        }
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < MAXG / 64; ++u)
            if (lane + 64 * u < G) acc += v[u];
        acc = wave_sum(acc);
        if (lane == 0) out[r] = acc * inv;
    }
}

// Reduce the G partials of this workgroup's slice of sketch rows into out[]
// (one wave per row, fixed order).
template <int SK>
__device__ __forceinline__ void reduce_partials(const KArgs& a, const long long* part, double inv, int tile, double* out)
{
    const int wave = threadIdx.x >> 6;
    const int r0 = (int)(((long long)tile * a.s) / a.G), r1 = (int)(((long long)(tile + 1) * a.s) / a.G);
    for (int r = r0 + wave; r < r1; r += NWAVE) reduce_row<SK>(part, a.G, a.s, r, inv, out);
}

// ------------------------------------------------------------------------
// coefficients: h = P^{-1} pv with P the unit lower triangular pivot block
// (P(i, c) = basis_c(pivot_i)), held in LDS as a column-packed strict lower
// triangle of a (k+1) x (k+1) block.  Column-oriented forward substitution by
// wave 0: h_c is final when column c is reached; the next column is read from
// LDS while the current one is applied.
// ------------------------------------------------------------------------
// Storage of the pivot block: the basis type, except FP32 for 16-bit bases,
// where the products s_i v_i(p_j) would otherwise be rounded a second time
// to 8 or 11 significant bits.
template <typename TB> struct PivotT { using type = TB; };
template <> struct PivotT<__bf16> { using type = float; };
template <> struct PivotT<_Float16> { using type = float; };

template <typename TS, int NQ>
__device__ __forceinline__ void forward_subst_nq(const TS* __restrict__ Pl, int k, const double* __restrict__ pv,
                                                 int nh, double* h)
{
    // Column-oriented: after h_c is final (lane c), every later row takes
    // v_i -= P(i, c) h_c.  The LDS loads of the next D columns are issued
    // before the current D steps run, so the step's critical path is
    // readlane -> fma rather than the LDS latency.
    constexpr int D = (NQ <= 1) ? 16 : ((NQ == 2) ? 8 : 4);   // columns in flight
    const int lane = threadIdx.x & 63;
    const int plast = (int)packed_size(k) - 1;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        v[q] = (i < nh) ? pv[i] : 0.0;
    }
    // Slot d of the ring holds column c0 + d as loaded (address clamped, no
    // condition, so the loads never become branches) and is refilled with
    // column c0 + d + D once used.  Entries of rows i <= c or i >= nh are
    // masked to zero at use, so the update needs no branch either
    // (fma(-0, h, v) == v); columns c >= nh - 1 are all masked.
    auto load = [&](int c, TS (&dst)[NQ]) {
        const int base = packed_col(c, k) - (c + 1);     // base + i = position of P(i, c)
#pragma unroll
        for (int q = 0; q < NQ; ++q) dst[q] = Pl[min(max(base + lane + 64 * q, 0), plast)];
    };
    TS ring[D][NQ];
#pragma unroll
    for (int d = 0; d < D; ++d) load(d, ring[d]);
    for (int c0 = 0; c0 + 1 < nh; c0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int c = c0 + d;
            double src = v[0];
#pragma unroll
            for (int q = 1; q < NQ; ++q)
                if ((c >> 6) == q) src = v[q];
            const double hc = readlane_d(src, c & 63);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = lane + 64 * q;
                const double pc = (i > c && i < nh) ? (double)ring[d][q] : 0.0;
                v[q] = fma(-pc, hc, v[q]);
            }
            load(c + D, ring[d]);
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        if (i < nh) h[i] = v[q];
    }
}

template <typename TS, int NQ>
__device__ __forceinline__ void forward_subst_seg_nq(const TS* __restrict__ Pl, int k, const double* __restrict__ pv,
                                                     int nh, double* h)
{
    // The same column-oriented substitution as forward_subst_nq, arranged for
    // the one-barrier kernel's wave 0.  After h_c is final (lane c & 63 of lane group c >> 6),
    // every later row takes v_i -= P(i, c) h_c.  The columns run in segments
    // of 64, one per lane group, unrolled at compile time: h_c is read from a
    // fixed register, and the groups above the segment (rows all final) take
    // neither loads nor updates.  Only the segment's own group masks its
    // rows i <= c (fma(-0, h, v) == v for finite h, so the arithmetic of
    // every row is the same as with all rows updated).  Rows i >= nh hold
    // whatever the unused part of the block gives them (LDS is not cleared:
    // possibly Inf or NaN) and are never read back; the columns c >= nh - 1
    // past the end, run by the last group of D, take h_c = 0, so they leave
    // every row i < nh as it is.  The LDS loads of the next D columns are
    // issued while the current D run.
    constexpr int D = (NQ <= 1) ? 16 : ((NQ == 2) ? 8 : 4);   // columns in flight (divides 64)
    const int lane = threadIdx.x & 63;
    const int plast = (int)packed_size(k) - 1;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        v[q] = (i < nh) ? pv[i] : 0.0;
    }
    // slot d of the ring holds column c0 + d as loaded (address clamped, so
    // the loads never become branches), refilled with column c0 + d + D
    auto load = [&](int c, TS (&dst)[NQ], int q0) {
        const int base = packed_col(c, k) - (c + 1);     // base + i = position of P(i, c)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q >= q0) dst[q] = Pl[min(max(base + lane + 64 * q, 0), plast)];
    };
    TS ring[D][NQ];
#pragma unroll
    for (int d = 0; d < D; ++d) load(d, ring[d], 0);
#pragma unroll
    for (int qc = 0; qc < NQ; ++qc) {
        const int cend = min(64 * qc + 64, nh - 1);
        for (int c0 = 64 * qc; c0 < cend; c0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int c = c0 + d;
                const double hr = readlane_d(v[qc], c & 63);
                const double hc = (c < nh - 1) ? hr : 0.0;     // uniform select
#pragma unroll
                for (int q = qc; q < NQ; ++q) {
                    TS pc = ring[d][q];
                    if (q == qc) pc = (lane > (c & 63)) ? pc : (TS)0;
                    v[q] = fma(-(double)pc, hc, v[q]);
                }
                load(c + D, ring[d], qc);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = lane + 64 * q;
        if (i < nh) h[i] = v[q];
    }
}

// the generic kernel's form (fewer registers: it runs beside the CSR state)
template <typename TS>
__device__ __forceinline__ void forward_subst(const TS* __restrict__ Pl, int k, const double* __restrict__ pv,
                                              int nh, double* h)
{
    const int nq = (nh + 63) >> 6;
    if (nq <= 1) forward_subst_nq<TS, 1>(Pl, k, pv, nh, h);
    else if (nq == 2) forward_subst_nq<TS, 2>(Pl, k, pv, nh, h);
    else if (nq == 3) forward_subst_nq<TS, 3>(Pl, k, pv, nh, h);
    else forward_subst_nq<TS, 4>(Pl, k, pv, nh, h);
}

template <typename TS>
__device__ __forceinline__ void forward_subst_seg(const TS* __restrict__ Pl, int k, const double* __restrict__ pv,
                                                  int nh, double* h)
{
    const int nq = (nh + 63) >> 6;
    if (nq <= 1) forward_subst_seg_nq<TS, 1>(Pl, k, pv, nh, h);
    else if (nq == 2) forward_subst_seg_nq<TS, 2>(Pl, k, pv, nh, h);
    else if (nq == 3) forward_subst_seg_nq<TS, 3>(Pl, k, pv, nh, h);
    else forward_subst_seg_nq<TS, 4>(Pl, k, pv, nh, h);
}

// Copy row i (entries c < i) of the row-major global pivot block into the
// packed LDS copy.
template <typename TS>
__device__ __forceinline__ void lds_append_row(TS* Pl, int k, const TS* __restrict__ P, int kp1, int i)
{
    for (int c = threadIdx.x; c < i; c += NT) Pl[packed_col(c, k) + (i - c - 1)] = P[(long long)i * kp1 + c];
}

// Bulk-load rows 1..nh-1 of the global pivot block into the packed LDS layout.
template <typename TS>
__device__ __forceinline__ void lds_load_block(TS* Pl, int k, const TS* __restrict__ P, int kp1, int nh)
{
    const int tot = nh * (nh - 1) / 2;
    for (int e = threadIdx.x; e < tot; e += NT) {
        int i = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)e)) * 0.5f);
        while (i * (i - 1) / 2 > e) --i;
        while ((i + 1) * i / 2 <= e) ++i;
        const int c = e - i * (i - 1) / 2;
        Pl[packed_col(c, k) + (i - c - 1)] = P[(long long)i * kp1 + c];
    }
}

// v -= sum_c h[c] * B_c over the thread's elements, columns in increasing
// order.  gi holds a valid index for every slot (masked slots point at a real
// element and are ignored by the caller), so all U * EPT loads of a batch
// issue back to back without branches.
template <typename TS, int EPT>
__device__ __forceinline__ void eliminate(double (&acc)[EPT], const int (&gi)[EPT],
                                          const TS* __restrict__ B, long long ld, const double* h,
                                          int ncols)
{
    constexpr int U = (EPT == 1) ? 32 : ((EPT == 2) ? 8 : 4);
    // unsigned 32-bit byte offsets: loads use a uniform column base + offset
    unsigned off[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) off[i] = (unsigned)gi[i] * (unsigned)sizeof(TS);
    const char* base = (const char*)B;
    const unsigned long long ldb = (unsigned long long)ld * sizeof(TS);
    int c = 0;
    for (; c + U <= ncols; c += U) {
        TS xv[U][EPT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const char* col = base + (unsigned long long)(c + u) * ldb;
#pragma unroll
            for (int i = 0; i < EPT; ++i) xv[u][i] = *(const TS*)(col + off[i]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double hu = h[c + u];
#pragma unroll
            for (int i = 0; i < EPT; ++i) acc[i] = fma(-hu, (double)xv[u][i], acc[i]);
        }
    }
    for (; c < ncols; ++c) {
        const char* col = base + (unsigned long long)c * ldb;
        const double hu = h[c];
        TS xv[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) xv[i] = *(const TS*)(col + off[i]);
#pragma unroll
        for (int i = 0; i < EPT; ++i) acc[i] = fma(-hu, (double)xv[i], acc[i]);
    }
}

// One element of a basis column through a buffer resource: a 32-bit lane
// offset plus a uniform column offset, so a batch of columns costs one VGPR
// per element instead of a 64-bit address per load.  Loads outside the
// resource's byte range return 0.
template <typename TS>
__device__ __forceinline__ TS buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    if constexpr (sizeof(TS) == 8) {
        return __builtin_bit_cast(TS, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
    } else if constexpr (sizeof(TS) == 4) {
        return __builtin_bit_cast(TS, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    } else {
        return __builtin_bit_cast(TS, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    }
}

// raw (unstructured) buffer resource over `bytes` bytes at p
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void* p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// The same elimination with the columns read through one buffer resource
// (fewer address registers; the 16-bit loads of the pointer form get
// serialised by the scheduler under register pressure).  The columns read lie
// in the first ncols * ld elements of B (at most 2^31 bytes; the host limits
// n and k).
template <typename TS, int EPT>
__device__ __forceinline__ void eliminate_buf(double (&acc)[EPT], const int (&gi)[EPT],
                                          const TS* __restrict__ B, long long ld, const double* h,
                                          int ncols)
{
    constexpr int U = (EPT == 1) ? 32 : ((EPT == 2) ? 8 : 4);
    const unsigned ldb = (unsigned)ld * (unsigned)sizeof(TS);
    const __amdgpu_buffer_rsrc_t rs = raw_rsrc(B, (unsigned)ncols * ldb);
    unsigned off[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) off[i] = (unsigned)gi[i] * (unsigned)sizeof(TS);
    int c = 0;
    for (; c + U <= ncols; c += U) {
        TS xv[U][EPT];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int i = 0; i < EPT; ++i) xv[u][i] = buf_load<TS>(rs, off[i], (unsigned)(c + u) * ldb);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double hu = h[c + u];
#pragma unroll
            for (int i = 0; i < EPT; ++i) acc[i] = fma(-hu, (double)xv[u][i], acc[i]);
        }
    }
    for (; c < ncols; ++c) {
        const double hu = h[c];
        TS xv[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) xv[i] = buf_load<TS>(rs, off[i], (unsigned)c * ldb);
#pragma unroll
        for (int i = 0; i < EPT; ++i) acc[i] = fma(-hu, (double)xv[i], acc[i]);
    }
}

// Per-tile argmax |v| (ties: smallest index) -> amv[slot], ami[slot];
// a non-finite value marks the slot with index -2.
template <int EPT>
__device__ __forceinline__ void tile_argmax(const double (&acc)[EPT], const int (&gi)[EPT], unsigned vmask,
                            double* amv, int* ami, int slot)
{
    __shared__ double s_b[NWAVE], s_v[NWAVE];
    __shared__ int s_i[NWAVE], s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    double best = -1.0, val = 0.0;
    int idx = INT_MAX;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        if (!((vmask >> i) & 1u)) continue;
        const double v = acc[i];
        if (!isfinite(v)) bad = true;
        const double av = fabs(v);
        if (am_better(av, gi[i], best, idx)) { best = av; idx = gi[i]; val = v; }
    }
    wave_argmax(best, idx, val);
    __syncthreads();
    if (bad) s_bad = 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { s_b[wave] = best; s_i[wave] = idx; s_v[wave] = val; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NWAVE; ++w)
            if (am_better(s_b[w], s_i[w], best, idx)) { best = s_b[w]; idx = s_i[w]; val = s_v[w]; }
        amv[slot] = val;
        ami[slot] = s_bad ? -2 : idx;
    }
}

// Reduce the G tile partials at amv[off..off+G) (every workgroup does the
// same reduction, so all agree).  Returns the signed value and the index;
// idx = -2 flags non-finite data.
// Global argmax over the G workgroup partials by one wave (the caller's wave
// 0); the result goes to *sv / *si (LDS), -2 if any partial saw a NaN.
__device__ __forceinline__ void global_argmax_wave(const double* amv, const int* ami, int off, int G,
                                                   double* sv, int* si)
{
    const int lane = threadIdx.x & 63;
    double best = -1.0, v = 0.0;
    int bi = INT_MAX;
    int bad = 0;
    int iv[MAXG / 64];
    double vv[MAXG / 64];
#pragma unroll
    for (int u = 0; u < MAXG / 64; ++u) {
        const int q = lane + 64 * u;
        const int qq = off + (q < G ? q : 0);
        iv[u] = ami[qq];
        vv[u] = amv[qq];
    }
#pragma unroll
    for (int u = 0; u < MAXG / 64; ++u) {
        if (lane + 64 * u >= G) continue;
        if (iv[u] == -2) bad = 1;
        if (am_better(fabs(vv[u]), iv[u], best, bi)) { best = fabs(vv[u]); bi = iv[u]; v = vv[u]; }
    }
    wave_argmax(best, bi, v);
    for (int o = 32; o > 0; o >>= 1) bad |= __shfl_xor(bad, o);
    if (lane == 0) { *sv = v; *si = bad ? -2 : bi; }
}

__device__ __forceinline__ void global_argmax(const double* amv, const int* ami, int off, int G, double& val, int& idx)
{
    __shared__ double s_val;
    __shared__ int s_idx;
    if (threadIdx.x < 64) global_argmax_wave(amv, ami, off, G, &s_val, &s_idx);
    __syncthreads();
    val = s_val;
    idx = s_idx;
    __syncthreads();
}

// ------------------------------------------------------------------------
// Sampled partial pivoting (Sec. 3.2: the pivot is the largest magnitude in
// a small random sample of the vector).  Candidate q = 4c + w (c < nc) of
// pivot search i in space sp is the row floor(word_w * len / 2^32) of the
// Philox words of counter (c, i, 3, sp); earlier pivots are skipped and the
// first ms other candidates form the sample (repeats allowed).  The tile that
// owns a candidate publishes its value, or index -1 for a pivot row; after the
// grid barrier every workgroup reads the nc * 4 slots and takes the largest
// |value| (ties to the smaller row).  An empty or all-zero sample leaves the
// full argmax in force.
// ------------------------------------------------------------------------
__device__ __forceinline__ void sample_publish(const Space& sp, int tile, const double* vals, const unsigned* bits,
                                               int len, int nc, uint32_t i, uint32_t space, uint32_t k0,
                                               uint32_t k1, double* sval, int* sidx)
{
    const int q = threadIdx.x;
    if (q < 4 * nc) {
        const Words w = philox10((uint32_t)(q >> 2), i, 3u, space, k0, k1);
        const int u = q & 3;
        const uint32_t word = u == 0 ? w.w[0] : (u == 1 ? w.w[1] : (u == 2 ? w.w[2] : w.w[3]));
        const int r = (int)(((unsigned long long)word * (unsigned)len) >> 32);
        int ot, oe;
        owner_of(sp, r, ot, oe);
        if (ot == tile) {
            const bool piv = (bits[oe >> 5] >> (oe & 31)) & 1u;
            sval[q] = vals[oe];
            sidx[q] = piv ? -1 : r;
        }
    }
}

// Wave level: pivot of the published sample; false if it is empty or all
// zero (the result is uniform over the wave).
__device__ __forceinline__ bool sample_pivot_wave(const double* sval, const int* sidx, int nc, int ms,
                                                  double& val, int& idx)
{
    const int lane = threadIdx.x & 63;
    const int C = 4 * nc;                     // <= SAMPLE_SLOTS <= 128
    const int q0 = lane, q1 = lane + 64;
    const int c0 = min(q0, C - 1), c1 = min(q1, C - 1);
    const int i0r = sidx[c0], i1r = sidx[c1];
    const double v0 = sval[c0], v1 = sval[c1];
    const int i0 = q0 < C ? i0r : -1, i1 = q1 < C ? i1r : -1;
    const unsigned long long m0 = __ballot(i0 >= 0), m1 = __ballot(i1 >= 0);
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const int r0 = __popcll(m0 & below);
    const int r1 = __popcll(m0) + __popcll(m1 & below);
    double best = -1.0, v = 0.0;
    int bi = INT_MAX;
    if (i0 >= 0 && r0 < ms && am_better(fabs(v0), i0, best, bi)) { best = fabs(v0); bi = i0; v = v0; }
    if (i1 >= 0 && r1 < ms && am_better(fabs(v1), i1, best, bi)) { best = fabs(v1); bi = i1; v = v1; }
    wave_argmax(best, bi, v);
    val = v;
    idx = bi;
    return best > 0.0;
}

// Workgroup level: replace (val, idx) of the full argmax by the sample's
// pivot unless the sample is empty or zero or the vector holds a non-finite
// value (idx == -2).
__device__ __forceinline__ void sample_override(const double* sval, const int* sidx, int nc, int ms, double& val, int& idx)
{
    __shared__ double s_v;
    __shared__ int s_i, s_ok;
    if (threadIdx.x < 64) {
        double v;
        int i;
        const bool ok = sample_pivot_wave(sval, sidx, nc, ms, v, i);
        if (threadIdx.x == 0) { s_v = v; s_i = i; s_ok = ok ? 1 : 0; }
    }
    __syncthreads();
    if (s_ok && idx != -2) { val = s_v; idx = s_i; }
    __syncthreads();
}

// ------------------------------------------------------------------------
// per-space state kept in LDS across the whole solve
// ------------------------------------------------------------------------
struct PivState {
    int* list_e;     // local element of each pivot in this tile
    int* list_c;     // basis column of that pivot
    unsigned* bits;  // bitmap of pivot elements of this tile
    int* count;      // number of pivots in this tile
};

template <int EPT>
__device__ __forceinline__ void zero_pivots(double (&acc)[EPT], unsigned vmask, const unsigned* bits)
{
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * NT;
        if (((vmask >> i) & 1u) && ((bits[e >> 5] >> (e & 31)) & 1u)) acc[i] = 0.0;
    }
}

// New pivot p found in column col: if this tile owns it, record it and
// write row col of the global, row-major pivot block (P(col, c) = B_c(p),
// P(col, col) = 1).
template <typename TS>
__device__ __forceinline__ void add_pivot(const Space& sp, int tile, int p, int col, PivState& ps, TS* P, int kp1,
                          const TS* B, long long ld)
{
    int ot, oe;
    owner_of(sp, p, ot, oe);
    if (ot != tile) return;
    for (int c = threadIdx.x; c < col; c += NT) P[(long long)col * kp1 + c] = B[(long long)c * ld + p];
    if (threadIdx.x == 0) {
        P[(long long)col * kp1 + col] = TS(1);
        const int n = *ps.count;
        ps.list_e[n] = oe;
        ps.list_c[n] = col;
        *ps.count = n + 1;
        ps.bits[oe >> 5] |= 1u << (oe & 31);
    }
}

// ------------------------------------------------------------------------
// the persistent basis-iteration kernel
// ------------------------------------------------------------------------
// TB: storage type of the bases; TO: storage type of the operator values,
// of b and of x.
template <typename TB, typename TO, int OP, int SK, int EPT, bool SAMP>
__global__ __launch_bounds__(NT) void iterate_kernel(KArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_cnt_m, s_cnt_n;
    double* h_l = (double*)(smem + a.lds_h);
    double* wt = (double*)(smem + a.lds_w);
    unsigned char* sk = smem + a.lds_sk;
    TB* stage = (TB*)(smem + a.lds_stage);
    double* vert = (double*)(smem + a.lds_vert);
    double* taps = (double*)(smem + a.lds_taps);
    TB* PlD = (TB*)(smem + a.lds_pD);     // packed pivot block of the data-space basis
    TB* PlL = (TB*)(smem + a.lds_pL);     // ... of L (sLSLU; same buffer in bulk mode)

    const int G = a.G;
    const int tile = tile_of_block(G, a.xcd_map);
    const int kp1 = a.k + 1;
    const bool rect = a.rect != 0;
    Ctl* ctl = a.ctl;
    BarState bs;

    PivState pm{(int*)(smem + a.lds_pl_m), (int*)(smem + a.lds_pc_m), (unsigned*)(smem + a.lds_bm_m), &s_cnt_m};
    PivState pn{(int*)(smem + a.lds_pl_n), (int*)(smem + a.lds_pc_n), (unsigned*)(smem + a.lds_bm_n), &s_cnt_n};
    if (!rect) pn = pm;

    const Tile tm = tile_info(a.spm, tile);
    const Tile tn = rect ? tile_info(a.spn, tile) : tm;

    // LDS init
    for (int q = threadIdx.x; q < (NT * EPT + 31) / 32; q += NT) {
        pm.bits[q] = 0u;
        if (rect) pn.bits[q] = 0u;
    }
    if (threadIdx.x == 0) { s_cnt_m = 0; s_cnt_n = 0; }
    PsfL psf{};
    if constexpr (OP == OP_BLUR) psf = psf_stage((unsigned char*)taps, a.r, a.taps_y, a.taps_x, a.toff, a.tw, a.ntap);
    __syncthreads();

    // element ownership of this thread in the m-tile (and n-tile)
    int gm[EPT], gn[EPT];
    unsigned vm = 0u, vn = 0u;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * NT;
        int g = 0;
        if (elem_global(a.spm, tm, e, g)) vm |= 1u << i; else g = 0;
        gm[i] = g;
        if (rect) {
            g = 0;
            if (elem_global(a.spn, tn, e, g)) vn |= 1u << i; else g = 0;
            gn[i] = g;
        } else {
            gn[i] = gm[i];
        }
    }
    if (!rect) vn = vm;

    const TO* bvec = (const TO*)a.b;
    TB* Lb = (TB*)a.L;
    TB* Db = rect ? (TB*)a.D : Lb;   // basis of the data space
    TB* PD = rect ? (TB*)a.PD : (TB*)a.PL;
    TB* PL = (TB*)a.PL;
    double* pvD = rect ? a.pvD : a.pvL;
    double* pvL = a.pvL;
    const long long ldd = rect ? a.ldd : a.ldl;
    const double inv_sk = (SK == SK_SPARSE) ? 1.0 / sqrt((double)a.zeta) : 1.0 / sqrt((double)a.s);

    // CSR: the tiles' row pointers are staged in LDS once (relative to the
    // tile's first entry, when the tile holds fewer than 2^31 entries)
    const int* rpl_m = nullptr;
    const int* rpl_n = nullptr;
    long long rb_m = 0, rb_n = 0;
    if constexpr (OP == OP_CSR) {
        auto stage_rp = [&](const int64_t* rp, const Tile& ti, int off, const int*& dst, long long& base) {
            if (off < 0) return;
            base = rp[ti.start];
            if (rp[ti.start + ti.E] - base >= 0x7fffffffLL) return;   // uniform over the workgroup
            int* l = (int*)(smem + off);
            for (int e = threadIdx.x; e <= ti.E; e += NT) l[e] = (int)(rp[ti.start + e] - base);
            dst = l;
        };
        stage_rp(a.rp, tm, a.lds_rp_m, rpl_m, rb_m);
        if (rect) stage_rp(a.rpt, tn, a.lds_rp_n, rpl_n, rb_n);
        __syncthreads();
    }
    auto op_forward = [&](const TB* xin) {   // wt = A xin on the m-tile
        if constexpr (OP == OP_BLUR) {
            blur_tile<TB>(xin, a.ny, a.nx, a.r, a.bc, tm, a.spm.TY, a.spm.TX, psf, stage, vert, wt);
        } else {
            csr_tile<TO, TB>(a.rp, a.ci, (const TO*)a.cv, xin, tm, a.lpr, wt, rpl_m, rb_m);
        }
    };
    auto op_adjoint = [&](const TB* xin) {   // wt = A^T xin on the n-tile
        if constexpr (OP == OP_CSR)
            csr_tile<TO, TB>(a.rpt, a.cit, (const TO*)a.cvt, xin, tn, a.lprt, wt, rpl_n, rb_n);
    };
    auto finish = [&](int k_done, int status, int nt, int ng) {
        if (tile == 0 && threadIdx.x == 0) {
            ctl->k_done = k_done;
            ctl->nt = nt;
            ctl->ng = ng;
            if (ctl->status == 0) ctl->status = status;
        }
    };
    auto fail = [&](int status) {
        if (tile == 0 && threadIdx.x == 0) ctl->status = status;
    };

    double acc[EPT], accn[EPT];

    if (!hbar_init(ctl, bs, (unsigned)G, a.timeout_ticks)) { fail(-3); return; }

    // ---------------- setup: first pivot(s) and first basis vectors --------
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const double v = (double)bvec[gm[i]];
        acc[i] = ((vm >> i) & 1u) ? v : 0.0;
    }
    tile_argmax<EPT>(acc, gm, vm, a.amv, a.ami, tile);
    // sampled pivoting: slots [0, SAMPLE_SLOTS) hold the candidates of t,
    // [SAMPLE_SLOTS, 2 SAMPLE_SLOTS) those of g
    auto publish = [&](const double (&v)[EPT], const Space& sp, const Tile& ti, const unsigned* bits,
                       int len, int pos, int space) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = threadIdx.x + i * NT;
            if (e < ti.E) wt[e] = v[i];
        }
        __syncthreads();
        sample_publish(sp, tile, wt, bits, len, a.pnc, (uint32_t)pos, (uint32_t)space, a.seed_lo, a.seed_hi,
                       a.sval + space * SAMPLE_SLOTS, a.sidx + space * SAMPLE_SLOTS);
        __syncthreads();
    };
    if constexpr (SAMP) publish(acc, a.spm, tm, pm.bits, a.m, 0, 0);
    if (rect) {
        if constexpr (OP == OP_CSR)                        // v0 = A^T b
            csr_tile<TO, TO>(a.rpt, a.cit, (const TO*)a.cvt, bvec, tn, a.lprt, wt, rpl_n, rb_n);
#pragma unroll
        for (int i = 0; i < EPT; ++i) accn[i] = ((vn >> i) & 1u) ? wt[threadIdx.x + i * NT] : 0.0;
        tile_argmax<EPT>(accn, gn, vn, a.amv, a.ami, G + tile);
        if constexpr (SAMP) publish(accn, a.spn, tn, pn.bits, a.n, 0, 1);
    }
    if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }

    double beta;
    int p1;
    global_argmax(a.amv, a.ami, 0, G, beta, p1);
    if constexpr (SAMP) sample_override(a.sval, a.sidx, a.pnc, a.psamp, beta, p1);
    double alpha = 0.0;
    int g1 = 0;
    if (rect) {
        global_argmax(a.amv, a.ami, G, G, alpha, g1);
        if constexpr (SAMP) sample_override(a.sval + SAMPLE_SLOTS, a.sidx + SAMPLE_SLOTS, a.pnc, a.psamp, alpha, g1);
    }
    if (p1 == -2 || (rect && g1 == -2)) { fail(-4); return; }
    if (beta == 0.0 || (rect && alpha == 0.0)) {
        if (tile == 0 && threadIdx.x == 0 && beta != 0.0) a.tp[0] = p1;
        finish(0, 1, beta != 0.0 ? 1 : 0, 0);
        return;
    }

    // c partial = S2 b (scale from max|b| = |beta|)
    const double scc = fx_scale((double)a.m * fabs(beta) * 1.000001);
    if (a.stepsk) {
        for (int e = threadIdx.x; e < tm.E; e += NT) {
            int gi;
            wt[e] = elem_global(a.spm, tm, e, gi) ? (double)bvec[gi] : 0.0;
        }
        __syncthreads();
        sketch_partial<TO, SK>(a, wt, a.spm, tm, 2u, scc, sk, a.cpart, tile);
        __syncthreads();
    }

    // d1 = b / beta (sLSLU) or l1 = b / beta (sCMRH)
#pragma unroll
    for (int i = 0; i < EPT; ++i)
        if ((vm >> i) & 1u) Db[gm[i]] = (TB)(acc[i] / beta);
    if (rect) {
#pragma unroll
        for (int i = 0; i < EPT; ++i)
            if ((vn >> i) & 1u) Lb[gn[i]] = (TB)(accn[i] / alpha);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    add_pivot<TB>(a.spm, tile, p1, 0, pm, PD, kp1, Db, ldd);
    if (rect) add_pivot<TB>(a.spn, tile, g1, 0, pn, PL, kp1, Lb, a.ldl);
    if (tile == 0 && threadIdx.x == 0) {
        a.tp[0] = p1;
        ctl->beta = beta;
        if (rect) { a.gp[0] = g1; a.W[0] = alpha / beta; }
    }
    if (a.lam > 0.0 && a.stepsk) {   // f_1 = S1 l_1
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = threadIdx.x + i * NT;
            if (e < tn.E) wt[e] = ((vn >> i) & 1u) ? (double)(TB)(rect ? accn[i] / alpha : acc[i] / beta) : 0.0;
        }
        __syncthreads();
        sketch_partial<TO, SK>(a, wt, a.spn, tn, 1u, a.scf, sk, a.fpart, tile);
    }
    if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }

    const double inv_c = (SK == SK_SPARSE) ? inv_sk / scc : inv_sk;
    const double inv_z = (SK == SK_SPARSE) ? inv_sk / a.scz : inv_sk;
    const double inv_f = (SK == SK_SPARSE) ? inv_sk / a.scf : inv_sk;

    // ---------------- basis iteration --------------------------------------
    const TB* PDc = rect ? (const TB*)a.PD : (const TB*)a.PL;
    for (int j = 0; j < a.k; ++j) {
        const int nh = j + 1;
        // ---- phase A: u = A l_j on the m-tile
        if (a.pmode == 0 && j > 0) {        // rows j of the pivot blocks, written last step
            lds_append_row<TB>(PlD, a.k, PDc, kp1, j);
            if (rect) lds_append_row<TB>(PlL, a.k, (const TB*)a.PL, kp1, j);
        }
        op_forward(Lb + (long long)j * a.ldl);
        if (j == 0 && a.stepsk) reduce_partials<SK>(a, a.cpart, inv_c, tile, a.c);
        if (a.lam > 0.0 && a.stepsk) reduce_partials<SK>(a, a.fpart, inv_f, tile, a.F + (long long)j * a.s);
#pragma unroll
        for (int i = 0; i < EPT; ++i) acc[i] = ((vm >> i) & 1u) ? wt[threadIdx.x + i * NT] : 0.0;
        for (int q = threadIdx.x; q < *pm.count; q += NT) pvD[pm.list_c[q]] = wt[pm.list_e[q]];
        if (a.stepsk) sketch_partial<TO, SK>(a, wt, a.spm, tm, 2u, a.scz, sk, a.zpart, tile);
        if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }

        // ---- phase B: coefficients and elimination against the data-space basis
        if (a.pmode == 1) {
            lds_load_block<TB>(PlD, a.k, PDc, kp1, nh);
            __syncthreads();
        }
        if (threadIdx.x < 64) forward_subst<TB>(PlD, a.k, pvD, nh, h_l);
        __syncthreads();
        if (tile == 0)
            for (int i = threadIdx.x; i < nh; i += NT) a.H[(long long)j * kp1 + i] = h_l[i];
        eliminate<TB, EPT>(acc, gm, Db, ldd, h_l, nh);
        zero_pivots<EPT>(acc, vm, pm.bits);
        tile_argmax<EPT>(acc, gm, vm, a.amv, a.ami, tile);
        if (a.stepsk) reduce_partials<SK>(a, a.zpart, inv_z, tile, a.Z + (long long)j * a.s);
        if constexpr (SAMP) {
            __syncthreads();
            publish(acc, a.spm, tm, pm.bits, a.m, j + 1, 0);
        }
        if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }

        // ---- phase C: pivot, normalise, store
        double hv;
        int p;
        global_argmax(a.amv, a.ami, 0, G, hv, p);
        if constexpr (SAMP) sample_override(a.sval, a.sidx, a.pnc, a.psamp, hv, p);
        if (p == -2) { fail(-4); return; }
        if (hv == 0.0 || j + 1 >= a.m) {                 // breakdown (or the space is exhausted)
            if (tile == 0 && threadIdx.x == 0) a.H[(long long)j * kp1 + j + 1] = 0.0;
            finish(j + 1, (j + 1 < a.k) ? 1 : 0, j + 1, rect ? j + 1 : 0);
            return;
        }
        if (tile == 0 && threadIdx.x == 0) {
            a.H[(long long)j * kp1 + j + 1] = hv;
            a.tp[j + 1] = p;
        }
        TB* dst = Db + (long long)(j + 1) * ldd;
#pragma unroll
        for (int i = 0; i < EPT; ++i)
            if ((vm >> i) & 1u) dst[gm[i]] = (TB)(acc[i] / hv);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        add_pivot<TB>(a.spm, tile, p, j + 1, pm, PD, kp1, Db, ldd);

        if (!rect) {
            if (a.lam > 0.0 && j + 1 < a.k && a.stepsk) {
#pragma unroll
                for (int i = 0; i < EPT; ++i) {
                    const int e = threadIdx.x + i * NT;
                    if (e < tm.E) wt[e] = ((vm >> i) & 1u) ? (double)(TB)(acc[i] / hv) : 0.0;
                }
                __syncthreads();
                sketch_partial<TO, SK>(a, wt, a.spm, tm, 1u, a.scf, sk, a.fpart, tile);
            }
            if (j + 1 == a.k) { finish(a.k, 0, a.k + 1, 0); return; }
            if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }
            continue;
        }

        // ---------------- sLSLU: adjoint half step ----------------
        if (j + 1 == a.k) { finish(a.k, 0, a.k + 1, a.k); return; }   // l_{k+1} is not needed for x_k
        if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }

        // ---- phase TA: q = A^T d_{j+1} on the n-tile
        op_adjoint(Db + (long long)(j + 1) * ldd);
#pragma unroll
        for (int i = 0; i < EPT; ++i) acc[i] = ((vn >> i) & 1u) ? wt[threadIdx.x + i * NT] : 0.0;
        for (int q = threadIdx.x; q < *pn.count; q += NT) pvL[pn.list_c[q]] = wt[pn.list_e[q]];
        if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }

        // ---- phase TB: coefficients W(1:j+1, j+2) and elimination against L
        if (a.pmode == 1) {
            lds_load_block<TB>(PlL, a.k, (const TB*)a.PL, kp1, nh);
            __syncthreads();
        }
        if (threadIdx.x < 64) forward_subst<TB>(PlL, a.k, pvL, nh, h_l);
        __syncthreads();
        if (tile == 0)
            for (int i = threadIdx.x; i < nh; i += NT) a.W[(long long)(j + 1) * a.k + i] = h_l[i];
        eliminate<TB, EPT>(acc, gn, Lb, a.ldl, h_l, nh);
        zero_pivots<EPT>(acc, vn, pn.bits);
        tile_argmax<EPT>(acc, gn, vn, a.amv, a.ami, tile);
        if constexpr (SAMP) {
            __syncthreads();
            publish(acc, a.spn, tn, pn.bits, a.n, j + 1, 1);
        }
        if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }

        // ---- phase TC: pivot of L, normalise, store, sketch S1 l_{j+1}
        double wv;
        int g;
        global_argmax(a.amv, a.ami, 0, G, wv, g);
        if constexpr (SAMP) sample_override(a.sval + SAMPLE_SLOTS, a.sidx + SAMPLE_SLOTS, a.pnc, a.psamp, wv, g);
        if (g == -2) { fail(-4); return; }
        if (wv == 0.0 || j + 1 >= a.n) { finish(j + 1, 1, j + 2, j + 1); return; }
        if (tile == 0 && threadIdx.x == 0) {
            a.W[(long long)(j + 1) * a.k + j + 1] = wv;
            a.gp[j + 1] = g;
        }
        TB* ldst = Lb + (long long)(j + 1) * a.ldl;
#pragma unroll
        for (int i = 0; i < EPT; ++i)
            if ((vn >> i) & 1u) ldst[gn[i]] = (TB)(acc[i] / wv);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        add_pivot<TB>(a.spn, tile, g, j + 1, pn, PL, kp1, Lb, a.ldl);
        if (a.lam > 0.0 && a.stepsk) {
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int e = threadIdx.x + i * NT;
                if (e < tn.E) wt[e] = ((vn >> i) & 1u) ? (double)(TB)(acc[i] / wv) : 0.0;
            }
            __syncthreads();
            sketch_partial<TO, SK>(a, wt, a.spn, tn, 1u, a.scf, sk, a.fpart, tile);
        }
        if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail(-3); return; }
    }
}


}  // namespace hk
