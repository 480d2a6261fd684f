// Persistent single-barrier Hessenberg iteration for blur operators (square
// A, the Hessenberg process with partial pivoting of Sec. 3.1,
// eq. (Hessenberg_s), sketched as in Sec. 3.2).
//
// Each step j is one phase between two grid barriers:
//   1. global argmax of v_j (partials of the previous phase): pivot p_j and
//      eta_j = v_j(p_j); l_j = v_j / eta_j is kept as the stored,
//      unnormalised v_j with the FP64 scale s_j = 1 / eta_j;
//   2. reduce last step's sketch partials: z_{j-1} = S2 A l_{j-1},
//      f_{j-1} = S1 l_{j-1};
//   3. coefficients: row j of the pivot block (P(j, i) = l_i(p_j), gathered
//      from the stored basis) and u(p_i) = (A l_j)(p_i) for all pivots:
//      window sums that the tiles owning each pivot's window left in the
//      previous phase, plus one redundant 31x31-type stencil at p_j; then
//      h = P^{-1} u(p) by forward substitution (identical in every
//      workgroup);
//   4. on the tile: u = A l_j (separable blur of v_j with an LDS halo),
//      z_j partials; v_{j+1} = u - sum_i h_i l_i streamed over the stored
//      basis; exact zeros at pivot rows; argmax partial; store v_{j+1};
//      window sums of A v_{j+1} at the pivots whose window meets the tile;
//      f_j partials.
// No inner product is formed; the only global synchronisation per step is
// the grid barrier.
#pragma once
#include "hk_device.hpp"

namespace hk {

struct WBox {
    int ylo, yhi, xlo, xhi;     // source pixels of the pivot's stencil window
    int tyl, tyh, txl, txh;     // tiles that hold them
};

__device__ __forceinline__ WBox wbox(int p, int ny, int nx, int r, int TY, int TX)
{
    const int py = p / nx, px = p - py * nx;
    WBox b;
    b.ylo = max(0, py - r); b.yhi = min(ny - 1, py + r);
    b.xlo = max(0, px - r); b.xhi = min(nx - 1, px + r);
    b.tyl = b.ylo / TY; b.tyh = b.yhi / TY;
    b.txl = b.xlo / TX; b.txh = b.xhi / TX;
    return b;
}

__device__ __forceinline__ double block_sum(double v, double* red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) t += red[w];
    return t;
}

// Several right-hand sides of one operator (a.nrhs, at most RMAX) advance in
// lock step: each has its own basis, pivots, coefficients and sketches (its
// workspace region, a.rhs_stride bytes apart, and its LDS block, a.lds_rhs
// bytes apart; the bases lie side by side, (k + 1) columns each), computed
// exactly as a single solve would; they share the grid barrier of each step
// (the first region's control block) and the argmax round trip.
template <typename TB, typename TO, int SK, int EPT>
__global__ __launch_bounds__(NT) void blur_iterate_kernel(KArgs a0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const KArgs& a = a0;
    __shared__ int s_cnt[RMAX];
    __shared__ int s_done[RMAX];                  // a right-hand side that has finished
    __shared__ double s_red[NWAVE];
    const int nrhs = a0.nrhs;
    // the workspace of right-hand side b: its region and basis (only these
    // pointers differ between right-hand sides)
    struct RhsP {
        double* H; int* tp; double* amv; int* ami;
        long long* zpart; long long* fpart; long long* cpart;
        double* Z; double* F; double* c; Ctl* ctl; double* scale; double* wpart; double* sval; int* sidx;
        void* L; const void* b;
    };
    auto rhs = [&](int b) -> RhsP {
        const long long st = (long long)b * a0.rhs_stride;
        auto sh = [&](auto* q) { return (decltype(q))((char*)q + st); };
        RhsP r;
        r.H = sh(a0.H); r.tp = sh(a0.tp); r.amv = sh(a0.amv); r.ami = sh(a0.ami);
        r.zpart = sh(a0.zpart); r.fpart = sh(a0.fpart); r.cpart = sh(a0.cpart);
        r.Z = sh(a0.Z); r.F = sh(a0.F); r.c = sh(a0.c); r.ctl = sh(a0.ctl);
        r.scale = sh(a0.scale); r.wpart = sh(a0.wpart); r.sval = sh(a0.sval); r.sidx = sh(a0.sidx);
        r.L = (void*)((TB*)a0.L + (long long)b * (a0.k + 1) * a0.ldl);
        r.b = (const void*)((const TO*)a0.b + (long long)b * a0.m);
        return r;
    };
    double* h_l = (double*)(smem + a.lds_h);
    double* hs_l = (double*)(smem + a.lds_hs);
    double* wt = (double*)(smem + a.lds_w);
    unsigned char* sk = smem + a.lds_sk;
    TB* stage = (TB*)(smem + a.lds_stage);
    double* vert = (double*)(smem + a.lds_vert);
    double* taps = (double*)(smem + a.lds_taps);
    using TP = typename PivotT<TB>::type;
    double* wred = (double*)(smem + a.lds_wred);
    // Per right-hand side (bound in its step): the scales s_j = 1 / eta_j
    // and fixed-point scales of f_j (lds_scale), the pivot block P (lds_pD), all pivots (lds_pl_n), the pivots whose window
    // meets this tile (lds_pc_n) and this tile's pivots (lds_pl_m, lds_pc_m,
    // lds_bm_m); right-hand side b's copy lies a.lds_rhs bytes further on
    auto lds_at = [&](int off, int b) { return smem + off + b * a0.lds_rhs; };
    // sparse-sign row lists of S2 and S1 over this tile's elements
    SkRows rows2{}, rows1{};
    if constexpr (SK == SK_SPARSE) {
        const size_t ne = (size_t)a.spm.TY * a.spm.TX * a.zeta;
        unsigned* ob = (unsigned*)(smem + a.lds_skt);
        rows2.offs = ob;
        rows1.offs = ob + (a.s + 1);
        rows2.ents = (unsigned short*)(ob + 2 * (a.s + 1));
        rows1.ents = rows2.ents + ne;
    }
    __shared__ int s_nw[RMAX];                    // length of wlist
    __shared__ double s_amv[RMAX];                // global argmax of the phase
    __shared__ int s_ami[RMAX];

    const int G = a.G;
    const int tile = tile_of_block(G, a.xcd_map);
    const int k = a.k;
    const int kp1 = k + 1;
    const int r = a.r, ny = a.ny, nx = a.nx, TY = a.spm.TY, TX = a.spm.TX;
    const int tw = 2 * r + 1;
    Ctl* ctl = a.ctl;
    BarState bs;

    const Tile tm = tile_info(a.spm, tile);
    const int tyi = tile / a.spm.ntx, txi = tile - tyi * a.spm.ntx;

    for (int b = 0; b < nrhs; ++b) {
        unsigned* bits = (unsigned*)lds_at(a.lds_bm_m, b);
        for (int q = threadIdx.x; q < (NT * EPT + 31) / 32; q += NT) bits[q] = 0u;
    }
    if (threadIdx.x < RMAX) { s_cnt[threadIdx.x] = 0; s_nw[threadIdx.x] = 0; s_done[threadIdx.x] = 0; }
    const PsfL psf = psf_stage((unsigned char*)taps, r, a.taps_y, a.taps_x, a.toff, a.tw, a.ntap);
    const double* tyl = psf.tyl;
    const double* txl = psf.txl;
    // the stencil's taps: the (2r+1)^2 offsets of a separable PSF, or the
    // list of a general one; tap_at gives offset (aa, bb) in [0, 2r] and weight
    const int ntaps = a.ntap > 0 ? a.ntap : tw * tw;
    auto tap_at = [&](int o, int& aa, int& bb) -> double {
        if (a.ntap > 0) {
            const int t = psf.toff[o];
            aa = t >> 16;
            bb = t & 0xffff;
            return psf.tw[o];
        }
        aa = o / tw;
        bb = o - aa * tw;
        return tyl[aa] * txl[bb];
    };
    if constexpr (SK == SK_SPARSE) {
        if (a.stepsk) {
            sketch_rows_build(a.spm, tm, a.s, a.zeta, 2u, a.seed_lo, a.seed_hi, rows2, (unsigned*)sk);
            if (a.lam > 0.0) sketch_rows_build(a.spm, tm, a.s, a.zeta, 1u, a.seed_lo, a.seed_hi, rows1, (unsigned*)sk);
        }
    }

    int gm[EPT];
    unsigned vm = 0u;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        int g = 0;
        if (elem_global(a.spm, tm, threadIdx.x + i * NT, g)) vm |= 1u << i; else g = 0;
        gm[i] = g;
    }
    const long long ld = a.ldl;
    const double inv_sk = (SK == SK_SPARSE) ? 1.0 / sqrt((double)a.zeta) : 1.0 / sqrt((double)a.s);
    const long long GS = (long long)G * a.s;

    // sub-phase timestamps of workgroup 0 (tracing only; the first
    // right-hand side): after the barrier timestamps, 16 slots per step
    unsigned long long* marks = a.trace ? a.trace + 2 * (kp1 + 2) : nullptr;
    int cur_b = 0;
    auto mark = [&](int j, int id) {
        if (marks && cur_b == 0 && tile == 0 && threadIdx.x == 0 && (2 * (kp1 + 2) + j * 16 + id) < a.trace_cap)
            marks[j * 16 + id] = wall_clock64();
    };
    // every right-hand side's status records a failed barrier
    auto fail_all = [&](int status) {
        if (tile == 0 && threadIdx.x == 0)
            for (int b = 0; b < nrhs; ++b) rhs(b).ctl->status = status;
    };
    if (!hbar_init(ctl, bs, (unsigned)G, a.timeout_ticks)) { fail_all(-3); return; }

    // ---- setup: v_0 = b (stored), argmax partial of b
    for (int b = 0; b < nrhs; ++b) {
        const RhsP R = rhs(b);
        TB* V = (TB*)R.L;
        const TO* bvec = (const TO*)R.b;
        PivState pm{(int*)lds_at(a.lds_pl_m, b), (int*)lds_at(a.lds_pc_m, b), (unsigned*)lds_at(a.lds_bm_m, b),
                    &s_cnt[b]};
        double acc[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const TO bv = bvec[gm[i]];
            acc[i] = ((vm >> i) & 1u) ? (double)bv : 0.0;
            if ((vm >> i) & 1u) V[gm[i]] = (TB)bv;
        }
        tile_argmax<EPT>(acc, gm, vm, R.amv + G, R.ami + G, tile);   // read as "previous" by step 0
        if (a.psamp) {   // sample candidates of p_0 (values as stored)
            for (int e = threadIdx.x; e < TY * TX; e += NT) {
                const int yy = e / TX, xx = e - yy * TX;
                const int gy = tm.y0 + yy, gx = tm.x0 + xx;
                wt[e] = (gy < ny && gx < nx) ? (double)(TB)bvec[gy * nx + gx] : 0.0;
            }
            __syncthreads();
            sample_publish(a.spm, tile, wt, pm.bits, a.n, a.pnc, 0u, 0u, a.seed_lo, a.seed_hi,
                           R.sval + SAMPLE_SLOTS, R.sidx + SAMPLE_SLOTS);
        }
    }
    if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail_all(-3); return; }

    for (int j = 0; j <= k; ++j) {
        const int par = j & 1;            // buffers written in this phase
        const int prv = par ^ 1;          // buffers written in the previous phase
        // ---- 1. pivot p_j and eta_j = v_j(p_j) of each right-hand side
        //         (wave b for right-hand side b), overlapped with
        // ---- 2. the previous column's sketch rows of this workgroup's slice
        //         (the other waves, one row per task)
        // the first halo loads of v_j (stored before the barrier) go out
        // here and overlap the pivot search (the first right-hand side)
        TB pre[BLUR_SB];
        unsigned pin = 0u;
        blur_stage_issue<TB>((const TB*)a.L + (long long)j * a.ldl, ny, nx, r, a.bc, tm, TY, TX, pre, pin);
        mark(j, 0);
        {
            const int r0 = (int)(((long long)tile * a.s) / G), r1 = (int)(((long long)(tile + 1) * a.s) / G);
            const int nr = r1 - r0;
            const int ntask = (j >= 1 && a.stepsk) ? nr * ((j == 1 ? 1 : 0) + 1 + (a.lam > 0.0 ? 1 : 0)) : 0;
            const int wave = threadIdx.x >> 6;
            const int w0 = nrhs < NWAVE ? nrhs : NWAVE;     // waves taking an argmax
            if (wave < nrhs && !s_done[wave]) {
                const RhsP ab = rhs(wave);
                global_argmax_wave(ab.amv + prv * G, ab.ami + prv * G, 0, G, &s_amv[wave], &s_ami[wave]);
                if (a.psamp) {
                    double sv;
                    int si;
                    const bool ok = sample_pivot_wave(ab.sval + prv * SAMPLE_SLOTS, ab.sidx + prv * SAMPLE_SLOTS,
                                                      a.pnc, a.psamp, sv, si);
                    if (ok && (threadIdx.x & 63) == 0 && s_ami[wave] != -2) { s_amv[wave] = sv; s_ami[wave] = si; }
                }
            }
            // sketch rows: on the waves left over, or on all waves after the
            // argmax when every wave took one
            if (w0 == NWAVE) __syncthreads();
            const int tw0 = (w0 == NWAVE) ? 0 : w0, twn = NWAVE - tw0;
            if (wave >= tw0) {
                for (int t = wave - tw0; t < ntask * nrhs; t += twn) {
                    const int b = t / max(ntask, 1), tt = t - b * ntask;
                    if (s_done[b]) continue;
                    const RhsP ab = rhs(b);
                    const double* sc_b = (const double*)lds_at(a.lds_scale, b);
                    const int kind = tt / nr, r = r0 + (tt - kind * nr);
                    // partials are FP64 for both sketch kinds in this kernel
                    if (kind == 0) {            // z_{j-1}
                        reduce_row<SK_GAUSS>(ab.zpart + prv * GS, G, a.s, r, inv_sk, ab.Z + (long long)(j - 1) * a.s);
                    } else if (kind == 1 && a.lam > 0.0) {   // f_{j-1}
                        reduce_row<SK_GAUSS>(ab.fpart + prv * GS, G, a.s, r, inv_sk * sc_b[j - 1],
                                             ab.F + (long long)(j - 1) * a.s);
                    } else {                    // c = S2 b (after step 0)
                        reduce_row<SK_GAUSS>(ab.cpart, G, a.s, r, inv_sk, ab.c);
                    }
                }
            }
            __syncthreads();
        }
        mark(j, 1);
      for (int b = 0; b < nrhs; ++b) {
        if (s_done[b]) continue;          // uniform: written before a barrier
        cur_b = b;
        // this right-hand side's region: its pointers are recomputed where
        // used (kernel argument + offset) rather than held in registers
        const long long rst = (long long)b * a0.rhs_stride;
        auto at = [&](auto* q) { return (decltype(q))((char*)q + rst); };
        Ctl* ctl = at(a0.ctl);
        TB* V = (TB*)a0.L + (long long)b * kp1 * a0.ldl;
        const TO* bvec = (const TO*)a0.b + (long long)b * a0.m;
        double* sc_l = (double*)lds_at(a0.lds_scale, b);     // s_j = 1 / eta_j
        double* scf_l = sc_l + kp1;                           // fixed-point scale of f_j
        TP* Pl = (TP*)lds_at(a0.lds_pD, b);
        int* pivs = (int*)lds_at(a0.lds_pl_n, b);
        int* wlist = (int*)lds_at(a0.lds_pc_n, b);
        PivState pm{(int*)lds_at(a0.lds_pl_m, b), (int*)lds_at(a0.lds_pc_m, b), (unsigned*)lds_at(a0.lds_bm_m, b),
                    &s_cnt[b]};
        int& s_nwb = s_nw[b];
        auto finish = [&](int k_done, int status, int nt) {
            if (tile == 0 && threadIdx.x == 0) {
                ctl->k_done = k_done;
                ctl->nt = nt;
                ctl->ng = 0;
                if (ctl->status == 0) ctl->status = status;
            }
        };
        auto done = [&]() {
            if (threadIdx.x == 0) s_done[b] = 1;
        };
        // The argmax compares the values before rounding to the storage
        // type; the pivot entry eta_j is the value as stored, so that
        // l_j = s_j v_j has l_j(p_j) = 1 up to the FP64 reciprocal for
        // every storage type.
        double eta = s_amv[b];
        if constexpr (sizeof(TB) < sizeof(double)) eta = (double)(TB)eta;
        const int p = s_ami[b];
        if (p == -2) {
            if (tile == 0 && threadIdx.x == 0) ctl->status = -4;
            done();
            continue;
        }
        const bool brk = (eta == 0.0) || (j >= a.n);
        mark(j, 2);
        if (brk) {
            if (tile == 0 && threadIdx.x == 0 && j >= 1) at(a0.H)[(long long)(j - 1) * kp1 + j] = 0.0;
            if (j == 0) finish(0, 1, 0);
            else finish(j, (j < k) ? 1 : 0, j);
            done();
            continue;
        }
        const double sj = 1.0 / eta;
        // |v_j| <= |eta_j|: fixed-point scale of the S1 v_j partial sums
        const double scf_j = fx_scale((double)a.n * fabs(eta) * 1.000001);
        if (threadIdx.x == 0) {
            sc_l[j] = sj; scf_l[j] = scf_j; pivs[j] = p;
            const WBox bx = wbox(p, ny, nx, r, TY, TX);
            if (tyi >= bx.tyl && tyi <= bx.tyh && txi >= bx.txl && txi <= bx.txh) wlist[s_nwb++] = j;
        }
        if (tile == 0 && threadIdx.x == 0) {
            at(a0.scale)[j] = sj;
            at(a0.tp)[j] = p;
            if (j >= 1) at(a0.H)[(long long)(j - 1) * kp1 + j] = eta;
            else ctl->beta = eta;
        }
        if (j == k) {
            finish(k, 0, k + 1);
            done();
            continue;
        }
        __syncthreads();
        // ---- 3. coefficients
        {
            int ot, oe;
            owner_of(a.spm, p, ot, oe);
            if (ot == tile && threadIdx.x == 0) {
                const int c = *pm.count;
                pm.list_e[c] = oe;
                pm.list_c[c] = j;
                *pm.count = c + 1;
                pm.bits[oe >> 5] |= 1u << (oe & 31);
            }
        }
        const double scc = fx_scale((double)a.m * fabs(eta) * 1.000001);   // used at j == 0
        mark(j, 3);
        double* pv = wred;                                   // pv[0..j]
        double* slotv = wred + kp1;                          // partials, [i * nslot + q]
        const double* wpp = at(a0.wpart) + (long long)prv * kp1 * a.nslot;
        const TB* vj = V + (long long)j * ld;
        const int py = p / nx, px = p - py * nx;
        const int tot = j * a.nslot;
        // The coefficients depend only on p_j: the row of the pivot block
        // (P(j, c) = l_c(p_j)), the window partials of A v_j left by the
        // tiles in the previous phase and the stencil of (A v_j)(p_j).  Their
        // first loads are all issued before any is consumed, and `middle`
        // (the blur of the sparse-sign path) runs while they are in flight.
        // Leaves pv[0..j] = u(p_0..p_j) in LDS.  Then h = P^{-1} u(p) by
        // forward substitution, the same in every workgroup.
        auto coef_loads = [&](auto&& middle) {
            constexpr int SBW = 2, SBS = 2;
            // (a) pivot-block row: thread c < j (j <= k < NT)
            const TB gv = V[(long long)min((int)threadIdx.x, max(j - 1, 0)) * ld + p];
            // (b) first batch of window partials
            double wv[SBW];
#pragma unroll
            for (int u = 0; u < SBW; ++u) {
                const int q = u * NT + (int)threadIdx.x;
                wv[u] = wpp[q < tot ? q : 0];
            }
            // (c) first batch of stencil taps at p_j
            TB sv[SBS];
            double sw[SBS];
#pragma unroll
            for (int u = 0; u < SBS; ++u) {
                const int o = u * NT + (int)threadIdx.x;
                int aa, bb;
                const double wgt = tap_at(o < ntaps ? o : 0, aa, bb);
                const int y = bc_map(py + aa - r, ny, a.bc), x = bc_map(px + bb - r, nx, a.bc);
                const bool in = o < ntaps && y >= 0 && x >= 0;
                sv[u] = vj[in ? y * nx + x : 0];
                sw[u] = in ? wgt : 0.0;
            }
            middle();
            // consume
            if ((int)threadIdx.x < j)
                Pl[packed_col(threadIdx.x, k) + (j - threadIdx.x - 1)] = (TP)(sc_l[threadIdx.x] * (double)gv);
#pragma unroll
            for (int u = 0; u < SBW; ++u) {
                const int q = u * NT + (int)threadIdx.x;
                if (q < tot) slotv[q] = wv[u];
            }
            for (int q = SBW * NT + (int)threadIdx.x; q < tot; q += NT) slotv[q] = wpp[q];
            double st = 0.0;
#pragma unroll
            for (int u = 0; u < SBS; ++u)
                if (sw[u] != 0.0) st = fma(sw[u], (double)sv[u], st);
            for (int o = SBS * NT + (int)threadIdx.x; o < ntaps; o += NT) {
                int aa, bb;
                const double wgt = tap_at(o, aa, bb);
                const int y = bc_map(py + aa - r, ny, a.bc), x = bc_map(px + bb - r, nx, a.bc);
                if (y >= 0 && x >= 0) st = fma(wgt, (double)vj[y * nx + x], st);
            }
            const double upj = block_sum(st, s_red);         // also publishes Pl and slotv
            for (int i = threadIdx.x; i < j; i += NT) {
                const WBox bx = wbox(pivs[i], ny, nx, r, TY, TX);
                double sum = 0.0;
                for (int ty = bx.tyl; ty <= bx.tyh; ++ty)
                    for (int tx = bx.txl; tx <= bx.txh; ++tx)
                        sum += slotv[i * a.nslot + (ty - bx.tyl) * a.spx + (tx - bx.txl)];
                pv[i] = sj * sum;
            }
            if (threadIdx.x == 0) pv[j] = sj * upj;
            mark(j, 4);
        };
        // wave 0: h by forward substitution, then h_i s_i and column j of H
        auto coef_solve_wave = [&]() {
            mark(j, 5);
            forward_subst_seg<TP>(Pl, k, pv, j + 1, h_l);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int i = threadIdx.x; i <= j; i += 64) hs_l[i] = h_l[i] * sc_l[i];
            if (tile == 0)
                for (int i = threadIdx.x; i <= j; i += 64) at(a0.H)[(long long)j * kp1 + i] = h_l[i];
            mark(j, 6);
        };
        auto c_sketch = [&]() {   // c = S2 b: b itself when the basis type is narrower
            for (int e = threadIdx.x; e < TY * TX; e += NT) {
                const int yy = e / TX, xx = e - yy * TX;
                if constexpr (sizeof(TB) < sizeof(TO)) {
                    const int gy = tm.y0 + yy, gx = tm.x0 + xx;
                    wt[e] = (gy < ny && gx < nx) ? (double)bvec[gy * nx + gx] : 0.0;
                } else {
                    wt[e] = (double)stage[(yy + r) * (TX + 2 * r) + xx + r];
                }
            }
            __syncthreads();
        };
        // ---- 4. the tile: u = A l_j = s_j * blur(v_j), with the coefficient
        //         loads in flight; then h; then (per-step sketches only) the
        //         sketches of u and of v_j
        double acc[EPT];
        const bool fsk = a.lam > 0.0 && a.stepsk;
        coef_loads([&]() {
            mark(j, 12);
            // the first right-hand side's halo loads went out before the
            // argmax; the others issue theirs here
            if (b == 0)
                blur_tile_staged<TB>(V + (long long)j * ld, ny, nx, r, a.bc, tm, TY, TX, psf, stage, vert,
                                     wt, pre, pin, (marks && tile == 0) ? marks + j * 16 + 13 : nullptr);
            else
                blur_tile<TB>(V + (long long)j * ld, ny, nx, r, a.bc, tm, TY, TX, psf, stage, vert, wt);
            mark(j, 7);
        });
#pragma unroll
        for (int i = 0; i < EPT; ++i) acc[i] = ((vm >> i) & 1u) ? sj * wt[threadIdx.x + i * NT] : 0.0;
        if (a.stepsk) {
            for (int e = threadIdx.x; e < TY * TX; e += NT) {
                wt[e] *= sj;
                if (SK == SK_SPARSE && fsk) {   // S1 v_j input (the vertical-pass buffer is free now)
                    const int yy = e / TX, xx = e - yy * TX;
                    vert[e] = (double)stage[(yy + r) * (TX + 2 * r) + xx + r];
                }
            }
        }
        __syncthreads();
        if constexpr (SK == SK_SPARSE) {
            // wave 0 forms h while waves 1..7 form the sketch partials
            if (threadIdx.x < 64) {
                coef_solve_wave();
            } else if (a.stepsk) {
                // z_j partial = S2 u; f_j partial = S1 v_j (scaled by s_j when reduced)
                sketch_rows_sum(wt, rows2, a.s, (double*)(at(a0.zpart) + par * GS + (long long)tile * a.s),
                                (int)threadIdx.x - 64, NT - 64);
                if (fsk)
                    sketch_rows_sum(vert, rows1, a.s, (double*)(at(a0.fpart) + par * GS + (long long)tile * a.s),
                                    (int)threadIdx.x - 64, NT - 64);
            }
        } else {
            if (threadIdx.x < 64) coef_solve_wave();
        }
        __syncthreads();
        mark(j, 15);
        if constexpr (SK == SK_SPARSE) {
            if (j == 0 && a.stepsk) {
                c_sketch();
                sketch_rows_partial(wt, rows2, a.s, (double*)(at(a0.cpart) + (long long)tile * a.s));
            }
        } else if (a.stepsk) {
            sketch_partial<TO, SK>(a, wt, a.spm, tm, 2u, a.scz, sk, at(a0.zpart) + par * GS, tile);   // z_j
            if (j == 0) {
                c_sketch();
                sketch_partial<TO, SK>(a, wt, a.spm, tm, 2u, scc, sk, at(a0.cpart), tile);
            }
            if (a.lam > 0.0) {   // f_j partial = S1 v_j (scaled by s_j when reduced)
                for (int e = threadIdx.x; e < TY * TX; e += NT) {
                    const int yy = e / TX, xx = e - yy * TX;
                    wt[e] = (double)stage[(yy + r) * (TX + 2 * r) + xx + r];
                }
                __syncthreads();
                sketch_partial<TO, SK>(a, wt, a.spm, tm, 1u, scf_j, sk, at(a0.fpart) + par * GS, tile);
            }
        }
        __syncthreads();
        mark(j, 8);
        // v_{j+1} = u - sum_i (h_i s_i) v_i
        eliminate_buf<TB, EPT>(acc, gm, V, ld, hs_l, j + 1);
        mark(j, 9);
        zero_pivots<EPT>(acc, vm, pm.bits);
        tile_argmax<EPT>(acc, gm, vm, at(a0.amv) + par * G, at(a0.ami) + par * G, tile);
        TB* dst = V + (long long)(j + 1) * ld;
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const TB vv = (TB)acc[i];
            if ((vm >> i) & 1u) dst[gm[i]] = vv;
            const int e = threadIdx.x + i * NT;
            if (e < TY * TX) wt[e] = ((vm >> i) & 1u) ? (double)vv : 0.0;
        }
        __syncthreads();
        if (a.psamp)   // sample candidates of p_{j+1} (values as stored)
            sample_publish(a.spm, tile, wt, pm.bits, a.n, a.pnc, (uint32_t)(j + 1), 0u, a.seed_lo, a.seed_hi,
                           at(a0.sval) + par * SAMPLE_SLOTS, at(a0.sidx) + par * SAMPLE_SLOTS);
        mark(j, 10);
        // window sums of A v_{j+1} at the pivots p_0..p_j over this tile's
        // pixels, one wave per pivot.  A window that stays inside the image
        // (or any window under the zero boundary) meets the tile in a
        // rectangle: lanes take its columns (two half-waves split the rows)
        // and the separable weights are applied per column; a window folded
        // by the reflective boundary walks all its offsets.
        {
            const int nw = s_nwb;
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            double* wpc = at(a0.wpart) + (long long)par * kp1 * a.nslot;
            for (int q = wave; q < nw; q += NWAVE) {
                const int i = wlist[q];
                const int p = pivs[i];
                const int py = p / nx, px = p - py * nx;
                double acc2 = 0.0;
                const bool rect = a.bc == 0 || (py - r >= 0 && py + r < ny && px - r >= 0 && px + r < nx);
                if (a.ntap > 0) {
                    // general PSF: lanes take its taps
                    for (int t = lane; t < a.ntap; t += 64) {
                        int aa, bb;
                        const double wgt = tap_at(t, aa, bb);
                        const int y = bc_map(py + aa - r, ny, a.bc), x = bc_map(px + bb - r, nx, a.bc);
                        if (y >= tm.y0 && y < tm.y0 + TY && x >= tm.x0 && x < tm.x0 + TX)
                            acc2 = fma(wgt, wt[(y - tm.y0) * TX + (x - tm.x0)], acc2);
                    }
                } else if (rect) {
                    const int ya = max(max(py - r, tm.y0), 0), yb = min(min(py + r, tm.y0 + TY - 1), ny - 1);
                    const int xa = max(max(px - r, tm.x0), 0), xb = min(min(px + r, tm.x0 + TX - 1), nx - 1);
                    // a window wider than 32 columns (r >= 16) meets a wide
                    // tile in more columns than a half-wave has lanes
                    for (int x = xa + (lane & 31); x <= xb; x += 32) {
                        double cs = 0.0;
                        for (int y = ya + (lane >> 5); y <= yb; y += 2)
                            cs = fma(tyl[y - py + r], wt[(y - tm.y0) * TX + (x - tm.x0)], cs);
                        acc2 = fma(txl[x - px + r], cs, acc2);
                    }
                } else {
                    // reflection folds each axis separately: lanes take the
                    // window's column offsets, half-waves split its rows
                    for (int bb = lane & 31; bb < tw; bb += 32) {
                        const int x = bc_map(px + bb - r, nx, a.bc);
                        if (x < tm.x0 || x >= tm.x0 + TX) continue;
                        double cs = 0.0;
                        for (int aa = lane >> 5; aa < tw; aa += 2) {
                            const int y = bc_map(py + aa - r, ny, a.bc);
                            if (y >= tm.y0 && y < tm.y0 + TY)
                                cs = fma(tyl[aa], wt[(y - tm.y0) * TX + (x - tm.x0)], cs);
                        }
                        acc2 = fma(txl[bb], cs, acc2);
                    }
                }
                acc2 = wave_sum(acc2);
                if (lane == 0) {
                    const WBox bx = wbox(p, ny, nx, r, TY, TX);
                    wpc[(long long)i * a.nslot + (tyi - bx.tyl) * a.spx + (txi - bx.txl)] = acc2;
                }
            }
        }
        mark(j, 11);
        if (b + 1 < nrhs) __syncthreads();   // the next right-hand side reuses the shared LDS buffers
      }
        cur_b = 0;
        // sampled arrival / release times of every workgroup (tracing only)
        unsigned long long* arr = (a.trace && (j & 7) == 4 && (j >> 3) < ARR_SAMPLES)
                                      ? a.trace + a.trace_cap + (long long)(j >> 3) * 2 * MAXG : nullptr;
        if (arr && threadIdx.x == 0) arr[tile] = wall_clock64();
        if (!hbar_sync(ctl, bs, a.timeout_ticks, a.trace, a.trace_cap)) { fail_all(-3); return; }
        if (arr && threadIdx.x == 0) arr[MAXG + tile] = wall_clock64();
        // every right-hand side has finished (the flags were set before the
        // barrier, in every workgroup alike)
        {
            bool all = true;
            for (int b = 0; b < nrhs; ++b) all = all && s_done[b];
            if (all) return;
        }
    }
}

}  // namespace hk
