// Small sketched least-squares solve in one workgroup, blocked:
//   min_y ||c - Z y||^2 + lam^2 ||F y||^2   (lambda-squared weighting, the
//   objective of the sketched Tikhonov problem of Sec. 3.3), i.e. the QR
//   factorisation of M = [Z; lam F] (R rows) with the right-hand side
//   [c; 0] appended as column kd.
//
// Block classical Gram-Schmidt with reorthogonalisation (BCGS2): panels of 16
// columns are held in LDS; each panel is projected twice against the Q
// columns already built (kept in global memory) with FP64 MFMA products
// (W = Q^T P, P -= Q W), then factored inside the panel by CholeskyQR2 on the
// column-scaled panel, which is exact to rounding whenever the panel is well
// conditioned; a panel whose scaled Gram matrix has a pivot below 1e-12 (a
// condition number above about 1e6) is factored by column-by-column CGS2
// instead.  The appended column ends as (d, rho) with d = Q^T [c; 0] and rho
// the norm of the part of [c; 0] outside range(M), so the minimised objective
// with the first j columns is res[j-1] = sqrt(sum_{i >= j} d_i^2 + rho^2),
// and y = R^{-1} d.
#include "hk_device.hpp"

#include <algorithm>

namespace hk {

constexpr int LSB_NT = 512;
constexpr int LSB_NW = LSB_NT / 64;
constexpr int PNB = 16;                            // panel width (the MFMA tile)
constexpr double CHOL_TINY = 1e-12;                // smallest accepted scaled pivot
constexpr int PD = 4;                              // pipelined steps (4 MFMA K steps each) in flight
constexpr int TNK = 16;                            // K steps per batch of the Q^T P product

typedef double d4v __attribute__((ext_vector_type(4)));

// Column stride of the LDS panel: R rounded up to 4 mod 32 doubles, so the 16
// columns x 4 rows that one MFMA operand load touches fall in different banks
// (a stride that is a multiple of 32 doubles puts all 16 columns in one bank).
__device__ __host__ __forceinline__ int panel_ld(int R)
{
    return R + ((4 - R) & 31);
}

// v_mfma_f64_16x16x4f64 operand layout: lane l holds A(l % 16, l / 16) and
// B(l / 16, l % 16); element v of the accumulator is D(l / 16 + 4 v, l % 16)
// (checked on gfx950).
__device__ __forceinline__ d4v mfma16(double a, double b, d4v d)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
}

// Sum over the workgroup of NV values per thread; the totals land in out[]
// (LDS) for every thread to read.  red holds LSB_NW * NV doubles.
template <int NV>
__device__ __forceinline__ void block_multi_sum(double (&v)[NV], double* red, double* out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < NV; ++t) v[t] = wave_sum_to63(v[t]);
    if (lane == 63) {
#pragma unroll
        for (int t = 0; t < NV; ++t) red[wave * NV + t] = v[t];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < LSB_NW; ++w) t += red[w * NV + threadIdx.x];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

__device__ __forceinline__ double block_sum1(double v, double* red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < LSB_NW; ++w) t += red[w];
    __syncthreads();
    return t;
}

// Row-split form: workgroup wg of nwg holds the rows [r0, r1) of M, and a
// sum over all rows is its partial plus the others', added in workgroup
// order, so every workgroup gets the same bits and takes the same branches.
// The partials meet in global memory (double-buffered by call parity: a
// workgroup cannot write call e + 2's partial before every workgroup has
// passed call e + 1's barrier, i.e. finished reading call e's) behind a
// counting barrier on ctl->lsb with the basis kernel's bounded wait.
struct XSum {
    double* part;                // 2 x nwg x cap doubles
    Ctl* ctl;
    unsigned long long timeout;
    int nwg, wg, cap;
    unsigned ep;                 // calls so far
    bool failed;                 // a barrier wait timed out (abort raised)
};

// v (LDS, n <= cap doubles, complete at entry) becomes the sum over the
// workgroups; false after a barrier time-out.
__device__ bool xsum(XSum& x, double* v, int n)
{
    if (x.nwg == 1) return true;
    double* buf = x.part + (size_t)(x.ep & 1u) * x.nwg * x.cap;
    for (int e = threadIdx.x; e < n; e += LSB_NT) buf[(size_t)x.wg * x.cap + e] = v[e];
    ++x.ep;
    __shared__ int s_xok;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&x.ctl->lsb.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool ok = spin_until(&x.ctl->lsb.v, x.ep * (unsigned)x.nwg, x.ctl, x.timeout);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_xok = ok ? 1 : 0;
    }
    __syncthreads();
    if (!s_xok) {
        x.failed = true;
        return false;
    }
    // the partials of 8 workgroups are loaded at once (latency, not
    // bandwidth, bounds this), then added in workgroup order
    for (int e = threadIdx.x; e < n; e += LSB_NT) {
        double t = 0.0;
        for (int w0 = 0; w0 < x.nwg; w0 += 8) {
            double q[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                q[u] = (w0 + u < x.nwg) ? buf[(size_t)(w0 + u) * x.cap + e] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) t += q[u];
        }
        v[e] = t;
    }
    __syncthreads();
    return true;
}

// W[c * 16 + p] = sum_i Q[i * QS + c] P[p * RP + i] for c < j0 (MFMA: A = Q^T
// block, B = P block, K = rows).  Work units: ncb column blocks x nsplit row
// groups, unit u on wave u % 8; row-group partials are summed in group order
// through red (at most 8 x 256 doubles).  A unit
// takes its rows in batches of TNK MFMA K steps (4 rows each) whose loads are
// all issued before the first product; rows past the unit's end are read at
// a clamped address and contribute exact zeros.
__device__ void proj_tn(const double* __restrict__ Q, int QS, int R, int j0, const double* P, double* W, double* red)
{
    // wave-uniform loop control (scalar branches)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ncb = (j0 + 15) >> 4;
    // 5..7 column blocks: two row halves each, so the 10..14 units spread
    // over the four SIMDs more evenly than 5..7 whole units on 8 waves; the
    // first half's sums go to W, the second half's to red (one slot per block)
    const bool halves = ncb > LSB_NW / 2 && ncb < LSB_NW;
    const int nsplit = halves ? 2 : max(1, LSB_NW / ncb);
    const int rows_per = (((R + nsplit - 1) / nsplit) + 3) & ~3;
    const int li = lane & 15, lk = lane >> 4;
    const int nun = ncb * nsplit;
    const int nu = wave < nun ? (nun - 1 - wave) / LSB_NW + 1 : 0;   // units of this wave
    // rows of a unit: [g rows_per, min(R, (g + 1) rows_per)), g = wave % nsplit
    // for every unit of the wave (units u and u + 8 share g); nsplit = 1: all R
    const int gw = nsplit > 1 ? wave % nsplit : 0;
    const int r0 = gw * rows_per, r1 = min(R, r0 + rows_per);
    for (int q = 0; q < nu; ++q) {
        const int u = wave + LSB_NW * q;
        const int cb = u / nsplit;
        const int c = cb * 16 + li;
        const bool cok = c < j0;
        const double* qc = Q + min(c, j0 - 1);
        const double* pc = P + li * panel_ld(R);
        d4v d = {0.0, 0.0, 0.0, 0.0};
        for (int i0 = r0; i0 < r1; i0 += 4 * TNK) {
            double qa[TNK], pb[TNK];
#pragma unroll
            for (int t = 0; t < TNK; ++t) {
                const int row = min(i0 + 4 * t + lk, R - 1);
                qa[t] = qc[(long long)row * QS];
                pb[t] = pc[row];
            }
#pragma unroll
            for (int t = 0; t < TNK; ++t) {
                const bool rok = i0 + 4 * t + lk < r1;
                d = mfma16((cok && rok) ? qa[t] : 0.0, rok ? pb[t] : 0.0, d);
            }
        }
        if (nsplit == 1 || (halves && gw == 0)) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int cr = cb * 16 + lk + 4 * v;
                if (cr < j0) W[cr * PNB + li] = d[v];
            }
        } else {
            const int slot = halves ? cb : wave;
#pragma unroll
            for (int v = 0; v < 4; ++v) red[slot * 256 + (lk + 4 * v) * 16 + li] = d[v];
        }
    }
    if (halves) {
        __syncthreads();
        for (int e = threadIdx.x; e < ncb * 256; e += LSB_NT) {
            const int cb = e >> 8, ij = e & 255;
            const int cr = cb * 16 + (ij >> 4);
            if (cr < j0) W[cr * PNB + (ij & 15)] += red[cb * 256 + ij];
        }
    } else if (nsplit > 1) {
        __syncthreads();
        // unit u = cb * nsplit + g (on wave u) sits in red[u]
        for (int e = threadIdx.x; e < ncb * 256; e += LSB_NT) {
            const int cb = e >> 8, ij = e & 255;
            const int cr = cb * 16 + (ij >> 4);
            double t = 0.0;
            for (int g = 0; g < nsplit; ++g) t += (g * rows_per < R) ? red[(cb * nsplit + g) * 256 + ij] : 0.0;
            if (cr < j0) W[cr * PNB + (ij & 15)] = t;
        }
    }
    __syncthreads();
}

// P[p * RP + i] -= sum_{c < j0} Q[i * QS + c] W[c * 16 + p] (MFMA: D = P block of
// 16 rows, A = Q block, B = W block, K = Q columns).  j0 is a panel start, a
// multiple of 16.  A wave's (row block, 16-column chunk) steps form one
// software pipeline with the loads of the next PD steps in flight; each row
// block takes the columns in increasing order.
__device__ void proj_update(const double* __restrict__ Q, int QS, int R, int j0, double* P, const double* W)
{
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int nrb = (R + 15) >> 4;
    const int nch = j0 >> 4;
    const int RP = panel_ld(R);
    const int nrw = wave < nrb ? (nrb - 1 - wave) / LSB_NW + 1 : 0;   // row blocks of this wave
    const int nit = nrw * nch;
    if (nit == 0) return;
    double qa[PD][4], wb[PD][4];
    int iq = 0, ic = 0;                            // row block and chunk of the next issue
    auto issue = [&](double (&q)[4], double (&w)[4]) {
        const int rb = wave + LSB_NW * min(iq, nrw - 1);
        const double* qrow = Q + (long long)min(rb * 16 + li, R - 1) * QS + 16 * ic;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            q[t] = qrow[4 * t + lk];
            w[t] = W[(16 * ic + 4 * t + lk) * PNB + li];
        }
        if (++ic == nch) { ic = 0; ++iq; }
    };
#pragma unroll
    for (int sl = 0; sl < PD; ++sl) issue(qa[sl], wb[sl]);
    int cq = 0, cc = 0;                            // row block and chunk being consumed
    d4v d;
    for (int it0 = 0; it0 < nit; it0 += PD) {
#pragma unroll
        for (int sl = 0; sl < PD; ++sl) {
            if (it0 + sl < nit) {
                const int rb = wave + LSB_NW * cq;
                const bool rAok = rb * 16 + li < R;
                if (cc == 0) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = rb * 16 + lk + 4 * v;
                        d[v] = row < R ? P[li * RP + row] : 0.0;
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) d = mfma16(rAok ? -qa[sl][t] : 0.0, wb[sl][t], d);
                if (cc == nch - 1) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int row = rb * 16 + lk + 4 * v;
                        if (row < R) P[li * RP + row] = d[v];
                    }
                    cc = 0;
                    ++cq;
                } else {
                    ++cc;
                }
            }
            issue(qa[sl], wb[sl]);                 // unconditional (clamped past the end)
        }
    }
}

// G = P^T P (16 x 16, LDS), rows split over the waves (MFMA with A = P^T and
// B = P: lane l holds the same element P(row, l % 16) for both).
__device__ void panel_gram(const double* P, int R, double* G, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int slice = (((R + LSB_NW - 1) / LSB_NW) + 3) & ~3;
    const int r0 = wave * slice, r1 = min(R, r0 + slice);
    const double* pc = P + li * panel_ld(R);
    d4v d = {0.0, 0.0, 0.0, 0.0};
    int i0 = r0;
    for (; i0 + 16 <= r1; i0 += 16) {              // four K steps' loads first
        double x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) x[t] = pc[i0 + 4 * t + lk];
#pragma unroll
        for (int t = 0; t < 4; ++t) d = mfma16(x[t], x[t], d);
    }
    for (; i0 < r1; i0 += 4) {
        const int row = i0 + lk;
        const double x = row < r1 ? pc[row] : 0.0;
        d = mfma16(x, x, d);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave * 256 + (lk + 4 * v) * 16 + li] = d[v];
    __syncthreads();
    if (threadIdx.x < 256) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < LSB_NW; ++w) t += red[w * 256 + threadIdx.x];
        G[threadIdx.x] = t;
    }
    __syncthreads();
}

// Timestamp of a traced run (tr null otherwise).
__device__ __forceinline__ void lsmark(unsigned long long* tr, int slot)
{
    if (tr && threadIdx.x == 0) tr[slot] = wall_clock64();
}

// Right-looking Cholesky of the nb x nb leading block, row i of the matrix in
// the registers of lane i (lanes 16..63 and rows >= nb hold zeros); column c
// is broadcast by readlane, so a step costs no LDS round trip.  Same
// operations, same order as the textbook right-looking loop.  FULL: nb == 16
// at compile time.  Returns false at a pivot below CHOL_TINY or not finite.
template <bool FULL>
__device__ __forceinline__ bool chol_rows(double (&r)[PNB], int lane, int nb_)
{
    const int nbc = FULL ? PNB : nb_;
    bool ok = true;
#pragma unroll
    for (int c = 0; c < PNB; ++c) {
        if (c < nbc && ok) {                    // uniform over the wave
            const double piv = readlane_d(r[c], c);
            if (!(piv > CHOL_TINY) || !isfinite(piv)) {
                ok = false;
            } else {
                const double lc = sqrt(piv);
                if (lane == c) r[c] = lc;
                else if (lane > c && lane < nbc) r[c] = r[c] / lc;
#pragma unroll
                for (int j = c + 1; j < PNB; ++j) {
                    if (j < nbc) {
                        const double ljc = readlane_d(r[c], j);
                        if (lane >= j && lane < nbc) r[j] = fma(-r[c], ljc, r[j]);
                    }
                }
            }
        }
    }
    return ok;
}

// One CholeskyQR stage on the nb leading panel columns:
//   G = P^T P, s = sqrt(diag G) (scale = true) or 1, S^-1 G S^-1 = L L^T,
//   P <- P S^-1 L^-T, and the stage's factor Rs = L^T S (upper) replaces
//   rcur by Rs rcur.  Returns false (P untouched) when a pivot of the scaled
//   Gram matrix is below CHOL_TINY.  G, Lm, rcur, rtmp: 256 doubles each.
__device__ bool cholqr_stage(double* P, int R, int nb, bool scale, double* G, double* Lm, double* sc,
                             double* rcur, double* rtmp, double* red, int* s_ok, unsigned long long* tr, XSum& xs)
{
    panel_gram(P, R, G, red);
    if (!xsum(xs, G, 256)) return false;
    lsmark(tr, 0);
    const int RP = panel_ld(R);
    if (threadIdx.x < 64) {
        // Cholesky of the scaled Gram matrix, row i in the registers of lane i
        const int lane = threadIdx.x;
        const double sl = (lane < nb && scale) ? sqrt(G[(lane & 15) * 16 + (lane & 15)]) : 1.0;
        if (lane < PNB) sc[lane] = sl;
        double r[PNB];
#pragma unroll
        for (int j = 0; j < PNB; ++j) {
            const double sj = readlane_d(sl, j);
            r[j] = (lane < nb && j < nb) ? G[(lane & 15) * 16 + j] / (sl * sj) : 0.0;
        }
        const bool ok = (nb == PNB) ? chol_rows<true>(r, lane, nb) : chol_rows<false>(r, lane, nb);
        double dg = 1.0;
#pragma unroll
        for (int j = 0; j < PNB; ++j) if (j == lane) dg = r[j];
        if (lane < PNB) {
#pragma unroll
            for (int j = 0; j < PNB; ++j) Lm[lane * 16 + j] = r[j];
        }
        if (lane == 0) *s_ok = ok ? 1 : 0;
        // reciprocals of the scales and of L's diagonal for the row solve
        if (ok && lane < PNB) {
            rtmp[lane] = (lane < nb) ? 1.0 / sl : 0.0;
            rtmp[16 + lane] = (lane < nb) ? 1.0 / dg : 0.0;
        }
    }
    __syncthreads();
    lsmark(tr, 1);
    if (!*s_ok) return false;
    // rows: y L^T = x S^-1, forward over the columns; a thread takes rows i
    // and i + LSB_NT together, two independent chains
    for (int i = threadIdx.x; i < R; i += 2 * LSB_NT) {
        const int i2 = min(i + LSB_NT, R - 1);
        const bool two = i + LSB_NT < R;
        double y[PNB], z[PNB];
#pragma unroll
        for (int j = 0; j < PNB; ++j) {
            double t = (j < nb) ? P[j * RP + i] * rtmp[j] : 0.0;
            double u = (j < nb) ? P[j * RP + i2] * rtmp[j] : 0.0;
#pragma unroll
            for (int q = 0; q < j; ++q) {
                const double l = Lm[j * 16 + q];
                t = fma(-y[q], l, t);
                u = fma(-z[q], l, u);
            }
            y[j] = (j < nb) ? t * rtmp[16 + j] : 0.0;
            z[j] = (j < nb) ? u * rtmp[16 + j] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < PNB; ++j) {
            if (j < nb) {
                P[j * RP + i] = y[j];
                if (two) P[j * RP + i2] = z[j];
            }
        }
    }
    lsmark(tr, 2);
    // rcur <- (L^T S) rcur (G is free once the Cholesky factor is in Lm)
    if (threadIdx.x < 256) {
        const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
        double t = 0.0;
        if (i <= j && j < nb)
            for (int q = i; q <= j; ++q) t = fma(Lm[q * 16 + i] * sc[q], rcur[q * 16 + j], t);
        G[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x < 256) rcur[threadIdx.x] = G[threadIdx.x];
    __syncthreads();
    lsmark(tr, 3);
    return true;
}

template <int NB>
__global__ __launch_bounds__(LSB_NT) void small_ls_blocked_kernel(LsArgs a_in)
{
    const LsArgs a = ls_rebase(a_in, blockIdx.y);     // a row of nwg workgroups per right-hand side
    static_assert(NB == PNB, "panel width is the MFMA tile");
    const int nwg = gridDim.x, wg = blockIdx.x;
    extern __shared__ __align__(16) unsigned char smem[];
    // timestamps: slot 0 start, 1 end, 8 + 8 b + id for panel b
    auto mark = [&](int slot) {
        if (a.trace && threadIdx.x == 0 && slot < LS_TRACE) a.trace[slot] = wall_clock64();
    };
    if (wg == 0) mark(0);
    if (wg == 0)
        for (int i = threadIdx.x; i < a.k; i += LSB_NT) a.res[i] = 0.0;
    if (a.ctl->status < 0) return;
    const int kd = a.ctl->k_done;
    if (kd <= 0) return;
    const int s = a.s, k = a.k;
    const int Rall = a.lam > 0.0 ? 2 * s : s;
    // this workgroup's rows of M: [g0, g0 + R)
    const int g0 = (int)(((long long)wg * Rall) / nwg);
    const int R = (int)(((long long)(wg + 1) * Rall) / nwg) - g0;
    XSum xs{a.xpart, a.ctl, a.timeout, nwg, wg, ls_xcap(k), 0u, false};
    auto fail_barrier = [&]() {
        if (threadIdx.x == 0) {
            a.ctl->ls_status = -3;
            if (a.ctl->status == 0) a.ctl->status = -3;
        }
    };
    const int ncol = kd + 1;                       // basis columns + right-hand side
    const int RP = panel_ld(R);
    double* P = (double*)smem;                     // NB x R panel, column-major, column stride RP
    double* W = P + (size_t)NB * RP;               // (k + 1) x NB projections
    double* red = W + (size_t)(k + 1) * NB;        // LSB_NW x 256
    double* racc = red + LSB_NW * 256;             // (k + 1) x NB: R(0 .. col, col) of the panel (d for column kd)
    double* G = racc + (size_t)(k + 1) * NB;       // 256
    double* Lm = G + 256;                          // 256
    double* rcur = Lm + 256;                       // 256: R of the panel's own block
    double* rtmp = rcur + 256;                     // 256
    double* sc = rtmp + 256;                       // 16
    double* coef = sc + 16;                        // 16
    double* Rm = a.R;                              // k x k, column-major: Rm[col * k + row]
    double* dv = a.d;
    double* Q = a.Q + (long long)g0 * k;           // this workgroup's rows, row-major: Q[i * k + c]
    __shared__ double s_rho;
    __shared__ int s_ok;

    if (wg == 0)
        for (int e = threadIdx.x; e < kd * k; e += LSB_NT) Rm[e] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();

    for (int j0 = 0; j0 < ncol; j0 += NB) {
        const int nb = min(NB, ncol - j0);
        // ---- panel: M(:, j0 .. j0 + nb) (column kd is [c; 0]); unused columns 0.
        // A thread takes rows i and i + LSB_NT of all 16 columns: 32 loads in
        // flight (clamped addresses, masked values), no index division.
        for (int ib = 0; ib < R; ib += 2 * LSB_NT) {
            double v[2][NB];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = g0 + min(ib + h * LSB_NT + (int)threadIdx.x, R - 1);   // row of M
#pragma unroll
                for (int p = 0; p < NB; ++p) {
                    const int col = min(j0 + p, kd);
                    const double* src = (col == kd) ? a.c + min(i, s - 1)
                                      : (i < s ? a.Z + (long long)col * s + i : a.F + (long long)col * s + (i - s));
                    v[h][p] = *src;
                }
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int i = ib + h * LSB_NT + (int)threadIdx.x;     // local row
                if (i < R) {
                    const int gi = g0 + i;
#pragma unroll
                    for (int p = 0; p < NB; ++p) {
                        const int col = j0 + p;
                        double x = 0.0;
                        if (col < kd) x = (gi < s) ? v[h][p] : a.lam * v[h][p];
                        else if (col == kd && gi < s) x = v[h][p];
                        P[p * RP + i] = x;
                    }
                }
            }
        }
        for (int e = threadIdx.x; e < (k + 1) * NB; e += LSB_NT) racc[e] = 0.0;
        if (threadIdx.x < 256) rcur[threadIdx.x] = ((threadIdx.x >> 4) == (threadIdx.x & 15)) ? 1.0 : 0.0;
        __syncthreads();
        const int pb = 8 + 8 * (j0 / NB);
        if (wg == 0) mark(pb);
        // ---- two projections against Q(:, 0 .. j0)
        if (j0 > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                proj_tn(Q, k, R, j0, P, W, red);
                if (!xsum(xs, W, j0 * NB)) { fail_barrier(); return; }
                if (wg == 0) mark(pb + 1 + 2 * pass);
                proj_update(Q, k, R, j0, P, W);
                for (int e = threadIdx.x; e < j0 * NB; e += LSB_NT) racc[e] += W[e];
                __syncthreads();
                if (wg == 0) mark(pb + 2 + 2 * pass);
            }
        }
        // ---- inside the panel: CholeskyQR2 (column-scaled first stage), or
        // CGS2 column by column for an ill-conditioned panel
        int stages = 0;
        // traced runs: slots 160 + 8 b + 4 stage + (0 .. 3) for panel b < 12
        unsigned long long* str = (a.trace && wg == 0 && j0 / NB < 12) ? a.trace + 160 + 8 * (j0 / NB) : nullptr;
        while (stages < 2) {
            unsigned long long* t4 = str ? str + 4 * stages : nullptr;
            if (!cholqr_stage(P, R, nb, stages == 0, G, Lm, sc, rcur, rtmp, red, &s_ok, t4, xs)) break;
            ++stages;
        }
        if (xs.failed) { fail_barrier(); return; }
        if (stages < 2) {
            // rtmp accumulates the CGS2 factor of the current P (upper, 16 x 16)
            if (threadIdx.x < 256) rtmp[threadIdx.x] = 0.0;
            __syncthreads();
            for (int p = 0; p < nb; ++p) {
                if (p > 0) {
                    for (int pass = 0; pass < 2; ++pass) {
                        double part[16];
#pragma unroll
                        for (int t = 0; t < 16; ++t) part[t] = 0.0;
                        for (int i = threadIdx.x; i < R; i += LSB_NT) {
                            const double x = P[p * RP + i];
#pragma unroll
                            for (int t = 0; t < NB; ++t) {
                                const double pt = P[t * RP + i];
                                part[t] = fma(t < p ? pt : 0.0, x, part[t]);
                            }
                        }
                        block_multi_sum<16>(part, red, coef);
                        if (!xsum(xs, coef, 16)) { fail_barrier(); return; }
                        for (int i = threadIdx.x; i < R; i += LSB_NT) {
                            double x = P[p * RP + i];
#pragma unroll
                            for (int t = 0; t < NB; ++t) {
                                const double pt = P[t * RP + i];
                                x = fma(t < p ? -coef[t] : 0.0, pt, x);
                            }
                            P[p * RP + i] = x;
                        }
                        if (threadIdx.x < p) rtmp[threadIdx.x * 16 + p] += coef[threadIdx.x];
                        __syncthreads();
                    }
                }
                double nn = 0.0;
                for (int i = threadIdx.x; i < R; i += LSB_NT) {
                    const double x = P[p * RP + i];
                    nn = fma(x, x, nn);
                }
                double* nsum = coef;           // free here: one slot for the cross-workgroup sum
                const double nloc = block_sum1(nn, red);
                if (threadIdx.x == 0) nsum[0] = nloc;
                __syncthreads();
                if (!xsum(xs, nsum, 1)) { fail_barrier(); return; }
                const double nrm = sqrt(nsum[0]);
                __syncthreads();
                if (nrm > 0.0 && isfinite(nrm))
                    for (int i = threadIdx.x; i < R; i += LSB_NT) P[p * RP + i] = P[p * RP + i] / nrm;
                if (threadIdx.x == 0) rtmp[p * 16 + p] = nrm;
                __syncthreads();
            }
            // rcur <- rtmp rcur (G as scratch)
            if (threadIdx.x < 256) {
                const int i = threadIdx.x >> 4, j = threadIdx.x & 15;
                double t = 0.0;
                if (i <= j && j < nb)
                    for (int q = i; q <= j; ++q) t = fma(rtmp[i * 16 + q], rcur[q * 16 + j], t);
                G[threadIdx.x] = t;
            }
            __syncthreads();
            if (threadIdx.x < 256) rcur[threadIdx.x] = G[threadIdx.x];
            __syncthreads();
        }
        // the panel's own block of R; a basis column with a zero (or non-finite)
        // diagonal makes the sketched problem rank deficient
        if (threadIdx.x < 256) {
            const int i = threadIdx.x >> 4, p = threadIdx.x & 15;
            if (i <= p && p < nb) racc[(j0 + i) * NB + p] = rcur[i * 16 + p];
        }
        if (threadIdx.x == 0) {
            int bad = 0;
            for (int p = 0; p < nb; ++p) {
                const double dg = rcur[p * 16 + p];
                if (j0 + p < kd && (!(dg > 0.0) || !isfinite(dg))) bad = 1;
                if (j0 + p == kd) s_rho = fabs(dg);
            }
            s_ok = bad ? 0 : 1;
        }
        __syncthreads();
        if (!s_ok) {
            if (threadIdx.x == 0) { a.ctl->ls_status = -4; a.ctl->status = -4; }
            return;
        }
        if (wg == 0) mark(pb + 5);
        // ---- the panel's orthonormal columns join Q (this workgroup's rows);
        // its R columns (and d), the same in every workgroup, are written by
        // the first
        for (int e = threadIdx.x; e < R * NB; e += LSB_NT) {
            const int i = e / NB, p = e - i * NB;
            if (p < nb && j0 + p < kd) Q[(long long)i * k + j0 + p] = P[p * RP + i];
        }
        for (int e = threadIdx.x; wg == 0 && e < (j0 + nb) * nb; e += LSB_NT) {
            const int c = e / nb, p = e - c * nb;
            const int col = j0 + p;
            if (c > col) continue;
            if (col < kd) Rm[(long long)col * k + c] = racc[c * NB + p];
            else if (c < kd) dv[c] = racc[c * NB + p];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        if (wg == 0) mark(pb + 6);
    }
    if (wg != 0) return;       // the substitution and the history: the first workgroup
    // ---- residual history and back substitution R y = d (d and the
    // reciprocals of R's diagonal staged in LDS).  The panels are done, so
    // this workgroup's LDS is free: when the strict upper triangle of R
    // (packed by columns, column c holding rows 0 .. c-1 from c(c-1)/2) fits
    // in it beside d, it is staged there as well and the substitution reads
    // R from LDS instead of global memory.
    const size_t lds_dbl = (size_t)NB * RP + 2 * (size_t)(k + 1) * NB + (size_t)LSB_NW * 256 + 4 * 256 + 32;
    const size_t npk = (size_t)kd * (kd - 1) / 2;
    const bool staged = npk + 3 * (size_t)kd <= lds_dbl;
    double* Rp = staged ? (double*)smem : nullptr;
    double* dl = staged ? (double*)smem + npk : W;     // kd, overwritten by the substitution
    double* rd = dl + kd;                              // kd
    double* d2 = dl + 2 * kd;                          // kd, read by the residual loop
    for (int i = threadIdx.x; i < kd; i += LSB_NT) {
        const double di = dv[i];
        dl[i] = di;
        d2[i] = di;
        rd[i] = 1.0 / Rm[(long long)i * k + i];
    }
    if (staged) {
        for (size_t e = threadIdx.x; e < npk; e += LSB_NT) {
            int c = (int)((1.0 + sqrt(1.0 + 8.0 * (double)e)) * 0.5);   // column of packed entry e
            while ((size_t)c * (c - 1) / 2 > e) --c;
            while ((size_t)(c + 1) * c / 2 <= e) ++c;
            const int q = (int)(e - (size_t)c * (c - 1) / 2);
            Rp[e] = Rm[(long long)c * k + q];
        }
    }
    __syncthreads();
    if (threadIdx.x == 64) {                       // wave 1, beside the substitution
        double acc = s_rho * s_rho;
        for (int j = kd - 1; j >= 0; --j) {
            a.res[j] = sqrt(acc);
            acc += d2[j] * d2[j];
        }
    }
    if (threadIdx.x < 64 && staged) {
        // column-oriented as below, with d and the reciprocals in registers
        // (row q = lane + 64 u in slot u) and y_i formed from lane i & 63 by
        // readlane: y_i = d_i (1 / R(i, i)), then d_q = fma(-R(q, i), y_i, d_q)
        // for q < i, the same operations in the same order.  The LDS column
        // of the next RING steps is read ahead.
        constexpr int RING = 4;
        const int lane = threadIdx.x;
        double dr[4], rr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = lane + 64 * u;
            dr[u] = q < kd ? dl[q] : 0.0;
            rr[u] = q < kd ? rd[q] : 0.0;
        }
        double ring[RING][4];
        auto load = [&](int i, double (&dst)[4]) {
            const int c = max(i, 1);
            const double* col = Rp + (size_t)c * (c - 1) / 2;
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[u] = col[min(lane + 64 * u, c - 1)];   // rows >= c masked at use
        };
#pragma unroll
        for (int r = 0; r < RING; ++r) load(kd - 1 - r, ring[r]);
        for (int i0 = kd - 1; i0 >= 0; i0 -= RING) {
#pragma unroll
            for (int r = 0; r < RING; ++r) {
                const int i = i0 - r;
                if (i >= 0) {
                    const int ui = i >> 6, li = i & 63;
                    double ds = dr[0], rs = rr[0];
#pragma unroll
                    for (int u = 1; u < 4; ++u)
                        if (ui == u) { ds = dr[u]; rs = rr[u]; }
                    const double yi = readlane_d(ds, li) * readlane_d(rs, li);
                    if (lane == 0) a.y[i] = yi;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int q = lane + 64 * u;
                        if (q < i) dr[u] = fma(-ring[r][u], yi, dr[u]);
                    }
                }
                load(i - RING, ring[r]);
            }
        }
    } else if (threadIdx.x < 64) {
        // column-oriented: y_i final, then d_q -= R(q, i) y_i for q < i; the
        // R column of the next RING steps is in flight meanwhile
        constexpr int RING = 4;
        const int lane = threadIdx.x;
        double ring[RING][4];
        auto load = [&](int i, double (&dst)[4]) {
            const long long base = (long long)max(i, 0) * k;
#pragma unroll
            for (int u = 0; u < 4; ++u) dst[u] = Rm[base + min(lane + 64 * u, k - 1)];
        };
#pragma unroll
        for (int r = 0; r < RING; ++r) load(kd - 1 - r, ring[r]);
        for (int i0 = kd - 1; i0 >= 0; i0 -= RING) {
#pragma unroll
            for (int r = 0; r < RING; ++r) {
                const int i = i0 - r;
                if (i >= 0) {
                    const double yi = dl[i] * rd[i];
                    __builtin_amdgcn_wave_barrier();
                    if (lane == 0) a.y[i] = yi;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int q = lane + 64 * u;
                        if (q < i) dl[q] = fma(-ring[r][u], yi, dl[q]);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                load(i - RING, ring[r]);
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) a.ctl->ls_status = 0;
    mark(1);
}

// LDS bytes of the blocked kernel (panel width 16)
static size_t lsb_bytes(int rows, int k)
{
    return sizeof(double) * ((size_t)PNB * panel_ld(rows) + 2 * (size_t)(k + 1) * PNB + (size_t)LSB_NW * 256 + 4 * 256 + 32);
}

// Workgroups of the row-split form: about LS_ROWS_PER_WG rows each (one
// workgroup below 256 rows, where the barriers would cost more than the
// rows), at most LS_MWG_MAX.
#ifndef LS_ROWS_PER_WG
#define LS_ROWS_PER_WG 100
#endif
int small_ls_wgs(int s, double lam)
{
    const int rows = lam > 0.0 ? 2 * s : s;
    if (rows < 256) return 1;
    return std::max(1, std::min(LS_MWG_MAX, rows / LS_ROWS_PER_WG));
}

int small_ls_panel(int s, int k, double lam, int nwg, size_t lds_max)
{
    const int rows = lam > 0.0 ? 2 * s : s;
    const int local = (rows + nwg - 1) / std::max(1, nwg);
    if (lsb_bytes(local, k) + 256 <= lds_max) return PNB;  // 256: static LDS of the kernel
    return 0;
}

hipError_t launch_small_ls_blocked(int nb, const LsArgs& a, hipStream_t st)
{
    const int rows = a.lam > 0.0 ? 2 * a.s : a.s;
    const int nwg = std::max(1, a.nwg);
    const size_t lds = lsb_bytes((rows + nwg - 1) / nwg, a.k);
    if (nb != PNB) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)small_ls_blocked_kernel<PNB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(small_ls_blocked_kernel<PNB>, dim3(nwg, std::max(1, a.nrhs)), dim3(LSB_NT), lds, st, a);
    return hipGetLastError();
}

}  // namespace hk
