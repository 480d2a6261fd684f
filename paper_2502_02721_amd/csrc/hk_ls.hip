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

namespace hk {

constexpr int LSB_NT = 512;
constexpr int LSB_NW = LSB_NT / 64;
constexpr int PNB = 16;                            // panel width (the MFMA tile)
constexpr double CHOL_TINY = 1e-12;                // smallest accepted scaled pivot

typedef double d4v __attribute__((ext_vector_type(4)));

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

// W[c * 16 + p] = sum_i Q[i * QS + c] P[p * R + i] for c < j0 (MFMA: A = Q^T
// block, B = P block, K = rows).  Work units: ncb column blocks x nsplit row
// groups (at most 8 units at a time, one per wave); row-group partials are
// summed through red (at most 8 x 256 doubles).
__device__ void proj_tn(const double* __restrict__ Q, int QS, int R, int j0, const double* P, double* W, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ncb = (j0 + 15) >> 4;
    const int nsplit = max(1, LSB_NW / ncb);
    const int rows_per = (((R + nsplit - 1) / nsplit) + 3) & ~3;
    const int li = lane & 15, lk = lane >> 4;
    for (int u0 = 0; u0 < ncb * nsplit; u0 += LSB_NW) {
        const int u = u0 + wave;
        const bool active = u < ncb * nsplit;
        const int cb = active ? u / nsplit : 0, g = active ? u - cb * nsplit : 0;
        const int c = cb * 16 + li;
        const bool cok = active && c < j0;
        const double* qc = Q + min(c, j0 - 1);    // row-major Q: qc[row * QS]
        const double* pc = P + li * R;
        const int r0 = g * rows_per, r1 = active ? min(R, r0 + rows_per) : r0;
        d4v d = {0.0, 0.0, 0.0, 0.0};
        int i0 = r0;
        for (; i0 + 16 <= r1; i0 += 16) {          // four K steps in flight
            double qa[4], pb[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int row = i0 + 4 * t + lk;
                qa[t] = qc[(long long)row * QS];
                pb[t] = pc[row];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) d = mfma16(cok ? qa[t] : 0.0, pb[t], d);
        }
        for (; i0 < r1; i0 += 4) {
            const int row = i0 + lk;
            const bool rok = row < r1;
            const double qa = qc[(long long)min(row, R - 1) * QS];
            const double pb = pc[min(row, R - 1)];
            d = mfma16((cok && rok) ? qa : 0.0, rok ? pb : 0.0, d);
        }
        if (nsplit == 1) {
            if (active) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int cr = cb * 16 + lk + 4 * v;
                    if (cr < j0) W[cr * PNB + li] = d[v];
                }
            }
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) red[wave * 256 + (lk + 4 * v) * 16 + li] = active ? d[v] : 0.0;
        }
    }
    if (nsplit > 1) {
        __syncthreads();
        // ncb * nsplit <= LSB_NW here: unit u = cb * nsplit + g sits in red[u]
        for (int e = threadIdx.x; e < ncb * 256; e += LSB_NT) {
            const int cb = e >> 8, ij = e & 255;
            const int cr = cb * 16 + (ij >> 4);
            double t = 0.0;
            for (int g = 0; g < nsplit; ++g) t += red[(cb * nsplit + g) * 256 + ij];
            if (cr < j0) W[cr * PNB + (ij & 15)] = t;
        }
    }
    __syncthreads();
}

// P[p * R + i] -= sum_{c < j0} Q[i * QS + c] W[c * 16 + p] (MFMA: D = P block of
// 16 rows, A = Q block, B = W block, K = Q columns).
__device__ void proj_update(const double* __restrict__ Q, int QS, int R, int j0, double* P, const double* W)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nrb = (R + 15) >> 4;
    for (int rb = wave; rb < nrb; rb += LSB_NW) {
        const int rA = rb * 16 + li;               // row of the A operand
        const bool rAok = rA < R;
        const double* qrow = Q + (long long)min(rA, R - 1) * QS;   // row-major Q
        d4v d;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = rb * 16 + lk + 4 * v;
            d[v] = row < R ? P[li * R + row] : 0.0;
        }
        int c = 0;
        for (; c + 16 <= j0; c += 16) {            // four K steps in flight
            double qa[4], wb[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int cc = c + 4 * t + lk;
                qa[t] = qrow[cc];
                wb[t] = W[cc * PNB + li];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) d = mfma16(rAok ? -qa[t] : 0.0, wb[t], d);
        }
        for (; c < j0; c += 4) {
            const int cc = c + lk;
            const bool ok = cc < j0;
            const double qa = qrow[min(cc, j0 - 1)];
            const double wb = W[min(cc, j0 - 1) * PNB + li];
            d = mfma16((ok && rAok) ? -qa : 0.0, ok ? wb : 0.0, d);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = rb * 16 + lk + 4 * v;
            if (row < R) P[li * R + row] = d[v];
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
    const double* pc = P + li * R;
    d4v d = {0.0, 0.0, 0.0, 0.0};
    for (int i0 = r0; i0 < r1; i0 += 4) {
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

// One CholeskyQR stage on the nb leading panel columns:
//   G = P^T P, s = sqrt(diag G) (scale = true) or 1, S^-1 G S^-1 = L L^T,
//   P <- P S^-1 L^-T, and the stage's factor Rs = L^T S (upper) replaces
//   rcur by Rs rcur.  Returns false (P untouched) when a pivot of the scaled
//   Gram matrix is below CHOL_TINY.  G, Lm, rcur, rtmp: 256 doubles each.
__device__ bool cholqr_stage(double* P, int R, int nb, bool scale, double* G, double* Lm, double* sc,
                             double* rcur, double* rtmp, double* red, int* s_ok)
{
    panel_gram(P, R, G, red);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        if (lane < PNB) sc[lane] = (lane < nb) ? (scale ? sqrt(G[lane * 16 + lane]) : 1.0) : 1.0;
        __builtin_amdgcn_wave_barrier();
        bool ok = true;
        for (int q = lane; q < 256; q += 64) {
            const int i = q >> 4, j = q & 15;
            Lm[q] = (i < nb && j < nb) ? G[q] / (sc[i] * sc[j]) : 0.0;
        }
        __builtin_amdgcn_wave_barrier();
        for (int c = 0; c < nb; ++c) {             // right-looking Cholesky, lower triangle
            const double piv = Lm[c * 16 + c];
            if (!(piv > CHOL_TINY) || !isfinite(piv)) { ok = false; break; }
            const double lc = sqrt(piv);
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) Lm[c * 16 + c] = lc;
            if (lane > c && lane < nb) Lm[lane * 16 + c] = Lm[lane * 16 + c] / lc;
            __builtin_amdgcn_wave_barrier();
            for (int q = lane; q < 256; q += 64) {
                const int i = q >> 4, j = q & 15;
                if (j > c && i >= j && i < nb) Lm[q] = fma(-Lm[i * 16 + c], Lm[j * 16 + c], Lm[q]);
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == 0) *s_ok = ok ? 1 : 0;
        // reciprocals of the scales and of L's diagonal for the row solve
        if (ok && lane < PNB) {
            rtmp[lane] = (lane < nb) ? 1.0 / sc[lane] : 0.0;
            rtmp[16 + lane] = (lane < nb) ? 1.0 / Lm[lane * 16 + lane] : 0.0;
        }
    }
    __syncthreads();
    if (!*s_ok) return false;
    // rows: y L^T = x S^-1, forward over the columns
    for (int i = threadIdx.x; i < R; i += LSB_NT) {
        double y[PNB];
#pragma unroll
        for (int j = 0; j < PNB; ++j) {
            double t = (j < nb) ? P[j * R + i] * rtmp[j] : 0.0;
#pragma unroll
            for (int q = 0; q < j; ++q) t = fma(-y[q], Lm[j * 16 + q], t);
            y[j] = (j < nb) ? t * rtmp[16 + j] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < PNB; ++j)
            if (j < nb) P[j * R + i] = y[j];
    }
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
    return true;
}

template <int NB>
__global__ __launch_bounds__(LSB_NT) void small_ls_blocked_kernel(LsArgs a)
{
    static_assert(NB == PNB, "panel width is the MFMA tile");
    extern __shared__ __align__(16) unsigned char smem[];
    // timestamps: slot 0 start, 1 end, 8 + 8 b + id for panel b
    auto mark = [&](int slot) {
        if (a.trace && threadIdx.x == 0 && slot < LS_TRACE) a.trace[slot] = wall_clock64();
    };
    mark(0);
    for (int i = threadIdx.x; i < a.k; i += LSB_NT) a.res[i] = 0.0;
    if (a.ctl->status < 0) return;
    const int kd = a.ctl->k_done;
    if (kd <= 0) return;
    const int s = a.s, k = a.k;
    const int R = a.lam > 0.0 ? 2 * s : s;
    const int ncol = kd + 1;                       // basis columns + right-hand side
    double* P = (double*)smem;                     // NB x R panel, column-major
    double* W = P + (size_t)NB * R;                // (k + 1) x NB projections
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
    double* Q = a.Q;                               // R x k, row-major: Q[i * k + c]
    __shared__ double s_rho;
    __shared__ int s_ok;

    for (int e = threadIdx.x; e < kd * k; e += LSB_NT) Rm[e] = 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();

    for (int j0 = 0; j0 < ncol; j0 += NB) {
        const int nb = min(NB, ncol - j0);
        // ---- panel: M(:, j0 .. j0 + nb) (column kd is [c; 0]); unused columns 0.
        // Eight loads in flight per thread (clamped addresses, masked values).
        for (int e0 = 0; e0 < NB * R; e0 += 8 * LSB_NT) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = min(e0 + u * LSB_NT + (int)threadIdx.x, NB * R - 1);
                const int p = e / R, i = e - p * R;
                const int col = min(j0 + p, kd);
                const double* src = (col == kd) ? a.c + min(i, s - 1)
                                  : (i < s ? a.Z + (long long)col * s + i : a.F + (long long)col * s + (i - s));
                v[u] = *src;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int e = e0 + u * LSB_NT + (int)threadIdx.x;
                if (e < NB * R) {
                    const int p = e / R, i = e - p * R;
                    const int col = j0 + p;
                    double x = 0.0;
                    if (col < kd) x = (i < s) ? v[u] : a.lam * v[u];
                    else if (col == kd && i < s) x = v[u];
                    P[e] = x;
                }
            }
        }
        for (int e = threadIdx.x; e < (k + 1) * NB; e += LSB_NT) racc[e] = 0.0;
        if (threadIdx.x < 256) rcur[threadIdx.x] = ((threadIdx.x >> 4) == (threadIdx.x & 15)) ? 1.0 : 0.0;
        __syncthreads();
        const int pb = 8 + 8 * (j0 / NB);
        mark(pb);
        // ---- two projections against Q(:, 0 .. j0)
        if (j0 > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                proj_tn(Q, k, R, j0, P, W, red);
                mark(pb + 1 + 2 * pass);
                proj_update(Q, k, R, j0, P, W);
                for (int e = threadIdx.x; e < j0 * NB; e += LSB_NT) racc[e] += W[e];
                __syncthreads();
                mark(pb + 2 + 2 * pass);
            }
        }
        // ---- inside the panel: CholeskyQR2 (column-scaled first stage), or
        // CGS2 column by column for an ill-conditioned panel
        int stages = 0;
        while (stages < 2 && cholqr_stage(P, R, nb, stages == 0, G, Lm, sc, rcur, rtmp, red, &s_ok)) ++stages;
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
                            const double x = P[p * R + i];
#pragma unroll
                            for (int t = 0; t < NB; ++t) {
                                const double pt = P[t * R + i];
                                part[t] = fma(t < p ? pt : 0.0, x, part[t]);
                            }
                        }
                        block_multi_sum<16>(part, red, coef);
                        for (int i = threadIdx.x; i < R; i += LSB_NT) {
                            double x = P[p * R + i];
#pragma unroll
                            for (int t = 0; t < NB; ++t) {
                                const double pt = P[t * R + i];
                                x = fma(t < p ? -coef[t] : 0.0, pt, x);
                            }
                            P[p * R + i] = x;
                        }
                        if (threadIdx.x < p) rtmp[threadIdx.x * 16 + p] += coef[threadIdx.x];
                        __syncthreads();
                    }
                }
                double nn = 0.0;
                for (int i = threadIdx.x; i < R; i += LSB_NT) {
                    const double x = P[p * R + i];
                    nn = fma(x, x, nn);
                }
                const double nrm = sqrt(block_sum1(nn, red));
                if (nrm > 0.0 && isfinite(nrm))
                    for (int i = threadIdx.x; i < R; i += LSB_NT) P[p * R + i] = P[p * R + i] / nrm;
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
        mark(pb + 5);
        // ---- the panel's orthonormal columns join Q; its R columns (and d)
        for (int e = threadIdx.x; e < R * NB; e += LSB_NT) {
            const int i = e / NB, p = e - i * NB;
            if (p < nb && j0 + p < kd) Q[(long long)i * k + j0 + p] = P[p * R + i];
        }
        for (int e = threadIdx.x; e < (j0 + nb) * nb; e += LSB_NT) {
            const int c = e / nb, p = e - c * nb;
            const int col = j0 + p;
            if (c > col) continue;
            if (col < kd) Rm[(long long)col * k + c] = racc[c * NB + p];
            else if (c < kd) dv[c] = racc[c * NB + p];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __syncthreads();
        mark(pb + 6);
    }
    // ---- residual history and back substitution R y = d (d and the
    // reciprocals of R's diagonal staged in LDS)
    double* dl = W;                                // kd, overwritten by the substitution
    double* rd = W + kd;                           // kd
    double* d2 = W + 2 * kd;                       // kd, read by the residual loop
    for (int i = threadIdx.x; i < kd; i += LSB_NT) {
        const double di = dv[i];
        dl[i] = di;
        d2[i] = di;
        rd[i] = 1.0 / Rm[(long long)i * k + i];
    }
    __syncthreads();
    if (threadIdx.x == 64) {                       // wave 1, beside the substitution
        double acc = s_rho * s_rho;
        for (int j = kd - 1; j >= 0; --j) {
            a.res[j] = sqrt(acc);
            acc += d2[j] * d2[j];
        }
    }
    if (threadIdx.x < 64) {
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
    return sizeof(double) * ((size_t)PNB * rows + 2 * (size_t)(k + 1) * PNB + (size_t)LSB_NW * 256 + 4 * 256 + 32);
}

int small_ls_panel(int s, int k, double lam, size_t lds_max)
{
    const int rows = lam > 0.0 ? 2 * s : s;
    if (lsb_bytes(rows, k) + 256 <= lds_max) return PNB;   // 256: static LDS of the kernel
    return 0;
}

hipError_t launch_small_ls_blocked(int nb, const LsArgs& a, hipStream_t st)
{
    const int rows = a.lam > 0.0 ? 2 * a.s : a.s;
    const size_t lds = lsb_bytes(rows, a.k);
    if (nb != PNB) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)small_ls_blocked_kernel<PNB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(small_ls_blocked_kernel<PNB>, dim3(1), dim3(LSB_NT), lds, st, a);
    return hipGetLastError();
}

}  // namespace hk
