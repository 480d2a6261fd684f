// Small sketched least-squares solve in one workgroup, blocked:
//   min_y ||c - Z y||^2 + lam^2 ||F y||^2   (lambda-squared weighting, the
//   objective of the sketched Tikhonov problem of Sec. 3.3), i.e. the QR
//   factorisation of M = [Z; lam F] (R rows) with the right-hand side
//   [c; 0] appended as column kd.
//
// Block classical Gram-Schmidt with reorthogonalisation (BCGS2): panels of NB
// columns are held in LDS; each panel is projected twice against the Q
// columns already built (kept in global memory), then orthonormalised column
// by column with CGS2 inside the panel.  The appended column ends as
// (d, rho) with d = Q^T [c; 0] and rho the norm of the part of [c; 0] outside
// range(M), so the minimised objective with the first j columns is
// res[j-1] = sqrt(sum_{i >= j} d_i^2 + rho^2), and y = R^{-1} d.
#include "hk_device.hpp"

namespace hk {

constexpr int LSB_NT = 512;
constexpr int LSB_NW = LSB_NT / 64;
constexpr int LSB_TROWS = 32;     // rows per lane in proj_tn: R <= 4 * LSB_TROWS * LSB_NW

// Sum over the workgroup of NV values per thread; the totals land in out[]
// (LDS) for every thread to read.  red holds LSB_NW * NV doubles.  The NV
// wave sums are independent DPP chains, so they overlap.
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

// W[c * NB + p] = sum_i Q[c * R + i] P[p * R + i] for c < j0, p < NB.
// Blocks of 16 Q columns; wave w takes a slice of the rows; lane (cc, ro)
// handles column cc of the block and rows ro, ro + 4, ... of the slice.
template <int NB>
__device__ void proj_tn(const double* __restrict__ Q, int R, int j0, const double* P, double* W, double* red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int cc = lane & 15, ro = lane >> 4;
    const int slice = (((R + LSB_NW - 1) / LSB_NW) + 3) & ~3;   // <= 4 * LSB_TROWS
    const int r0 = wave * slice, r1 = min(R, r0 + slice);
    const int nt = (max(r1 - r0, 0) + 3) >> 2;                   // rows per lane
    for (int cb = 0; cb < j0; cb += 16) {
        const int c = cb + cc;
        const double* qc = Q + (long long)min(c, j0 - 1) * R;
        double acc[NB];
#pragma unroll
        for (int p = 0; p < NB; ++p) acc[p] = 0.0;
        // the lane's rows in chunks of 16 Q values in flight (clamped
        // addresses; rows past the slice are masked at use)
        for (int t0 = 0; t0 < nt; t0 += 16) {
            double q[16];
#pragma unroll
            for (int t = 0; t < 16; ++t) q[t] = qc[min(r0 + ro + 4 * (t0 + t), R - 1)];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                if (t0 + t < nt) {
                    const int row = r0 + ro + 4 * (t0 + t);
                    const int i = min(row, R - 1);
                    const double qt = (row < r1 && c < j0) ? q[t] : 0.0;
#pragma unroll
                    for (int p = 0; p < NB; ++p) acc[p] = fma(qt, P[p * R + i], acc[p]);
                }
            }
        }
        // sum over the 4 row offsets (lanes cc, cc+16, cc+32, cc+48)
#pragma unroll
        for (int p = 0; p < NB; ++p) {
            acc[p] += __shfl_xor(acc[p], 16);
            acc[p] += __shfl_xor(acc[p], 32);
        }
        if (ro == 0) {
#pragma unroll
            for (int p = 0; p < NB; ++p) red[(wave * 16 + cc) * NB + p] = acc[p];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 16 * NB; e += LSB_NT) {
            const int c2 = cb + e / NB;
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < LSB_NW; ++w) t += red[w * 16 * NB + e];
            if (c2 < j0) W[c2 * NB + (e % NB)] = t;
        }
        __syncthreads();
    }
}

// P[p * R + i] -= sum_{c < j0} Q[c * R + i] W[c * NB + p]; one row per
// thread, columns in increasing order.
template <int NB>
__device__ void proj_update(const double* __restrict__ Q, int R, int j0, double* P, const double* W)
{
    constexpr int U = 16;                          // Q values in flight per thread
    for (int i = threadIdx.x; i < R; i += LSB_NT) {
        double v[NB];
#pragma unroll
        for (int p = 0; p < NB; ++p) v[p] = P[p * R + i];
        for (int c = 0; c < j0; c += U) {
            double q[U];
#pragma unroll
            for (int u = 0; u < U; ++u) q[u] = Q[(long long)min(c + u, j0 - 1) * R + i];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (c + u < j0) {
#pragma unroll
                    for (int p = 0; p < NB; ++p) v[p] = fma(-q[u], W[(c + u) * NB + p], v[p]);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < NB; ++p) P[p * R + i] = v[p];
    }
}

template <int NB>
__global__ __launch_bounds__(LSB_NT) void small_ls_blocked_kernel(LsArgs a)
{
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
    double* red = W + (size_t)(k + 1) * NB;        // LSB_NW x 16 x NB
    double* coef = red + LSB_NW * 16 * NB;         // 16
    double* racc = coef + 16;                      // (k + 1) x NB: R(0 .. col, col) of the panel (d for column kd)
    double* Rm = a.R;                              // k x k, column-major: Rm[col * k + row]
    double* dv = a.d;
    double* Q = a.Q;                               // R x k, column-major
    __shared__ double s_rho;

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
        __syncthreads();
        const int pb = 8 + 8 * (j0 / NB);
        mark(pb);
        // ---- two projections against Q(:, 0 .. j0)
        if (j0 > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                proj_tn<NB>(Q, R, j0, P, W, red);
                mark(pb + 1 + 2 * pass);
                proj_update<NB>(Q, R, j0, P, W);
                for (int e = threadIdx.x; e < j0 * NB; e += LSB_NT) racc[e] += W[e];
                __syncthreads();
                mark(pb + 2 + 2 * pass);
            }
        }
        // ---- inside the panel: CGS2 column by column
        for (int p = 0; p < nb; ++p) {
            const int col = j0 + p;
            // fine marks for the columns of panel 1: 160 + 8 p + id
            const int fm = (j0 == NB) ? 160 + 8 * p : LS_TRACE;
            mark(fm);
            if (p > 0) {
                for (int pass = 0; pass < 2; ++pass) {
                    double part[16];
#pragma unroll
                    for (int t = 0; t < 16; ++t) part[t] = 0.0;
                    // loads are unconditional (all NB panel columns exist);
                    // columns t >= p contribute zero
                    for (int i = threadIdx.x; i < R; i += LSB_NT) {
                        const double x = P[p * R + i];
#pragma unroll
                        for (int t = 0; t < NB; ++t) {
                            const double pt = P[t * R + i];
                            part[t] = fma(t < p ? pt : 0.0, x, part[t]);
                        }
                    }
                    mark(fm + 1 + 3 * pass);
                    block_multi_sum<16>(part, red, coef);
                    mark(fm + 2 + 3 * pass);
                    for (int i = threadIdx.x; i < R; i += LSB_NT) {
                        double x = P[p * R + i];
#pragma unroll
                        for (int t = 0; t < NB; ++t) {
                            const double pt = P[t * R + i];
                            x = fma(t < p ? -coef[t] : 0.0, pt, x);
                        }
                        P[p * R + i] = x;
                    }
                    if (threadIdx.x < p) racc[(j0 + threadIdx.x) * NB + p] += coef[threadIdx.x];
                    __syncthreads();
                    mark(fm + 3 + 3 * pass);
                }
            }
            double nn = 0.0;
            for (int i = threadIdx.x; i < R; i += LSB_NT) {
                const double x = P[p * R + i];
                nn = fma(x, x, nn);
            }
            const double nrm = sqrt(block_sum1(nn, red));
            mark(fm + 7);
            if (col < kd) {
                if (!(nrm > 0.0) || !isfinite(nrm)) {
                    if (threadIdx.x == 0) { a.ctl->ls_status = -4; a.ctl->status = -4; }
                    return;
                }
                for (int i = threadIdx.x; i < R; i += LSB_NT) P[p * R + i] = P[p * R + i] / nrm;
                if (threadIdx.x == 0) racc[col * NB + p] = nrm;
            } else if (threadIdx.x == 0) {
                s_rho = nrm;
            }
            __syncthreads();
        }
        mark(pb + 5);
        // ---- the panel's orthonormal columns join Q; its R columns (and d)
        for (int e = threadIdx.x; e < nb * R; e += LSB_NT) {
            const int p = e / R, i = e - p * R;
            if (j0 + p < kd) Q[(long long)(j0 + p) * R + i] = P[e];
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

// LDS bytes of the blocked kernel for panel width NB
static size_t lsb_bytes(int nb, int rows, int k)
{
    return sizeof(double) * ((size_t)nb * rows + 2 * (size_t)(k + 1) * nb + (size_t)LSB_NW * 16 * nb + 16);
}

int small_ls_panel(int s, int k, double lam, size_t lds_max)
{
    const int rows = lam > 0.0 ? 2 * s : s;
    if (rows <= 4 * LSB_TROWS * LSB_NW && lsb_bytes(16, rows, k) + 256 <= lds_max)
        return 16;                                 // 256: static LDS of the kernel
    return 0;
}

hipError_t launch_small_ls_blocked(int nb, const LsArgs& a, hipStream_t st)
{
    const int rows = a.lam > 0.0 ? 2 * a.s : a.s;
    const size_t lds = lsb_bytes(nb, rows, a.k);
    if (nb != 16) return hipErrorInvalidValue;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)small_ls_blocked_kernel<16>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(small_ls_blocked_kernel<16>, dim3(1), dim3(LSB_NT), lds, st, a);
    return hipGetLastError();
}

}  // namespace hk
