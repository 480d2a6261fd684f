// Block sketch: C = S B for a Gaussian embedding S (s x len) that is
// generated on the fly, never stored, and a block B of columns (len x ncol),
// as FP64 MFMA contractions.  Used to sketch a whole basis at the end of a
// solve (Z = S2 A L_k = (S2 L_{k+1}) H_{k+1,k} by the Hessenberg relation,
// eq. (Hessenberg_s) / (Hessenberg_r); F = S1 L_k; c = S2 b): every entry of
// S is generated once per 64-column block of B instead of once per step.
#include "hk_device.hpp"

namespace hk {

typedef double d4v __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: lane l holds A(l % 16, l / 16) and B(l / 16, l % 16);
// element v of the accumulator is D(l / 16 + 4 v, l % 16).
__device__ __forceinline__ d4v bsk_mfma(double a, double b, d4v d)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
}

constexpr int BSK_NT = 256;      // 4 waves; a workgroup computes a 64 x 64 tile of C
constexpr int BSK_KB = 16;       // entries of the contraction per LDS block

// Workgroup b = (ct * rt + rtile) * kc + kchunk sums its chunk of the
// contraction into part[b] (64 x 64, row-major).
template <typename TQ, typename TG>
__global__ __launch_bounds__(BSK_NT) void block_sketch_kernel(BskArgs a)
{
    __shared__ double sS[64][BSK_KB + 1];
    __shared__ double sQ[BSK_KB][64 + 1];
    const int bid = blockIdx.x;
    const int kc = bid % a.kc, tt = bid / a.kc;
    const int rt = tt % a.rt, ct = tt / a.rt;
    const int row0 = rt * 64, col0 = ct * 64;
    const int i_beg = kc * a.chunk, i_end = min(a.len, i_beg + a.chunk);
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const TQ* Q = (const TQ*)a.q;
    d4v acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int i0 = i_beg; i0 < i_end; i0 += BSK_KB) {
        {   // S block: 16 row groups of 4 x 16 entries, one Philox call per thread
            const int g = t >> 4, kk = t & 15;
            const int i = i0 + kk;
            const int grp = (row0 >> 2) + g;
            double gv[4] = {0.0, 0.0, 0.0, 0.0};
            if (i < i_end && 4 * grp < a.s) gauss4<TG>((uint32_t)i, (uint32_t)grp, a.stream, a.k0, a.k1, gv);
#pragma unroll
            for (int q = 0; q < 4; ++q) sS[4 * g + q][kk] = (row0 + 4 * g + q < a.s) ? gv[q] : 0.0;
        }
        {   // B block: 16 x 64, four entries of one column per thread
            const int c = t >> 2, kb = (t & 3) * 4;
            const int col = col0 + c;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + kb + u;
                const bool ok = col < a.ncol && i < i_end;
                const long long idx = ok ? (long long)col * a.ldq + i : 0;
                const double qv = (double)Q[idx];
                sQ[kb + u][c] = ok ? qv : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BSK_KB / 4; ++ks) {
            const double av = sS[16 * w + (lane & 15)][4 * ks + (lane >> 4)];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                acc[c] = bsk_mfma(av, sQ[4 * ks + (lane >> 4)][16 * c + (lane & 15)], acc[c]);
        }
        __syncthreads();
    }
    double* P = a.part + (long long)bid * 4096;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[(16 * w + (lane >> 4) + 4 * v) * 64 + 16 * c + (lane & 15)] = acc[c][v];
}

// out[r + c * ldo] = scale * sum over the chunks, in chunk order.
__global__ __launch_bounds__(256) void block_sketch_reduce(BskArgs a)
{
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long long)a.s * a.ncol) return;
    const int c = (int)(q / a.s), r = (int)(q - (long long)c * a.s);
    const int rt = r >> 6, ct = c >> 6;
    const double* P = a.part + ((long long)(ct * a.rt + rt) * a.kc) * 4096 + (r & 63) * 64 + (c & 63);
    double acc = 0.0;
    for (int k = 0; k < a.kc; ++k) acc += P[(long long)k * 4096];
    a.out[r + (long long)c * a.ldo] = a.scale * acc;
}

// Z(:, j) = sum_{i <= j+1} T(:, i) sc_i H(i, j) and F(:, j) = T1(:, j) sc_j
// (sc: the FP64 column scales of an unnormalised basis, or null).
__global__ __launch_bounds__(256) void sketch_finish_kernel(const double* T, const double* T1, const double* H,
                                                            const double* sc, int s, int k, double* Z, double* F)
{
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= (long long)s * k) return;
    const int j = (int)(q / s), r = (int)(q - (long long)j * s);
    const int kp1 = k + 1;
    double acc = 0.0;
    for (int i = 0; i <= j + 1 && i <= k; ++i) {
        const double h = H[(long long)j * kp1 + i];
        if (h != 0.0) acc = fma(T[(long long)i * s + r] * (sc ? sc[i] : 1.0), h, acc);   // columns past a breakdown
    }
    Z[(long long)j * s + r] = acc;
    if (T1) F[(long long)j * s + r] = T1[(long long)j * s + r] * (sc ? sc[j] : 1.0);
}

// tq: storage of B (0 f64, 1 f32, 2 bf16, 3 f16); tg: generation precision (0 f64, 1 f32)
template <typename TQ>
static void launch_bsk_tq(int tg, const BskArgs& a, hipStream_t st)
{
    const int blocks = a.rt * a.ct * a.kc;
    if (tg == 0) hipLaunchKernelGGL((block_sketch_kernel<TQ, double>), dim3(blocks), dim3(BSK_NT), 0, st, a);
    else hipLaunchKernelGGL((block_sketch_kernel<TQ, float>), dim3(blocks), dim3(BSK_NT), 0, st, a);
}

hipError_t launch_block_sketch(int tq, int tg, const BskArgs& a, hipStream_t st)
{
    if (tq == 0) launch_bsk_tq<double>(tg, a, st);
    else if (tq == 1) launch_bsk_tq<float>(tg, a, st);
    else if (tq == 2) launch_bsk_tq<__bf16>(tg, a, st);
    else launch_bsk_tq<_Float16>(tg, a, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long nout = (long long)a.s * a.ncol;
    hipLaunchKernelGGL(block_sketch_reduce, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sketch_finish(const double* T, const double* T1, const double* H, const double* sc, int s, int k,
                                double* Z, double* F, hipStream_t st)
{
    const long long n = (long long)s * k;
    hipLaunchKernelGGL(sketch_finish_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, T, T1, H, sc, s,
                       k, Z, F);
    return hipGetLastError();
}

}  // namespace hk
