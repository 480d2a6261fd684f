// Non-iterative kernels (small least squares, combine, control reset,
// standalone operator products) and the host-side launchers.
#include "hk_device.hpp"

#include <algorithm>

namespace hk {

// ------------------------------------------------------------------------
// small sketched least squares, one workgroup:
//   min_y ||c - Z y||^2 + lam^2 ||F y||^2,  M = [Z; lam F]
// Classical Gram-Schmidt with one reorthogonalisation pass (CGS2) builds
// M = Q R column by column; the right-hand side is projected column by
// column, so res[j] is the minimised objective with the first j+1 columns.
// ------------------------------------------------------------------------
constexpr int LS_NT = 1024;
constexpr int LS_NW = LS_NT / 64;

__device__ double block_sum_ls(double v, double* red)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < LS_NW; ++w) t += red[w];
    return t;
}

__global__ __launch_bounds__(LS_NT) void small_ls_kernel(LsArgs a_in)
{
    const LsArgs a = ls_rebase(a_in, blockIdx.x);     // one workgroup per right-hand side
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[LS_NW];
    for (int i = threadIdx.x; i < a.k; i += LS_NT) a.res[i] = 0.0;
    if (a.ctl->status < 0) return;
    const int kd = a.ctl->k_done;
    if (kd <= 0) return;
    const int s = a.s;
    const bool tik = a.lam > 0.0;
    const int rows = tik ? 2 * s : s;
    double* av = (double*)smem;           // rows
    double* coef = av + rows;             // k
    double* Q = a.Q;                      // rows x k
    double* R = a.R;                      // k x k, column-major
    double* r = a.r;                      // rows: residual of the right-hand side

    for (int i = threadIdx.x; i < rows; i += LS_NT) r[i] = (i < s) ? a.c[i] : 0.0;
    for (int i = threadIdx.x; i < a.k * a.k; i += LS_NT) R[i] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = 0; j < kd; ++j) {
        for (int i = threadIdx.x; i < rows; i += LS_NT)
            av[i] = (i < s) ? a.Z[(long long)j * s + i] : a.lam * a.F[(long long)j * s + (i - s)];
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int c = wave; c < j; c += LS_NW) {
                const double* qc = Q + (long long)c * rows;
                double d = 0.0;
                for (int i = lane; i < rows; i += 64) d = fma(qc[i], av[i], d);
                d = wave_sum(d);
                if (lane == 0) coef[c] = d;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < rows; i += LS_NT) {
                double t = av[i];
                for (int c = 0; c < j; ++c) t = fma(-Q[(long long)c * rows + i], coef[c], t);
                av[i] = t;
            }
            for (int c = threadIdx.x; c < j; c += LS_NT) R[(long long)j * a.k + c] += coef[c];
            __syncthreads();
        }
        double nn = 0.0;
        for (int i = threadIdx.x; i < rows; i += LS_NT) nn = fma(av[i], av[i], nn);
        const double nrm = sqrt(block_sum_ls(nn, red));
        if (!(nrm > 0.0) || !isfinite(nrm)) {
            if (threadIdx.x == 0) { a.ctl->ls_status = -4; a.ctl->status = -4; }
            return;
        }
        if (threadIdx.x == 0) R[(long long)j * a.k + j] = nrm;
        double dd = 0.0;
        for (int i = threadIdx.x; i < rows; i += LS_NT) {
            const double q = av[i] / nrm;
            Q[(long long)j * rows + i] = q;
            dd = fma(q, r[i], dd);
        }
        const double dj = block_sum_ls(dd, red);
        double rr = 0.0;
        for (int i = threadIdx.x; i < rows; i += LS_NT) {
            const double t = fma(-dj, Q[(long long)j * rows + i], r[i]);
            r[i] = t;
            rr = fma(t, t, rr);
        }
        const double rn = sqrt(block_sum_ls(rr, red));
        if (threadIdx.x == 0) { a.d[j] = dj; a.res[j] = rn; }
        __syncthreads();
    }
    // back substitution R y = d by wave 0, column-oriented, d staged in LDS
    for (int i = threadIdx.x; i < kd; i += LS_NT) coef[i] = a.d[i];
    __syncthreads();
    if (threadIdx.x < 64) {
        for (int i = kd - 1; i >= 0; --i) {
            const double yi = coef[i] * (1.0 / R[(long long)i * a.k + i]);
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) a.y[i] = yi;
            for (int q = lane; q < i; q += 64) coef[q] = fma(-R[(long long)i * a.k + q], yi, coef[q]);
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (threadIdx.x == 0) a.ctl->ls_status = 0;
}

// ------------------------------------------------------------------------
// x = L_k y (FP64 accumulation, columns in increasing order)
// ------------------------------------------------------------------------
template <typename TB, typename TO>
__global__ __launch_bounds__(256) void combine_kernel(CombineArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int b = blockIdx.y;                           // right-hand side
    const long long st_b = (long long)b * a.rhs_stride;
    const TB* L = (const TB*)a.L + (long long)b * (a.k + 1) * a.ldl;
    TO* x = (TO*)a.x + (long long)b * a.n;
    const Ctl* ctl = (const Ctl*)((const char*)a.ctl + st_b);
    const double* y = (const double*)((const char*)a.y + st_b);
    const double* scale = a.scale ? (const double*)((const char*)a.scale + st_b) : nullptr;
    const int st = ctl->status;
    int kd = (st < 0) ? 0 : ctl->k_done;
    if (a.kcap > 0) kd = min(kd, a.kcap);
    // unrolled so that the loads of 16 columns are in flight together; the
    // FMAs still run in increasing j
    double acc = 0.0;
    if (scale) {
#pragma unroll 16
        for (int j = 0; j < kd; ++j) acc = fma((double)L[(long long)j * a.ldl + i], y[j] * scale[j], acc);
    } else {
#pragma unroll 16
        for (int j = 0; j < kd; ++j) acc = fma((double)L[(long long)j * a.ldl + i], y[j], acc);
    }
    x[i] = (TO)acc;
}

// Unsketched projected problem (CMRH / LSLU): F = [I; 0] (s = k + 1 rows)
// and c = beta e_1; Z is H itself.
__global__ __launch_bounds__(256) void hess_rhs_kernel(double* F, double* c, int s, int k, double lam,
                                                        const Ctl* ctl)
{
    for (int i = threadIdx.x; i < s; i += 256) c[i] = (i == 0) ? ctl->beta : 0.0;
    if (lam > 0.0)
        for (int q = threadIdx.x; q < s * k; q += 256) {
            const int j = q / s, i = q - j * s;
            F[q] = (i == j) ? 1.0 : 0.0;
        }
}

hipError_t launch_hess_rhs(double* F, double* c, int s, int k, double lam, const Ctl* ctl, hipStream_t st)
{
    hipLaunchKernelGGL(hess_rhs_kernel, dim3(1), dim3(256), 0, st, F, c, s, k, lam, ctl);
    return hipGetLastError();
}

__global__ void ctl_init_kernel(Ctl* ctl)
{
    unsigned* w = (unsigned*)ctl;
    for (unsigned i = threadIdx.x; i < sizeof(Ctl) / sizeof(unsigned); i += blockDim.x) w[i] = 0u;
}

// ------------------------------------------------------------------------
// standalone operator product y = A x or A^T x (tiles of the output space)
// ------------------------------------------------------------------------
template <typename TS, int OP>
__global__ __launch_bounds__(NT) void apply_kernel(ApplyArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double* wt = (double*)(smem + a.lds_w);
    TS* stage = (TS*)(smem + a.lds_stage);
    double* vert = (double*)(smem + a.lds_vert);
    double* taps = (double*)(smem + a.lds_taps);
    const Tile ti = tile_info(a.sp, blockIdx.x);
    if constexpr (OP == OP_BLUR) {
        const PsfL psf = psf_stage((unsigned char*)taps, a.r, a.taps_y, a.taps_x, a.toff, a.tw, a.ntap);
        __syncthreads();
        blur_tile<TS>((const TS*)a.x, a.ny, a.nx, a.r, a.bc, ti, a.sp.TY, a.sp.TX, psf, stage, vert, wt);
    } else {
        csr_tile<TS, TS>(a.rp, a.ci, (const TS*)a.cv, (const TS*)a.x, ti, a.lpr, wt);
    }
    TS* y = (TS*)a.y;
    for (int e = threadIdx.x; e < ti.E; e += NT) {
        int gi;
        if (elem_global(a.sp, ti, e, gi)) y[gi] = (TS)wt[e];
    }
}

// ------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------
const void* select_iterate_f64(int op, int sketch, int ept, int samp);
const void* select_iterate_f32(int op, int sketch, int ept, int samp);
const void* select_iterate_mix(int op, int sketch, int ept, int samp);
const void* select_blur_f64(int sketch, int ept);
const void* select_blur_f32(int sketch, int ept);
const void* select_blur_mix(int sketch, int ept);
const void* select_blur_h16(int tb, int sketch, int ept);

// basis storage / operator storage: (f64, f64), (f32, f32), (f64, f32), and
// for the single-barrier blur kernel also (bf16, f32) and (f16, f32).
// op = OP_BLUR_ONEBAR selects the single-barrier blur kernel
// samp: the generic kernel is instantiated with and without sampled pivoting
// (the sampling code costs the CSR products registers when compiled in)
static const void* select_iterate(int tb, int to, int op, int sketch, int ept, int samp)
{
    if (op == OP_BLUR_ONEBAR) {
        if (tb == 0 && to == 0) return select_blur_f64(sketch, ept);
        if (tb == 1 && to == 1) return select_blur_f32(sketch, ept);
        if (tb == 0 && to == 1) return select_blur_mix(sketch, ept);
        if ((tb == 2 || tb == 3) && to == 1) return select_blur_h16(tb, sketch, ept);
        return nullptr;
    }
    if (tb == 0 && to == 0) return select_iterate_f64(op, sketch, ept, samp);
    if (tb == 1 && to == 1) return select_iterate_f32(op, sketch, ept, samp);
    if (tb == 0 && to == 1) return select_iterate_mix(op, sketch, ept, samp);
    return nullptr;
}

hipError_t iterate_occupancy(int tb, int to, int op, int sketch, int ept, int samp, int lds_bytes,
                             int* blocks_per_cu)
{
    const void* f = select_iterate(tb, to, op, sketch, ept, samp);
    if (!f) return hipErrorInvalidValue;
    if (lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, NT, lds_bytes);
}

hipError_t launch_iterate(int tb, int to, int op, int sketch, int ept, const KArgs& a, hipStream_t st)
{
    const void* f = select_iterate(tb, to, op, sketch, ept, a.psamp > 0 ? 1 : 0);
    if (f && a.lds_total > 65536) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds_total);
        if (e != hipSuccess) return e;
    }
    if (!f) return hipErrorInvalidValue;
    KArgs args = a;
    void* kargs[] = {&args};
    // A cooperative launch guarantees that the whole grid is resident, but
    // such launches do not run side by side.  A capped grid (a.coop == 0) is
    // launched as an ordinary kernel: its workgroups are co-resident as long
    // as the grids running at once fit on the device (one workgroup per
    // compute unit), which the caller keeps; the grid barrier's time-out
    // turns a violation into an error instead of a hang.
    if (a.coop) return hipLaunchCooperativeKernel(f, dim3(a.G), dim3(NT), kargs, (unsigned)a.lds_total, st);
    return hipLaunchKernel(f, dim3(a.G), dim3(NT), kargs, (unsigned)a.lds_total, st);
}

hipError_t launch_ctl_init(Ctl* ctl, hipStream_t st)
{
    hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(256), 0, st, ctl);
    return hipGetLastError();
}

// Zero `n16` 16-byte words (a kernel rather than a memset node, so that the
// sequence stays capturable in a HIP graph).
__global__ __launch_bounds__(256) void fill_zero_kernel(uint4* p, size_t n16)
{
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (size_t)gridDim.x * 256) p[i] = z;
}

// info[0] = status of the run (an aborted grid barrier is HK_EDEVICE),
// info[1] = basis columns built
__global__ void solve_info_kernel(const Ctl* ctl, int32_t* info)
{
    if (threadIdx.x == 0) {
        info[0] = ctl->abort ? -3 : ctl->status;
        info[1] = ctl->k_done;
    }
}

hipError_t launch_solve_info(const Ctl* ctl, int32_t* info, hipStream_t st)
{
    hipLaunchKernelGGL(solve_info_kernel, dim3(1), dim3(64), 0, st, ctl, info);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)p & 15u) || (bytes & 15u)) return hipErrorInvalidValue;
    const size_t n16 = bytes / 16;
    const size_t want = (n16 + 255) / 256;
    const unsigned blocks = (unsigned)std::min<size_t>(want, 4096);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, st, (uint4*)p, n16);
    return hipGetLastError();
}

size_t small_ls_lds_bytes(int s, int k, double lam)
{
    const int rows = lam > 0.0 ? 2 * s : s;
    return sizeof(double) * (size_t)(rows + k);
}

hipError_t launch_small_ls(const LsArgs& a, hipStream_t st)
{
    if (a.nb > 0) return launch_small_ls_blocked(a.nb, a, st);
    const size_t lds = small_ls_lds_bytes(a.s, a.k, a.lam);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)small_ls_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(small_ls_kernel, dim3(std::max(1, a.nrhs)), dim3(LS_NT), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_combine(int tb, int to, const CombineArgs& a, int nrhs, hipStream_t st)
{
    const dim3 blocks((a.n + 255) / 256, std::max(1, nrhs));
    if (tb == 0 && to == 0) hipLaunchKernelGGL((combine_kernel<double, double>), dim3(blocks), dim3(256), 0, st, a);
    else if (tb == 1 && to == 1) hipLaunchKernelGGL((combine_kernel<float, float>), dim3(blocks), dim3(256), 0, st, a);
    else if (tb == 0 && to == 1) hipLaunchKernelGGL((combine_kernel<double, float>), dim3(blocks), dim3(256), 0, st, a);
    else if (tb == 2 && to == 1) hipLaunchKernelGGL((combine_kernel<__bf16, float>), dim3(blocks), dim3(256), 0, st, a);
    else if (tb == 3 && to == 1) hipLaunchKernelGGL((combine_kernel<_Float16, float>), dim3(blocks), dim3(256), 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Prefix solution of the small problem: with [Z; lambda F] = Q R, the first
// kp columns have the factors Q(:, 1:kp), R(1:kp, 1:kp), so
// y_kp = R(1:kp, 1:kp)^{-1} d(1:kp), d = Q^T [c; 0] (eq. (sketched_LSLU),
// eq. (sketched_LSLU_hybrid) restricted to the first kp basis vectors).
// One wave, column-oriented like the least-squares kernels' substitution.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(64) void prefix_y_kernel(const double* R, const double* d, int k, int kp, int recip,
                                                      double* yp)
{
    __shared__ double dl[256];
    const int lane = threadIdx.x;
    for (int i = lane; i < kp; i += 64) dl[i] = d[i];
    __syncthreads();
    for (int i = kp - 1; i >= 0; --i) {
        const double rii = R[(long long)i * k + i];
        const double yi = recip ? dl[i] * (1.0 / rii) : dl[i] / rii;
        __syncthreads();
        if (lane == 0) yp[i] = yi;
        for (int q = lane; q < i; q += 64) dl[q] = fma(-R[(long long)i * k + q], yi, dl[q]);
        __syncthreads();
    }
}

hipError_t launch_prefix_y(const double* R, const double* d, int k, int kp, int recip, double* yp, hipStream_t st)
{
    if (kp < 1 || kp > k || k > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(prefix_y_kernel, dim3(1), dim3(64), 0, st, R, d, k, kp, recip, yp);
    return hipGetLastError();
}

// out = ||b - y||_2 over m entries of the operator's type, accumulated in
// FP64: each thread sums a fixed stride of entries, then a fixed tree over
// the workgroup (one workgroup, so the order never changes).
template <typename T>
__global__ __launch_bounds__(1024) void resid_norm_kernel(const T* b, const T* y, long long m, double* out)
{
    __shared__ double red[1024];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < m; i += 1024) {
        const double d = (double)b[i] - (double)y[i];
        acc = fma(d, d, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sqrt(red[0]);
}

hipError_t launch_resid_norm(int dtype, const void* b, const void* y, long long m, double* out, hipStream_t st)
{
    if (dtype == 0) hipLaunchKernelGGL(resid_norm_kernel<double>, dim3(1), dim3(1024), 0, st, (const double*)b,
                                       (const double*)y, m, out);
    else hipLaunchKernelGGL(resid_norm_kernel<float>, dim3(1), dim3(1024), 0, st, (const float*)b,
                            (const float*)y, m, out);
    return hipGetLastError();
}

// dst[j * len + i] = scale[j] * src[j * ld + i] (normalised copy of a basis)
template <typename TB>
__global__ __launch_bounds__(256) void scale_basis_kernel(const TB* src, int64_t ld, const double* scale,
                                                          int64_t len, TB* dst)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= len) return;
    const double s = scale ? scale[j] : 1.0;
    dst[(int64_t)j * len + i] = (TB)(s * (double)src[(int64_t)j * ld + i]);
}

hipError_t launch_scale_basis(int tb, const void* src, int64_t ld, const double* scale, int64_t len,
                              int ncols, void* dst, hipStream_t st)
{
    const dim3 grid((unsigned)((len + 255) / 256), (unsigned)ncols);
    if (tb == 0)
        hipLaunchKernelGGL(scale_basis_kernel<double>, grid, dim3(256), 0, st, (const double*)src, ld, scale, len, (double*)dst);
    else if (tb == 1)
        hipLaunchKernelGGL(scale_basis_kernel<float>, grid, dim3(256), 0, st, (const float*)src, ld, scale, len, (float*)dst);
    else if (tb == 2)
        hipLaunchKernelGGL(scale_basis_kernel<__bf16>, grid, dim3(256), 0, st, (const __bf16*)src, ld, scale, len, (__bf16*)dst);
    else
        hipLaunchKernelGGL(scale_basis_kernel<_Float16>, grid, dim3(256), 0, st, (const _Float16*)src, ld, scale, len, (_Float16*)dst);
    return hipGetLastError();
}

hipError_t launch_apply(int dtype, int op, int ept, const ApplyArgs& a, hipStream_t st)
{
    (void)ept;
    const dim3 grid(a.sp.ntile), block(NT);
    const unsigned lds = (unsigned)a.lds_total;
    if (dtype == 0) {
        if (op == OP_BLUR) hipLaunchKernelGGL((apply_kernel<double, OP_BLUR>), grid, block, lds, st, a);
        else hipLaunchKernelGGL((apply_kernel<double, OP_CSR>), grid, block, lds, st, a);
    } else {
        if (op == OP_BLUR) hipLaunchKernelGGL((apply_kernel<float, OP_BLUR>), grid, block, lds, st, a);
        else hipLaunchKernelGGL((apply_kernel<float, OP_CSR>), grid, block, lds, st, a);
    }
    return hipGetLastError();
}

}  // namespace hk
