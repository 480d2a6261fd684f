// Drives the library's host runtime through the C ABI on one GPU, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host side only (the
// kernels are ordinary device code); tests/test_gpu_host_sanitize.py runs
// it.  Every host array handed to the library is allocated at exactly the
// size hk.h documents, so a write past one is reported.  Covered: contexts,
// blur (separable and general PSF) and CSR operators, solves with every
// getter, prefix solutions and true residuals, several right-hand sides,
// the caller-owned workspace (including its two errors), the allocation-
// free run, the serving loop, and the argument checks.  Prints one line per
// check; exits non-zero when one fails.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <utility>
#include <vector>

#include "hk.h"

static int failures = 0;

static void check(const char* what, bool ok)
{
    std::printf("%-44s %s\n", what, ok ? "ok" : "FAILED");
    if (!ok) {
        std::printf("  last error: %s\n", hk_last_error());
        ++failures;
    }
    std::fflush(stdout);
}

static bool hip_ok(hipError_t e) { return e == hipSuccess; }
static void dfree(void* p) { (void)hipFree(p); }

// deterministic values in [-1, 1)
static double lcg(uint64_t& st)
{
    st = st * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(st >> 11) / 4503599627370496.0 - 1.0;
}

template <typename T>
static T* to_device(const std::vector<T>& h)
{
    T* d = nullptr;
    if (!hip_ok(hipMalloc(&d, h.size() * sizeof(T)))) return nullptr;
    if (!hip_ok(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice))) return nullptr;
    return d;
}

static hk_params params(int k, int s, double lam, hk_sketch sk)
{
    hk_params p{};
    p.k = k;
    p.s = s;
    p.lambda = lam;
    p.sketch = sk;
    p.zeta = 4;
    p.seed = 0x1234abcdULL;
    p.method = HK_METHOD_AUTO;
    p.basis_dtype = HK_F64;
    return p;
}

// every getter of a finished solve, into host arrays of the documented sizes
static void read_all(hk_solve* sv, const hk_params& p, int64_t m, int64_t n, bool rect, const char* tag)
{
    char name[96];
    int32_t kd = -1;
    std::snprintf(name, sizeof name, "%s: info", tag);
    check(name, hk_solve_info(sv, &kd) >= 0 && kd >= 1 && kd <= p.k);
    const int k = p.k;
    const int s = p.sketch == HK_SKETCH_NONE ? k + 1 : p.s;
    std::vector<double> H((size_t)(k + 1) * k), W(rect ? (size_t)k * k : 0), res(k), Z((size_t)s * k),
        F((size_t)s * k), c(s);
    std::vector<int64_t> t(k + 1), g(rect ? k : 0);
    std::snprintf(name, sizeof name, "%s: hessenberg", tag);
    check(name, hk_solve_get_hessenberg(sv, H.data(), rect ? W.data() : nullptr) == HK_OK);
    std::snprintf(name, sizeof name, "%s: pivots", tag);
    check(name, hk_solve_get_pivots(sv, t.data(), rect ? g.data() : nullptr) == HK_OK);
    std::snprintf(name, sizeof name, "%s: residuals", tag);
    check(name, hk_solve_get_residuals(sv, res.data()) == HK_OK);
    std::snprintf(name, sizeof name, "%s: sketches", tag);
    check(name, hk_solve_get_sketches(sv, Z.data(), F.data(), c.data()) == HK_OK);
    void* xd = nullptr;
    void* Ld = nullptr;
    const size_t es = p.basis_dtype == HK_F32 ? 4 : 8;
    if (hip_ok(hipMalloc(&xd, (size_t)n * 8)) && hip_ok(hipMalloc(&Ld, (size_t)n * (k + 1) * es))) {
        std::snprintf(name, sizeof name, "%s: prefix solution kp = 1 and k_done", tag);
        check(name, hk_solve_get_prefix_solution(sv, 1, xd) == HK_OK && hk_solve_get_prefix_solution(sv, kd, xd) == HK_OK);
        std::snprintf(name, sizeof name, "%s: prefix solution kp = k_done + 1 refused", tag);
        check(name, hk_solve_get_prefix_solution(sv, kd + 1, xd) == HK_EINVAL);
        std::snprintf(name, sizeof name, "%s: basis L", tag);
        check(name, hk_solve_get_basis(sv, 0, Ld) == HK_OK);
    } else {
        check("device buffers", false);
    }
    dfree(xd);
    dfree(Ld);
    std::vector<double> tr(k);
    std::snprintf(name, sizeof name, "%s: true residuals", tag);
    check(name, hk_solve_get_true_residuals(sv, tr.data()) == HK_OK && std::isfinite(tr[0]));
    double it = 0, tot = 0;
    std::vector<double> ith(4), toth(4);
    int32_t nh = 0, G = 0;
    std::snprintf(name, sizeof name, "%s: timing, history, grid", tag);
    check(name, hk_solve_timing(sv, &it, &tot) == HK_OK && hk_solve_timing_history(sv, 4, ith.data(), toth.data(), &nh) == HK_OK &&
                    nh >= 1 && hk_solve_grid(sv, &G) == HK_OK && G >= 1);
    (void)m;
}

int main()
{
    uint64_t st = 99;
    hk_context* ctx = nullptr;
    check("context", hk_context_create(0, nullptr, &ctx) == HK_OK);
    if (!ctx) return 1;

    // ---- a 64 x 64 Gaussian blur, FP64
    const int64_t ny = 64, nx = 64, n = ny * nx;
    hk_op* blur = nullptr;
    check("gaussian blur operator", hk_op_create_gaussian_blur(ctx, ny, nx, 2.0, 6, HK_BC_REFLECT, HK_F64, &blur) == HK_OK);
    std::vector<double> bh(2 * n);
    for (auto& v : bh) v = lcg(st);
    double* bd = to_device(bh);
    double* xd = nullptr;
    check("device b, x", bd && hip_ok(hipMalloc(&xd, (size_t)2 * n * 8)));
    {
        hk_params p = params(12, 30, 1e-3, HK_SKETCH_GAUSSIAN);
        hk_solve* sv = nullptr;
        check("blur solve create", hk_solve_create(blur, &p, &sv) == HK_OK);
        check("blur solve run + wait", sv && hk_solve_run(sv, bd, xd) == HK_OK && hk_solve_wait(sv) >= 0);
        if (sv) read_all(sv, p, n, n, false, "blur");
        check("blur solve destroy", hk_solve_destroy(sv) == HK_OK);
    }
    {   // sparse sign, FP32 operator and bases, unsketched, sampled pivoting
        hk_op* b32 = nullptr;
        check("FP32 blur operator", hk_op_create_gaussian_blur(ctx, ny, nx, 1.5, 4, HK_BC_ZERO, HK_F32, &b32) == HK_OK);
        std::vector<float> bf(n);
        for (auto& v : bf) v = (float)lcg(st);
        float* bfd = to_device(bf);
        float* xfd = nullptr;
        check("device FP32 b, x", bfd && hip_ok(hipMalloc(&xfd, (size_t)n * 4)));
        hk_params p = params(10, 24, 1e-2, HK_SKETCH_SPARSE_SIGN);
        p.basis_dtype = HK_F32;
        hk_solve* sv = nullptr;
        check("FP32 sparse-sign solve", hk_solve_create(b32, &p, &sv) == HK_OK && hk_solve_run(sv, bfd, xfd) == HK_OK &&
                                            hk_solve_wait(sv) >= 0);
        if (sv) read_all(sv, p, n, n, false, "fp32");
        hk_solve_destroy(sv);
        hk_params q = params(8, 0, 0.0, HK_SKETCH_NONE);
        q.basis_dtype = HK_F32;
        q.pivot_sample = 5;
        sv = nullptr;
        check("unsketched sampled-pivot solve", hk_solve_create(b32, &q, &sv) == HK_OK && hk_solve_run(sv, bfd, xfd) == HK_OK &&
                                                    hk_solve_wait(sv) >= 0);
        if (sv) read_all(sv, q, n, n, false, "unsketched");
        hk_solve_destroy(sv);
        dfree(bfd);
        dfree(xfd);
        check("FP32 operator destroy", hk_op_destroy(b32) == HK_OK);
    }
    {   // general PSF
        const int r = 2;
        std::vector<double> psf((2 * r + 1) * (2 * r + 1));
        for (size_t i = 0; i < psf.size(); ++i) psf[i] = 0.02 + 0.01 * (double)(i % 5) + (i == 12 ? 0.6 : 0.0);
        hk_op* g = nullptr;
        check("general PSF operator", hk_op_create_blur_psf(ctx, ny, nx, psf.data(), r, HK_BC_ZERO, HK_F64, &g) == HK_OK);
        hk_params p = params(10, 22, 0.0, HK_SKETCH_GAUSSIAN);
        hk_solve* sv = nullptr;
        check("general PSF solve", hk_solve_create(g, &p, &sv) == HK_OK && hk_solve_run(sv, bd, xd) == HK_OK &&
                                       hk_solve_wait(sv) >= 0);
        hk_solve_destroy(sv);
        psf[3] = NAN;
        hk_op* bad = nullptr;
        check("non-finite PSF refused", hk_op_create_blur_psf(ctx, ny, nx, psf.data(), r, HK_BC_ZERO, HK_F64, &bad) == HK_ENUMERIC);
        hk_op_destroy(g);
    }
    {   // several right-hand sides
        hk_params p = params(10, 24, 1e-2, HK_SKETCH_GAUSSIAN);
        p.nrhs = 2;
        hk_solve* sv = nullptr;
        check("two right-hand sides", hk_solve_create(blur, &p, &sv) == HK_OK && hk_solve_run(sv, bd, xd) == HK_OK &&
                                          hk_solve_wait(sv) >= 0);
        check("select right-hand side 1", sv && hk_solve_select_rhs(sv, 1) == HK_OK);
        if (sv) read_all(sv, p, n, n, false, "rhs 1");
        check("select right-hand side 2 refused", sv && hk_solve_select_rhs(sv, 2) == HK_EINVAL);
        hk_solve_destroy(sv);
    }
    {   // caller-owned workspace
        hk_params p = params(12, 30, 0.0, HK_SKETCH_GAUSSIAN);
        size_t bytes = 0;
        check("workspace bytes", hk_solve_workspace_bytes(blur, &p, &bytes) == HK_OK && bytes > 0);
        char* ws = nullptr;
        check("workspace alloc", hip_ok(hipMalloc(&ws, bytes + 256)));
        hk_solve* sv = nullptr;
        check("misaligned workspace refused", hk_solve_create_with_workspace(blur, &p, ws + 8, bytes, &sv) == HK_EINVAL);
        check("small workspace refused", hk_solve_create_with_workspace(blur, &p, ws, bytes / 2, &sv) == HK_ENOMEM);
        check("workspace solve", hk_solve_create_with_workspace(blur, &p, ws, bytes, &sv) == HK_OK &&
                                     hk_solve_run(sv, bd, xd) == HK_OK && hk_solve_wait(sv) >= 0);
        hk_solve_destroy(sv);
        dfree(ws);
    }
    {   // allocation-free run
        hk_params p = params(8, 20, 0.0, HK_SKETCH_SPARSE_SIGN);
        int32_t* info = nullptr;
        check("noalloc run", hip_ok(hipMalloc(&info, 8)) && hk_solve_run_noalloc(blur, &p, bd, xd, info) == HK_OK &&
                                 hip_ok(hipDeviceSynchronize()));
        std::vector<int32_t> ih(2);
        check("noalloc info", hip_ok(hipMemcpy(ih.data(), info, 8, hipMemcpyDeviceToHost)) && ih[0] >= 0 && ih[1] == 8);
        dfree(info);
    }

    // ---- a 300 x 250 CSR matrix, FP32 (the rectangular method)
    const int64_t m = 300, nc = 250;
    std::vector<int64_t> rp(m + 1, 0);
    std::vector<int32_t> col;
    std::vector<float> val;
    for (int64_t i = 0; i < m; ++i) {
        const int cnt = 1 + (int)(i % 9);
        for (int q = 0; q < cnt; ++q) {
            col.push_back((int32_t)((i * 11 + q * 29) % nc));
            val.push_back((float)(lcg(st) + (q == 0 ? 2.0 : 0.0)));
        }
        rp[i + 1] = (int64_t)col.size();
    }
    // columns sorted within each row
    for (int64_t i = 0; i < m; ++i) {
        std::vector<std::pair<int32_t, float>> e;
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) e.emplace_back(col[q], val[q]);
        std::sort(e.begin(), e.end());
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) { col[q] = e[q - rp[i]].first; val[q] = e[q - rp[i]].second; }
    }
    hk_op* csr = nullptr;
    check("CSR operator", hk_op_create_csr(ctx, m, nc, (int64_t)col.size(), rp.data(), col.data(), val.data(), HK_F32, &csr) == HK_OK);
    std::vector<float> bc(m);
    for (auto& v : bc) v = (float)lcg(st);
    float* bcd = to_device(bc);
    float* xcd = nullptr;
    float* ycd = nullptr;
    check("device CSR b, x", bcd && hip_ok(hipMalloc(&xcd, (size_t)nc * 4)) && hip_ok(hipMalloc(&ycd, (size_t)m * 4)));
    check("CSR products", hk_op_apply(csr, 1, bcd, xcd) == HK_OK && hk_op_apply(csr, 0, xcd, ycd) == HK_OK &&
                              hip_ok(hipDeviceSynchronize()));
    {
        int64_t mm = 0, nn = 0;
        check("CSR shape", hk_op_shape(csr, &mm, &nn) == HK_OK && mm == m && nn == nc);
        hk_params p = params(8, 18, 1e-3, HK_SKETCH_GAUSSIAN);
        hk_solve* sv = nullptr;
        check("CSR solve", hk_solve_create(csr, &p, &sv) == HK_OK && hk_solve_run(sv, bcd, xcd) == HK_OK &&
                               hk_solve_wait(sv) >= 0);
        if (sv) read_all(sv, p, m, nc, true, "csr");
        hk_solve_destroy(sv);
    }

    // ---- the serving loop: blur and CSR requests side by side
    {
        hk_server* srv = nullptr;
        check("server", hk_server_create(ctx, 3, 0, 0, &srv) == HK_OK);
        std::vector<int64_t> tickets;
        hk_params pb = params(10, 22, 0.0, HK_SKETCH_SPARSE_SIGN);
        hk_params pc = params(6, 14, 0.0, HK_SKETCH_GAUSSIAN);
        std::vector<double*> xs;
        std::vector<float*> xcs;
        bool ok = srv != nullptr;
        for (int r = 0; r < 6 && ok; ++r) {
            int64_t tk = -1;
            if (r % 2 == 0) {
                double* x = nullptr;
                ok = hip_ok(hipMalloc(&x, (size_t)n * 8)) && hk_server_submit(srv, blur, &pb, bd, x, &tk) == HK_OK;
                xs.push_back(x);
            } else {
                float* x = nullptr;
                ok = hip_ok(hipMalloc(&x, (size_t)nc * 4)) && hk_server_submit(srv, csr, &pc, bcd, x, &tk) == HK_OK;
                xcs.push_back(x);
            }
            tickets.push_back(tk);
        }
        check("server submits", ok);
        for (int64_t tk : tickets) ok = ok && hk_server_wait(srv, tk) >= 0;
        int64_t done = 0;
        check("server waits and poll", ok && hk_server_poll(srv, &done) == HK_OK && done == (int64_t)tickets.size());
        hk_status rs;
        int32_t kd, wg;
        double t0, t1, t2;
        check("server result", ok && hk_server_result(srv, tickets[1], &rs, &kd, &wg, &t0, &t1, &t2) == HK_OK && rs >= 0 &&
                                   t0 <= t1 && t1 <= t2);
        check("server destroy", hk_server_destroy(srv) == HK_OK);
        for (auto* x : xs) dfree(x);
        for (auto* x : xcs) dfree(x);
    }

    // ---- argument checks
    {
        hk_solve* sv = nullptr;
        hk_params p = params(0, 30, 0.0, HK_SKETCH_GAUSSIAN);
        check("k = 0 refused", hk_solve_create(blur, &p, &sv) == HK_EINVAL);
        p = params(12, 12, 0.0, HK_SKETCH_GAUSSIAN);
        check("s < k + 1 refused", hk_solve_create(blur, &p, &sv) == HK_EINVAL);
        p = params(12, 30, -1.0, HK_SKETCH_GAUSSIAN);
        check("lambda < 0 refused", hk_solve_create(blur, &p, &sv) == HK_EINVAL);
        p = params(12, 30, 0.0, HK_SKETCH_SPARSE_SIGN);
        p.zeta = 31;
        check("zeta > s refused", hk_solve_create(blur, &p, &sv) == HK_EINVAL);
        p = params(256, 600, 0.0, HK_SKETCH_GAUSSIAN);
        check("k > 255 refused", hk_solve_create(blur, &p, &sv) == HK_EUNSUPPORTED);
        p = params(8, 18, 0.0, HK_SKETCH_GAUSSIAN);
        p.method = HK_METHOD_HESSENBERG;
        check("square method on a 300 x 250 matrix refused", hk_solve_create(csr, &p, &sv) == HK_EINVAL);
        check("A^T of a blur refused", hk_op_apply(blur, 1, xd, xd) == HK_EUNSUPPORTED);
        std::vector<int64_t> brp = {0, 2, 1};
        std::vector<int32_t> bcol = {0};
        std::vector<float> bval = {1.0f};
        hk_op* bop = nullptr;
        check("decreasing row pointers refused",
              hk_op_create_csr(ctx, 2, 2, 1, brp.data(), bcol.data(), bval.data(), HK_F32, &bop) == HK_EINVAL);
        std::vector<int64_t> grp = {0, 1, 1};
        std::vector<int32_t> gcol = {5};
        check("column index out of range refused",
              hk_op_create_csr(ctx, 2, 2, 1, grp.data(), gcol.data(), bval.data(), HK_F32, &bop) == HK_EINVAL);
        check("null solve refused", hk_solve_wait(nullptr) == HK_EINVAL);
    }

    // ---- lifecycle: each handle is destroyed once; a second destroy or a use
    // after destroy is refused without touching the freed handle
    {
        hk_params p = params(8, 20, 0.0, HK_SKETCH_GAUSSIAN);
        hk_solve* sv = nullptr;
        check("solve for the lifecycle checks", hk_solve_create(blur, &p, &sv) == HK_OK);
        check("solve destroy", hk_solve_destroy(sv) == HK_OK);
        check("second solve destroy refused", hk_solve_destroy(sv) == HK_EINVAL);
        check("wait on a destroyed solve refused", hk_solve_wait(sv) == HK_EINVAL);
        int32_t kd = 0;
        check("info of a destroyed solve refused", hk_solve_info(sv, &kd) == HK_EINVAL);
        hk_server* srv = nullptr;
        check("server for the lifecycle checks", hk_server_create(ctx, 2, 0, 0, &srv) == HK_OK);
        check("server destroy", hk_server_destroy(srv) == HK_OK);
        check("second server destroy refused", hk_server_destroy(srv) == HK_EINVAL);
        int64_t done = 0;
        check("poll of a destroyed server refused", hk_server_poll(srv, &done) == HK_EINVAL);
    }

    dfree(bd);
    dfree(xd);
    dfree(bcd);
    dfree(xcd);
    dfree(ycd);
    check("operators destroy", hk_op_destroy(blur) == HK_OK && hk_op_destroy(csr) == HK_OK);
    check("second operator destroy refused", hk_op_destroy(blur) == HK_EINVAL);
    check("solve on a destroyed operator refused", [&] {
        hk_params p = params(8, 20, 0.0, HK_SKETCH_GAUSSIAN);
        hk_solve* sv = nullptr;
        return hk_solve_create(blur, &p, &sv) == HK_EINVAL;
    }());
    check("context destroy", hk_context_destroy(ctx) == HK_OK);
    check("second context destroy refused", hk_context_destroy(ctx) == HK_EINVAL);
    std::printf("failures %d\n", failures);
    std::fflush(stdout);
    // Leave without running static destructors: the HIP runtime's own
    // teardown frees memory after the sanitizer runtime's device-memory hooks
    // are gone, which the sanitizer reports as an internal check failure.
    // Nothing of this library runs past this point.
    std::_Exit(failures ? 1 : 0);
}
