/*
 * hk.h - C ABI of the MI355X (gfx950) library for the sketched
 * inner-product-free Krylov methods sCMRH and sLSLU of
 *   M. Sabate Landman, A. N. Brown, J. Chung, J. G. Nagy,
 *   "Randomized and Inner-product Free Krylov Methods for Large-scale
 *    Inverse Problems".
 *
 * The library solves the linear inverse problem b = A x_true + e (Sec. 1,
 * eq. (ip)) with A reached only through products with A (and A^T).  A solve
 * runs k steps of the Hessenberg process with partial pivoting (square A,
 * eq. (Hessenberg_s); "sCMRH") or of the generalized Hessenberg process
 * (rectangular A, eq. (Hessenberg_r); "sLSLU", Algorithm 1), sketches each
 * new column A l_j with a random embedding S2 (Sec. 2), and returns
 *   x_k = L_k y,  y = argmin ||S2 (b - A L_k y)||^2 + lambda^2 ||S1 L_k y||^2
 * (Sec. 3.2, eq. (sketched_LSLU); Sec. 3.3, eq. (sketched_LSLU_hybrid) and
 * Algorithm 2), with x0 = 0.
 *
 * Conventions
 *  - Every call returns an hk_status.  0 = HK_OK; HK_BREAKDOWN (1) is
 *    informational: the Krylov subspace became invariant after k_done < k
 *    steps (a zero pivot) and the solution was computed from the k_done
 *    columns built; negative values are errors.  hk_last_error() returns a
 *    thread-local message describing the last error.
 *  - "device" pointers are HIP device allocations of the context's device
 *    (e.g. torch tensors on that GPU); "host" pointers are ordinary memory.
 *  - The library copies every operator input it is given (taps, CSR arrays)
 *    and never frees or retains caller memory.  Handles are opaque and are
 *    destroyed exactly once by the caller, dependents first: a solve (and a
 *    server with requests of the operator) before its operator, operators
 *    and servers before their context.
 *  - All device work of a context is ordered on the context's HIP stream;
 *    hk_solve_run is asynchronous.  Getters wait for the solve to finish.
 *  - Indices (pivots) are 0-based row indices of the original problem.
 *  - b and x are stored in the operator's storage type (hk_dtype), the
 *    Krylov bases in hk_params.basis_dtype.  All arithmetic is done in FP64;
 *    FP32 storage halves the bytes streamed.
 */
#ifndef HK_H
#define HK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HK_ABI_VERSION 2

typedef int32_t hk_status;
enum {
    HK_OK = 0,
    HK_BREAKDOWN = 1,      /* zero pivot: k_done < k columns were built */
    HK_EINVAL = -1,        /* invalid argument */
    HK_ENOMEM = -2,        /* device or host allocation failed */
    HK_EDEVICE = -3,       /* HIP runtime error or device-side abort */
    HK_ENUMERIC = -4,      /* NaN/Inf in the data, or a rank-deficient sketched problem */
    HK_EUNSUPPORTED = -5   /* valid request outside what this library implements */
};

typedef int32_t hk_dtype;
enum {
    HK_F64 = 0,
    HK_F32 = 1,
    HK_BF16 = 2,   /* bfloat16 (8 significant bits); basis storage only */
    HK_F16 = 3     /* IEEE binary16 (11 significant bits); basis storage only */
};

typedef int32_t hk_bc;     /* boundary condition of the blur */
enum { HK_BC_ZERO = 0, HK_BC_REFLECT = 1 };

typedef int32_t hk_sketch;
enum {
    HK_SKETCH_GAUSSIAN = 0,
    HK_SKETCH_SPARSE_SIGN = 1,
    /* no sketch: the unsketched methods CMRH (square) and LSLU (rectangular)
     * of Sec. 3.1, eq. (Hessenber_LS), with Tikhonov eq. (TP); the small
     * problem is eq. (TSP): min ||beta e_1 - H_{k+1,k} y||^2 + lambda^2 ||y||^2
     * with beta = b(t_1).  s and zeta are ignored (s is taken as k + 1). */
    HK_SKETCH_NONE = 3
};

typedef int32_t hk_method;
enum { HK_METHOD_AUTO = 0, HK_METHOD_HESSENBERG = 1, HK_METHOD_CHANGING_HESSENBERG = 2 };

enum { HK_FLAG_TRACE = 1 };

/* Opaque handles.  The caller destroys each one exactly once.  Every entry
 * point refuses, with HK_EINVAL and before reading the handle's memory, a
 * null handle, one this library did not create, or one already destroyed
 * (a destroyed handle whose address a newer handle reuses is that newer
 * handle).  Operators and solves hold their context, and solves their
 * operator: destroy solves before their operator, operators before their
 * context. */
typedef struct hk_context hk_context;
typedef struct hk_op hk_op;
typedef struct hk_solve hk_solve;
typedef struct hk_server hk_server;

/* ABI version (HK_ABI_VERSION) and the thread-local last error message.
 * Logging: the environment variable HK_LOG, read once per process, selects
 * 0 (unset: silent), 1 (every refused call and failure is also written to
 * stderr as "hk: status <code>: <message>") or 2 (as 1, plus one line per
 * solve plan: kernel, workgroups, tiles, LDS and workspace bytes, and one
 * per server admission). */
int32_t hk_abi_version(void);
const char* hk_last_error(void);

/* Create a context on HIP device `device`, ordering work on `stream`
 * (a hipStream_t, or NULL for the default stream).  The stream is borrowed:
 * the caller keeps it alive for the context's lifetime. */
hk_status hk_context_create(int32_t device, void* stream, hk_context** out);
hk_status hk_context_destroy(hk_context* ctx);

/* Blur operator on an ny x nx image stored row-major (index y*nx + x), the
 * blur model of the deblurring experiment (Sec. 4.1):
 *   (A u)(y, x) = sum_{a,b=-r..r} taps_y[a+r] taps_x[b+r] u(y+a, x+b),
 * a 2-D correlation with the separable PSF taps_y (x) taps_x.  Pixels outside
 * the image are 0 (HK_BC_ZERO) or the half-sample mirror image
 * u(-1) = u(0), u(N) = u(N-1) (HK_BC_REFLECT).  taps_y / taps_x: host arrays
 * of 2r+1 doubles, copied.  dt: storage type of vectors used with the op.
 * Square (m = n = ny*nx); only the forward product is provided, so blur
 * operators take the square (Hessenberg) method. */
hk_status hk_op_create_blur(hk_context* ctx, int64_t ny, int64_t nx, const double* taps_y,
                            const double* taps_x, int32_t radius, hk_bc bc, hk_dtype dt,
                            hk_op** out);

/* Convenience: Gaussian PSF, taps g(a) ~ exp(-a^2 / (2 sigma^2)) normalised to
 * sum 1 in each direction. */
hk_status hk_op_create_gaussian_blur(hk_context* ctx, int64_t ny, int64_t nx, double sigma,
                                     int32_t radius, hk_bc bc, hk_dtype dt, hk_op** out);

/* Blur with a general PSF (the motion blur of the deblurring experiment,
 * Sec. 4.1): (A u)(y, x) = sum_{a,b=-r..r} psf[(a+r)(2r+1) + (b+r)] u(y+a, x+b),
 * a 2-D correlation, with the boundary conditions of hk_op_create_blur.
 * psf: host array of (2r+1)^2 doubles, row-major over a (rows), copied.  A
 * PSF of rank one (equal to an outer product ty (x) tx to within 4 ulp of its
 * largest entry) is stored as its two factors and takes the separable path;
 * any other is stored as the list of its nonzero entries, at most
 * HK_PSF_MAX_TAPS of them (more: HK_EUNSUPPORTED).  Non-finite entries:
 * HK_ENUMERIC. */
#define HK_PSF_MAX_TAPS 2048
hk_status hk_op_create_blur_psf(hk_context* ctx, int64_t ny, int64_t nx, const double* psf, int32_t radius,
                                hk_bc bc, hk_dtype dt, hk_op** out);

/* Sparse operator A (m x n) in CSR form: host arrays rowptr[m+1] (int64,
 * rowptr[0] = 0, nondecreasing, rowptr[m] = nnz), col[nnz] (int32, in
 * [0, n)), val[nnz] of type dt.  All copied.  The library also builds A^T
 * so that both products (Algorithm 1) are available. */
hk_status hk_op_create_csr(hk_context* ctx, int64_t m, int64_t n, int64_t nnz,
                           const int64_t* rowptr, const int32_t* col, const void* val,
                           hk_dtype dt, hk_op** out);

hk_status hk_op_shape(const hk_op* op, int64_t* m, int64_t* n);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1, CSR only): device
 * vectors of the operator's dtype, lengths n -> m (or m -> n).  FP64
 * accumulation.  Stream-ordered, asynchronous. */
hk_status hk_op_apply(hk_op* op, int32_t transpose, const void* x_dev, void* y_dev);
hk_status hk_op_destroy(hk_op* op);

/* Solve parameters.
 *   k       number of Hessenberg steps (basis size), 1 <= k <= min(m, n), k <= 255
 *   s       sketch rows (the embedding dimension l of Sec. 2), s >= k + 1
 *   lambda  Tikhonov parameter >= 0; it enters squared (Sec. 3.3)
 *   sketch  Gaussian (entries N(0, 1/s), Sec. 2) or sparse sign (zeta nonzeros
 *           of value +-1/sqrt(zeta) per column, one in each of zeta row blocks)
 *   zeta    nonzeros per column of the sparse-sign embedding, 1 <= zeta <= s
 *   seed    64-bit key of the Philox4x32-10 generator that defines S1, S2
 *   method  AUTO: Hessenberg (sCMRH) for square operators, generalized
 *           (sLSLU) otherwise
 *   basis_dtype  storage type of the Krylov bases L (and D): HK_F64, or
 *           HK_F32 when the operator is FP32 as well (halves the basis bytes;
 *           all arithmetic stays FP64).  FP64 bases with an FP32 operator
 *           are allowed.  A zero-initialised struct selects HK_F64.
 *           Reduced-precision tier: HK_BF16 or HK_F16 bases with an FP32
 *           blur operator (b and x stay FP32).  Each new basis vector is
 *           rounded once to the 16-bit type when stored; the operator
 *           product, the elimination, the sketches and the small least
 *           squares read the stored values and compute in FP64, so
 *           z_j = S2 A l_j and f_j = S1 l_j are exact for the stored l_j and
 *           c = S2 b uses the FP32 b.  The pivot is the argmax of the values
 *           before rounding; the pivot entry is the rounded value.  HK_F16
 *           needs |b| and the pivot magnitudes |H(j+1, j)| inside FP16's
 *           range (about 6e-5 to 65504); a value that overflows makes the
 *           solve fail with HK_ENUMERIC.
 *   flags   0, or HK_FLAG_TRACE: workgroup 0 of the basis kernel records a
 *           wall-clock timestamp before and after every grid barrier
 *           (read them with hk_solve_get_trace)
 *   pivot_sample  0: partial pivoting on the whole vector (the argmax of
 *           |v|); 1..64: sampled pivoting (Sec. 3.2; the experiments use
 *           5 for sCMRH and 25 for sLSLU): the pivot is the largest |v| in
 *           a sample of that many non-pivot rows, drawn from Philox4x32-10
 *           with counter (c, i, 3, space) and the solve's seed; word w of
 *           call c (c < ceil(m/4) + 2) is candidate 4c + w, the row
 *           floor(w * len / 2^32); earlier pivots are skipped, the first m
 *           others are the sample (repeats allowed), ties go to the smaller
 *           row.  i is the pivot's position in its list and space is 0 for
 *           t, 1 for g.  An empty or all-zero sample falls back to the whole
 *           vector.  Basis entries may then exceed 1 in magnitude.
 *   max_workgroups  0: the basis kernel takes one workgroup per compute
 *           unit; > 0: at most that many (larger tiles), so that several
 *           solves fit on the device side by side; a problem that needs
 *           more tiles than allowed is refused with HK_EUNSUPPORTED.
 *   nrhs    right-hand sides solved together on the operator, 1..8 (0 means
 *           1).  Each has its own Krylov basis, pivots, H and small problem,
 *           computed exactly as its solve alone (same sketch S), so its
 *           results equal the single-right-hand-side solve's bit for bit;
 *           the right-hand sides share the basis kernel's grid barriers and
 *           argmax round trips, and with a Gaussian sketch the sketches of
 *           all their bases are one block contraction in which every entry
 *           of S is generated once per 64 columns.  The multi-right-hand-side
 *           basis is limited to blur operators with FP64 or FP32 bases and
 *           full partial pivoting, and to a k and a count whose per-right-
 *           hand-side state fits the kernel's LDS (HK_EUNSUPPORTED
 *           otherwise).  See hk_solve_run and hk_solve_select_rhs. */
typedef struct {
    int32_t k;
    int32_t s;
    double lambda;
    hk_sketch sketch;
    int32_t zeta;
    uint64_t seed;
    hk_method method;
    hk_dtype basis_dtype;
    uint32_t flags;
    int32_t pivot_sample;
    int32_t max_workgroups;
    int32_t nrhs;
} hk_params;

/* Device workspace a solve of `op` with `params` holds (bases, Hessenberg
 * matrices, sketches and partial sums), for admission control. */
hk_status hk_solve_workspace_bytes(const hk_op* op, const hk_params* params, size_t* bytes);

/* Create a solve: validates the parameters and allocates its workspace.
 * The solve can be run many times (each run overwrites its results). */
hk_status hk_solve_create(hk_op* op, const hk_params* params, hk_solve** out);

/* Create a solve on a workspace the caller owns (for callers that manage
 * device memory themselves: pools, arenas, one allocation shared by several
 * solves run one after another).  ws_dev: NULL, then this is hk_solve_create;
 * else a device pointer on the op's device, 256-byte aligned, to at least
 * ws_bytes >= hk_solve_workspace_bytes(op, params) bytes.  The caller keeps
 * it alive, and touches it with nothing else, until hk_solve_destroy; the
 * library never frees it.  It is cleared here by a kernel on the context
 * stream (nothing must start at particular values).  The library still
 * allocates the host handle and its timing events.  Errors: HK_EINVAL for a
 * misaligned pointer, HK_ENOMEM when ws_bytes is too small; the rest as
 * hk_solve_create. */
hk_status hk_solve_create_with_workspace(hk_op* op, const hk_params* params, void* ws_dev, size_t ws_bytes,
                                         hk_solve** out);

/* Run: enqueue the whole solve on the context stream and return at once.
 * b_dev: device array of the op's dtype, m x nrhs column-major (right-hand
 * side r at b_dev + r m; read during the run).  x_dev: n x nrhs likewise
 * (written during the run). */
hk_status hk_solve_run(hk_solve* sv, const void* b_dev, void* x_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * solve of `op` with `params`, enqueued on the context stream like
 * hk_solve_create + hk_solve_run, but with no allocation of any kind (no
 * hipMalloc, no event, no solve handle).  Its workspace is a static device
 * array of HK_NOALLOC_MAX_BYTES held by the library on each device until the
 * process ends (its address is taken when a context is created on the
 * device).  A problem whose workspace (hk_solve_workspace_bytes) exceeds it
 * is refused with HK_ENOMEM.  b_dev / x_dev as for hk_solve_run.  info_dev:
 * NULL, or a device array of two int32 that receives the run's status
 * (as hk_solve_wait) and the number of basis columns built, stream-ordered.
 * The array keeps the previous call's contents; each call clears what must
 * start at zero.  Calls that overlap on one device (other streams, other
 * threads) share the array and race: the caller orders them.  Asynchronous:
 * returns once the work is queued.  CSR operators: the row ranges balanced
 * by nonzeros are computed (and allocated) when a solve is created; this
 * call uses them only if a solve with the same grid was created on the
 * operator before, and equal row ranges otherwise, in which case x equals
 * the allocating path's to rounding rather than bit for bit. */
#define HK_NOALLOC_MAX_BYTES (128u << 20)
hk_status hk_solve_run_noalloc(hk_op* op, const hk_params* params, const void* b_dev, void* x_dev,
                               int32_t* info_dev);

/* Wait for the last run.  Returns HK_OK, HK_BREAKDOWN, or an error.  With
 * several right-hand sides: an error of any of them (the first), else
 * HK_BREAKDOWN if any broke down, else HK_OK. */
hk_status hk_solve_wait(hk_solve* sv);

/* Results of the last run (each call waits for it first).
 *   k_done      number of basis columns used (k, or fewer after breakdown)
 *   H           host, (k+1) x k FP64 column-major upper Hessenberg H_{k+1,k}
 *   W           host, k x k FP64 column-major upper triangular (sLSLU), or NULL
 *   t           host, k+1 int64 pivots of L (sCMRH) or of D (sLSLU); -1 unused
 *   g           host, k int64 pivots of L (sLSLU), or NULL
 *   res         host, k FP64: res[j] = minimised sketched objective
 *               (||S2(b - A L y)||^2 + lambda^2 ||S1 L y||^2)^(1/2) using the
 *               first j+1 columns; entries past k_done are 0.  Without a
 *               sketch: (||beta e_1 - H y||^2 + lambda^2 ||y||^2)^(1/2)
 *   Z, F, c     host: S2 A L_k (s x k), S1 L_k (s x k, zero if lambda = 0),
 *               S2 b (s), FP64 column-major.  Without a sketch (s = k + 1):
 *               H_{k+1,k}, [I; 0] (zero if lambda = 0) and beta e_1
 *   basis       which = 0: L (n x (k+1)), which = 1: D (m x (k+1), sLSLU),
 *               copied to a device buffer of basis_dtype, column-major;
 *               which = 2: the columns of L as stored.  The single-barrier
 *               blur kernel stores v_j = eta_j l_j unnormalised (eta_j =
 *               v_j(t_j), the pivot entry), so l_j = v_j / v_j(t_j); which = 0
 *               then returns l_j rounded to basis_dtype a second time.  For
 *               the other kernels which = 2 equals which = 0. */
hk_status hk_solve_info(hk_solve* sv, int32_t* k_done);

/* The right-hand side (0 .. nrhs-1) whose results hk_solve_info and the
 * getters report from now on (0 after creation); hk_solve_info then
 * returns that right-hand side's own status. */
hk_status hk_solve_select_rhs(hk_solve* sv, int32_t rhs);
hk_status hk_solve_get_hessenberg(hk_solve* sv, double* H, double* W);
hk_status hk_solve_get_pivots(hk_solve* sv, int64_t* t, int64_t* g);
hk_status hk_solve_get_residuals(hk_solve* sv, double* res);
hk_status hk_solve_get_sketches(hk_solve* sv, double* Z, double* F, double* c);
hk_status hk_solve_get_basis(hk_solve* sv, int32_t which, void* dst_dev);

/* The solution after the first kp basis vectors, 1 <= kp <= k_done, of the
 * selected right-hand side: x_kp = L_kp y_kp with y_kp the minimiser of the
 * small problem of eq. (sketched_LSLU) (eq. (sketched_LSLU_hybrid) when
 * lambda > 0) over the first kp columns.  The factors of the full small
 * problem already hold it (the leading kp x kp block of its triangular
 * factor and the first kp rotated right-hand-side entries), so no new
 * factorisation is done; its objective value is res[kp-1] above, and
 * kp = k_done gives the run's x bit for bit.  x_dev: device array of n
 * elements of the op's dtype.  Runs on the context stream and returns once
 * x_dev is written.  Errors: HK_EINVAL for kp outside [1, k_done]. */
hk_status hk_solve_get_prefix_solution(hk_solve* sv, int32_t kp, void* x_dev);

/* True residual norms of the selected right-hand side: res[kp-1] =
 * ||b - A x_kp||_2 for kp = 1 .. k_done (x_kp as hk_solve_get_prefix_solution;
 * the quantity the paper's sketched residual stands in for, Sec. 2),
 * entries past k_done are 0.  res: host array of k doubles.  Optional and
 * not free: one prefix solution, one product with A and one FP64 norm per
 * kp, on the context stream, in device buffers allocated for the call.
 * b is read from the array the last hk_solve_run was given, which must
 * still hold that right-hand side.  Errors: HK_EINVAL before any run. */
hk_status hk_solve_get_true_residuals(hk_solve* sv, double* res);

/* Workgroups of the solve's basis kernel (its grid; one per tile). */
hk_status hk_solve_grid(const hk_solve* sv, int32_t* workgroups);

/* Device-side duration of the last run's Hessenberg kernel and of the whole
 * run, in milliseconds (HIP events on the context stream). */
hk_status hk_solve_timing(hk_solve* sv, double* iterate_ms, double* total_ms);

/* The same for each of the most recent runs (up to 256 are kept, oldest
 * first): writes min(max_runs, runs kept) entries to iterate_ms / total_ms
 * (host arrays) and their number to *n.  Waits for the newest run. */
hk_status hk_solve_timing_history(hk_solve* sv, int32_t max_runs, double* iterate_ms,
                                  double* total_ms, int32_t* n);

/* Barrier timestamps of the last run (needs HK_FLAG_TRACE): ticks[2e] when
 * workgroup 0 reached grid barrier e, ticks[2e+1] when it was released.
 * Writes min(max, recorded) values, their count to *n and the tick length in
 * nanoseconds to *tick_ns. */
hk_status hk_solve_get_trace(hk_solve* sv, int32_t max, uint64_t* ticks, int32_t* n, double* tick_ns);

hk_status hk_solve_destroy(hk_solve* sv);

/* ---------------------------------------------------------------- serving
 * Continuous batching of solves on one device (a serving
 * loop).  Requests are queued on arrival and admitted in arrival order as
 * soon as a slot is free, the workspace they need fits in the device-memory
 * budget and the compute units their basis kernel takes are free; admitted
 * solves run on per-slot streams, side by side.  Finished requests free
 * their slot, units and workspace (kept in a pool for reuse) for the next
 * ones.  The server is driven by the caller's calls (submit, poll, wait);
 * it holds no thread of its own.
 *   slots        solves that may run at once, 1..16
 *   budget_bytes device bytes of workspace the server may allocate (0: 80%
 *                of the free device memory at creation)
 *   workgroups   compute units shared by the running basis kernels (0: all
 *                but 8, which stay free for the short kernels)
 * A request whose params->max_workgroups is 0 gets an equal share of the
 * units (workgroups / slots), or more if its problem needs more tiles.  The
 * caller keeps b_dev, x_dev and the operator alive until the request has
 * finished; its result is written to x_dev.  A request's solve is ordered
 * after the work queued on the context's stream when it was submitted (an
 * event recorded there at submission), so b_dev and x_dev may still be in
 * production on that stream; work queued there later is not waited for.
 * The slots' streams run side by side only as far as the HIP runtime gives
 * them hardware queues: GPU_MAX_HW_QUEUES (4 by default, read when the
 * process first uses HIP) should exceed the number of slots. */
hk_status hk_server_create(hk_context* ctx, int32_t slots, size_t budget_bytes, int32_t workgroups,
                           hk_server** out);
hk_status hk_server_destroy(hk_server* srv);   /* waits for the running solves */

/* Queue a request (returns at once with its ticket, 0, 1, 2, ...). */
hk_status hk_server_submit(hk_server* srv, hk_op* op, const hk_params* params, const void* b_dev, void* x_dev,
                           int64_t* ticket);

/* Retire finished solves and admit queued requests; *completed = requests
 * finished so far (may be NULL).  Does not block. */
hk_status hk_server_poll(hk_server* srv, int64_t* completed);

/* Poll until request `ticket` has finished; returns its status. */
hk_status hk_server_wait(hk_server* srv, int64_t ticket);

/* Result of a finished request: status (as hk_solve_wait), basis columns
 * built, workgroups of its basis kernel, and host steady-clock times in
 * seconds of its submission, admission and observed completion. */
hk_status hk_server_result(hk_server* srv, int64_t ticket, hk_status* status, int32_t* k_done,
                           int32_t* workgroups, double* t_submit, double* t_start, double* t_finish);

#ifdef __cplusplus
}
#endif
#endif /* HK_H */
