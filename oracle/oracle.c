/*
 * CPU oracle for the sketched inner-product-free Krylov methods sCMRH and
 * sLSLU (Sabate Landman, Brown, Chung, Nagy, "Randomized and inner-product
 * free Krylov methods for large-scale inverse problems").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 reference the
 * GPU library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the GPU library neither links
 * nor calls it, and it shares no code with that library.
 *
 * Everything is written in the order the paper states it:
 *   - Sec. 2: Gaussian embedding (entries N(0, 1/l)) and the sparse-sign
 *     embedding (named there, defined here as described below);
 *     sketch-and-solve least squares, eq. (sketched_LS).
 *   - Sec. 3.1: the Hessenberg process with partial pivoting for square A,
 *     eq. (Hessenberg_s), and the generalized Hessenberg process for
 *     rectangular A, eq. (Hessenberg_r).
 *   - Sec. 3.2, Algorithm 1 (sLSLU) and its square specialisation (sCMRH);
 *     Sec. 3.3, Algorithm 2 (Tikhonov), objective (sketched_LSLU_hybrid).
 *
 * Readings taken where the printed algorithms are garbled (each is listed
 * in the design notes): the forward step applies A to l_k (not A^T to d_k);
 * the new basis vectors are d_{k+1} and l_{k+1}; W(k+1,k+1) is read from q;
 * f_j is the S1-sketch of the normalised l_j; both objective terms are
 * squared and lambda enters squared; pivot ties go to the smallest row index;
 * a zero pivot (breakdown) stops the iteration and the small problem is
 * solved with the columns built so far; x0 = 0.
 *
 * Compiled with -ffp-contract=off so every a - h*b is a rounded product
 * followed by a rounded difference, exactly as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_BREAKDOWN 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENUMERIC (-4)

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, from its published definition     */
/* (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2,  */
/* 3", SC'11): ten rounds of two 32x32->64 multiplications on a four-word   */
/* counter, with a two-word key advanced by the Weyl constants per round.   */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from the top 23 bits of a word: (2*(w>>9)+1) * 2^-24. */
double orc_uniform(uint32_t w)
{
    return (double)(2u * (w >> 9) + 1u) * (1.0 / 16777216.0);
}

/* Entry (r, i) of the Gaussian embedding S in R^{s x m}: N(0, 1/s) (Sec. 2).
 * Row group c = r/4 and column i select one Philox block (counter
 * (i, c, stream, 0), key (seed lo, seed hi)); Box-Muller turns its four
 * uniforms into the four standard normals of rows 4c..4c+3. */
double orc_gaussian_entry(uint64_t seed, uint32_t stream, int64_t s, int64_t r, int64_t i)
{
    uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(r / 4), stream, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    int q = (int)(r % 4);
    double ua = orc_uniform(w[q < 2 ? 0 : 2]);
    double ub = orc_uniform(w[q < 2 ? 1 : 3]);
    double rad = sqrt(-2.0 * log(ua));
    double g = (q % 2 == 0) ? rad * cos(2.0 * M_PI * ub) : rad * sin(2.0 * M_PI * ub);
    return g / sqrt((double)s);
}

/* Column i of the sparse-sign embedding S in R^{s x m}: zeta nonzeros of
 * value +-1/sqrt(zeta), one in each of the zeta row blocks
 * [floor(b s/zeta), floor((b+1) s/zeta)).  Block b reads word (b mod 4) of
 * Philox block (i, b/4, stream, 1): row offset floor((w>>1) |B_b| / 2^31),
 * sign negative iff the lowest bit is set. */
void orc_sparse_sign_column(uint64_t seed, uint32_t stream, int64_t s, int zeta, int64_t i,
                            int64_t* rows, double* vals)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int b = 0; b < zeta; ++b) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(b / 4), stream, 1u};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        uint32_t word = w[b % 4];
        int64_t start = (int64_t)b * s / zeta;
        int64_t end = (int64_t)(b + 1) * s / zeta;
        int64_t size = end - start;
        int64_t off = (int64_t)(((uint64_t)(word >> 1) * (uint64_t)size) >> 31);
        rows[b] = start + off;
        vals[b] = ((word & 1u) ? -1.0 : 1.0) / sqrt((double)zeta);
    }
}

/* A sketch operator S in R^{s x m}, materialised: dense row-major for the
 * Gaussian embedding, zeta (row, value) pairs per column for sparse sign. */
typedef struct {
    int kind; /* 0 dense (Gaussian, identity), 1 sparse sign */
    int64_t s, m;
    int zeta;
    double* dense;   /* s*m, S[r*m + i] */
    int64_t* rows;   /* m*zeta */
    double* vals;    /* m*zeta */
} orc_sketch;

static void sketch_free(orc_sketch* S)
{
    free(S->dense); free(S->rows); free(S->vals);
    memset(S, 0, sizeof(*S));
}

static int sketch_make(orc_sketch* S, int kind, int64_t s, int64_t m, int zeta, uint64_t seed,
                       uint32_t stream)
{
    memset(S, 0, sizeof(*S));
    S->kind = kind; S->s = s; S->m = m; S->zeta = zeta;
    if (kind == 2) {
        /* identity embedding [I_m; 0] (test-only: with it the sketched
         * problem is the unsketched one, eq. (original_LS_proj)) */
        if (s < m) return ORC_EINVAL;
        S->dense = (double*)calloc((size_t)(s * m), sizeof(double));
        if (!S->dense) return ORC_ENOMEM;
        for (int64_t i = 0; i < m; ++i) S->dense[i * m + i] = 1.0;
        S->kind = 0;
    } else if (kind == 0) {
        S->dense = (double*)malloc(sizeof(double) * (size_t)(s * m));
        if (!S->dense) return ORC_ENOMEM;
        for (int64_t r = 0; r < s; ++r)
            for (int64_t i = 0; i < m; ++i)
                S->dense[r * m + i] = orc_gaussian_entry(seed, stream, s, r, i);
    } else {
        S->rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m * zeta));
        S->vals = (double*)malloc(sizeof(double) * (size_t)(m * zeta));
        if (!S->rows || !S->vals) { sketch_free(S); return ORC_ENOMEM; }
        for (int64_t i = 0; i < m; ++i)
            orc_sparse_sign_column(seed, stream, s, zeta, i, S->rows + i * zeta, S->vals + i * zeta);
    }
    return ORC_OK;
}

/* z = S a: the definition of a matrix-vector product. */
static void sketch_apply(const orc_sketch* S, const double* a, double* z)
{
    for (int64_t r = 0; r < S->s; ++r) z[r] = 0.0;
    if (S->kind == 0) {
        for (int64_t r = 0; r < S->s; ++r) {
            double acc = 0.0;
            for (int64_t i = 0; i < S->m; ++i) acc += S->dense[r * S->m + i] * a[i];
            z[r] = acc;
        }
    } else {
        for (int64_t i = 0; i < S->m; ++i)
            for (int b = 0; b < S->zeta; ++b)
                z[S->rows[i * S->zeta + b]] += S->vals[i * S->zeta + b] * a[i];
    }
}

/* Materialise S (test helper): Gaussian row-major s*m; sparse sign as dense too. */
int orc_sketch_dense(int kind, int64_t s, int64_t m, int zeta, uint64_t seed, uint32_t stream,
                     double* out)
{
    orc_sketch S;
    int st = sketch_make(&S, kind, s, m, zeta, seed, stream);
    if (st) return st;
    if (S.kind == 0) {
        memcpy(out, S.dense, sizeof(double) * (size_t)(s * m));
    } else {
        memset(out, 0, sizeof(double) * (size_t)(s * m));
        for (int64_t i = 0; i < m; ++i)
            for (int b = 0; b < zeta; ++b)
                out[S.rows[i * zeta + b] * m + i] += S.vals[i * zeta + b];
    }
    sketch_free(&S);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Operators: A and A^T reached only through products (Sec. 1, eq. (1)).    */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind;            /* 0: blur, 1: CSR matrix */
    int64_t m, n;
    /* blur: image ny x nx row-major, PSF p(a,b) = taps_y[a+r] * taps_x[b+r],
     * or psf[(a+r)(2r+1) + (b+r)] when psf is not NULL (a general PSF) */
    int64_t ny, nx;
    int32_t radius;
    int32_t bc;          /* 0 zero outside, 1 half-sample reflection */
    const double* taps_y;
    const double* taps_x;
    const double* psf;
    /* CSR */
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
} orc_op;

static int64_t bc_index(int64_t i, int64_t N, int bc)
{
    if (i >= 0 && i < N) return i;
    if (bc == 0) return -1;
    /* half-sample symmetric: x(-1) = x(0), x(N) = x(N-1) */
    if (i < 0) i = -i - 1;
    if (i >= N) i = 2 * N - i - 1;
    return (i >= 0 && i < N) ? i : -1;
}

/* 2-D correlation u(y,x) = sum_{a,b} p(a,b) in(y+a, x+b) with the boundary
 * condition applied to out-of-range pixels (the blur model of Sec. 4.1). */
double orc_blur_pixel(const orc_op* A, const double* in, int64_t y, int64_t x)
{
    const int r = A->radius;
    double acc = 0.0;
    for (int a = -r; a <= r; ++a) {
        int64_t yy = bc_index(y + a, A->ny, A->bc);
        if (yy < 0) continue;
        for (int b = -r; b <= r; ++b) {
            int64_t xx = bc_index(x + b, A->nx, A->bc);
            if (xx < 0) continue;
            double p = A->psf ? A->psf[(int64_t)(a + r) * (2 * r + 1) + (b + r)]
                              : A->taps_y[a + r] * A->taps_x[b + r];
            acc += p * in[yy * A->nx + xx];
        }
    }
    return acc;
}

void orc_op_apply(const orc_op* A, const double* in, double* out)
{
    if (A->kind == 0) {
        #pragma omp parallel for schedule(static)
        for (int64_t y = 0; y < A->ny; ++y)
            for (int64_t x = 0; x < A->nx; ++x)
                out[y * A->nx + x] = orc_blur_pixel(A, in, y, x);
    } else {
        #pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < A->m; ++r) {
            double acc = 0.0;
            for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; ++p) acc += A->val[p] * in[A->col[p]];
            out[r] = acc;
        }
    }
}

/* out = A^T in, by scattering each row (CSR only). */
void orc_op_apply_t(const orc_op* A, const double* in, double* out)
{
    for (int64_t c = 0; c < A->n; ++c) out[c] = 0.0;
    for (int64_t r = 0; r < A->m; ++r)
        for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; ++p) out[A->col[p]] += A->val[p] * in[r];
}

/* ------------------------------------------------------------------------ */
/* Small dense sketched least squares (Sec. 3.2, eq. (sketched_LSLU); with  */
/* Tikhonov, eq. (sketched_LSLU_hybrid) with both terms squared):           */
/*    min_y || c - Z y ||^2 + lam^2 || F y ||^2                             */
/* by Householder QR of the stacked matrix [Z; lam F] (rows x k, col-major).*/
/* res[j] = minimised objective (square-rooted) using the first j+1 columns.*/
/* ------------------------------------------------------------------------ */
int orc_small_ls(int64_t s, int64_t k, const double* Z, const double* F, double lam,
                 const double* c, double* y, double* res)
{
    const int64_t rows = (lam > 0.0) ? 2 * s : s;
    if (k < 1 || rows < k) return ORC_EINVAL;
    double* M = (double*)calloc((size_t)(rows * k), sizeof(double));
    double* g = (double*)calloc((size_t)rows, sizeof(double));
    double* v = (double*)calloc((size_t)rows, sizeof(double));
    if (!M || !g || !v) { free(M); free(g); free(v); return ORC_ENOMEM; }
    for (int64_t j = 0; j < k; ++j) {
        for (int64_t i = 0; i < s; ++i) M[j * rows + i] = Z[j * s + i];
        if (lam > 0.0)
            for (int64_t i = 0; i < s; ++i) M[j * rows + s + i] = lam * F[j * s + i];
    }
    for (int64_t i = 0; i < s; ++i) g[i] = c[i];
    int status = ORC_OK;
    for (int64_t j = 0; j < k; ++j) {
        /* reflector that maps M[j:, j] to (alpha, 0, ..., 0) */
        double nrm2 = 0.0;
        for (int64_t i = j; i < rows; ++i) nrm2 += M[j * rows + i] * M[j * rows + i];
        double nrm = sqrt(nrm2);
        if (nrm == 0.0) { status = ORC_ENUMERIC; break; }
        double x0 = M[j * rows + j];
        double alpha = (x0 >= 0.0) ? -nrm : nrm;
        for (int64_t i = j; i < rows; ++i) v[i] = M[j * rows + i];
        v[j] = x0 - alpha;
        double vnorm2 = 0.0;
        for (int64_t i = j; i < rows; ++i) vnorm2 += v[i] * v[i];
        /* apply H = I - 2 v v^T / (v^T v) to the remaining columns and to g */
        for (int64_t jj = j; jj < k; ++jj) {
            double dot = 0.0;
            for (int64_t i = j; i < rows; ++i) dot += v[i] * M[jj * rows + i];
            double f = 2.0 * dot / vnorm2;
            for (int64_t i = j; i < rows; ++i) M[jj * rows + i] -= f * v[i];
        }
        double dot = 0.0;
        for (int64_t i = j; i < rows; ++i) dot += v[i] * g[i];
        double f = 2.0 * dot / vnorm2;
        for (int64_t i = j; i < rows; ++i) g[i] -= f * v[i];
    }
    if (status == ORC_OK) {
        for (int64_t j = 0; j < k; ++j) {
            double t = 0.0;
            for (int64_t i = j + 1; i < rows; ++i) t += g[i] * g[i];
            res[j] = sqrt(t);
        }
        for (int64_t j = k - 1; j >= 0; --j) {
            double t = g[j];
            for (int64_t jj = j + 1; jj < k; ++jj) t -= M[jj * rows + j] * y[jj];
            y[j] = t / M[j * rows + j];
        }
    }
    free(M); free(g); free(v);
    return status;
}

/* ------------------------------------------------------------------------ */
/* The solvers.                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t k, s;
    double lam;
    int32_t sketch;      /* 0 Gaussian, 1 sparse sign, 2 identity [I; 0],
                            3 none: the unsketched projected problem */
    int32_t zeta;
    uint64_t seed;
    int32_t method;      /* 0 sCMRH (square Hessenberg), 1 sLSLU (generalized) */
    int32_t pivot_sample;/* 0: full partial pivoting; m_s > 0: sampled pivoting */
} orc_params;

typedef struct {
    double* x;       /* n */
    double* H;       /* (k+1) x k, column-major, zero-initialised by the caller */
    double* W;       /* k x k col-major (sLSLU) or NULL */
    int64_t* t;      /* k+1 pivots of L (sCMRH) or of D (sLSLU) */
    int64_t* g;      /* k pivots of L (sLSLU) or NULL */
    double* res;     /* k: minimised sketched objective per prefix */
    double* Lb;      /* optional n x (k+1) column-major basis L */
    double* Db;      /* optional m x (k+1) basis D (sLSLU) */
    double* Z;       /* optional s x k */
    double* F;       /* optional s x k */
    double* c;       /* optional s */
    int32_t k_done;
    int32_t n_t;     /* valid entries written to t */
    int32_t n_g;     /* valid entries written to g */
} orc_out;

/* argmax |v(r)| over rows not yet used as pivots; ties -> smallest r.
 * Returns -1 if every candidate is zero (breakdown). */
static int64_t pivot_search(const double* v, int64_t len, const unsigned char* used)
{
    int64_t best = -1;
    double bestabs = 0.0;
    for (int64_t r = 0; r < len; ++r) {
        if (used[r]) continue;
        double a = fabs(v[r]);
        if (a > bestabs) { bestabs = a; best = r; }
    }
    return best;
}

/* Sampled partial pivoting (Sec. 3.2: the pivot is the largest magnitude in
 * a small random sample of the vector's entries).  The paper does not fix
 * the sample; the reading taken here:
 *   - candidates come from Philox4x32-10 with counter (c, i, 3, space),
 *     c = 0 .. nc-1, nc = ceil(m_s / 4) + 2, key (seed lo, seed hi); word w
 *     of call c is candidate 4c + w, the row floor(w * len / 2^32);
 *   - i is the position of the pivot being chosen in its list (t or g) and
 *     space is 0 for t (rows of D, or of L for sCMRH) and 1 for g;
 *   - candidates that are earlier pivots are skipped; the first m_s others
 *     form the sample (repeats allowed);
 *   - the pivot is the sample's largest |v(r)|, ties to the smallest r;
 *     if the sample is empty or all zero, the full search decides, so a
 *     breakdown is declared only when every candidate row is zero. */
static int64_t pivot_search_sampled(const double* v, int64_t len, const unsigned char* used, int ms,
                                    uint64_t seed, uint32_t i, uint32_t space)
{
    if (ms <= 0) return pivot_search(v, len, used);
    const int nc = (ms + 3) / 4 + 2;
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    int taken = 0;
    int64_t best = -1;
    double bestabs = 0.0;
    for (int c = 0; c < nc && taken < ms; ++c) {
        const uint32_t ctr[4] = {(uint32_t)c, i, 3u, space};
        uint32_t w[4];
        orc_philox4x32_10(ctr, key, w);
        for (int q = 0; q < 4 && taken < ms; ++q) {
            const int64_t r = (int64_t)(((uint64_t)w[q] * (uint64_t)len) >> 32);
            if (used[r]) continue;
            ++taken;
            const double a = fabs(v[r]);
            if (a > bestabs || (a == bestabs && a > 0.0 && r < best)) { bestabs = a; best = r; }
        }
    }
    return best >= 0 ? best : pivot_search(v, len, used);
}

int orc_solve(const orc_op* A, const orc_params* P, const double* b, orc_out* out)
{
    const int ms = P->pivot_sample;
    const uint64_t sd = P->seed;
    const int k = P->k;
    const int none = (P->sketch == 3);
    /* without a sketch the small problem has the k+1 rows of H_{k+1,k} */
    const int64_t m = A->m, n = A->n, s = none ? k + 1 : P->s;
    const int rect = (P->method == 1);
    if (k < 1 || s < k + 1) return ORC_EINVAL;
    if (!rect && m != n) return ORC_EINVAL;
    if (rect && A->kind != 1) return ORC_EINVAL;
    if (k > (m < n ? m : n)) return ORC_EINVAL;

    orc_sketch S1, S2;
    memset(&S1, 0, sizeof S1);
    memset(&S2, 0, sizeof S2);
    int st = none ? ORC_OK : sketch_make(&S2, P->sketch, s, m, P->zeta, P->seed, 2u);
    if (st) return st;
    if (P->lam > 0.0 && !none) {
        st = sketch_make(&S1, P->sketch, s, n, P->zeta, P->seed, 1u);
        if (st) { sketch_free(&S2); return st; }
    }

    /* L: n x (k+1); D: m x (k+1) (sCMRH uses L only: D == L, t == g) */
    double* L = (double*)calloc((size_t)(n * (k + 1)), sizeof(double));
    double* D = rect ? (double*)calloc((size_t)(m * (k + 1)), sizeof(double)) : NULL;
    double* Z = (double*)calloc((size_t)(s * k), sizeof(double));
    double* F = (double*)calloc((size_t)(s * k), sizeof(double));
    double* c = (double*)calloc((size_t)s, sizeof(double));
    double* u = (double*)calloc((size_t)(m > n ? m : n), sizeof(double));
    double* q = (double*)calloc((size_t)n, sizeof(double));
    unsigned char* used_m = (unsigned char*)calloc((size_t)m, 1);
    unsigned char* used_n = (unsigned char*)calloc((size_t)n, 1);
    double* y = (double*)calloc((size_t)k, sizeof(double));
    int64_t* tp = (int64_t*)calloc((size_t)(k + 1), sizeof(int64_t));
    int64_t* gp = (int64_t*)calloc((size_t)(k + 1), sizeof(int64_t));
    if (!L || (rect && !D) || !Z || !F || !c || !u || !q || !used_m || !used_n || !y || !tp || !gp) {
        st = ORC_ENOMEM;
        goto done;
    }
    const int64_t kk1 = k + 1;
#define HH(i, j) out->H[(int64_t)(j) * kk1 + (i)]
#define WW(i, j) out->W[(int64_t)(j) * k + (i)]

    int k_done = 0, nt = 0, ng = 0;
    double beta0 = 0.0;                      /* b(t_1): D_{k+1}^+ b = beta e_1 */
    if (!none) sketch_apply(&S2, b, c);      /* S2 r0 with x0 = 0 */

    if (!rect) {
        /* ---- sCMRH: Hessenberg process with partial pivoting ---- */
        int64_t p = pivot_search_sampled(b, m, used_m, ms, sd, 0u, 0u);
        if (p < 0) goto small_ls;            /* b = 0: x = 0 */
        double beta = b[p];
        beta0 = beta;
        for (int64_t r = 0; r < n; ++r) L[r] = b[r] / beta;
        tp[0] = p; used_m[p] = 1; nt = 1;
        if (P->lam > 0.0 && !none) sketch_apply(&S1, L, F);
        for (int j = 0; j < k; ++j) {       /* iteration j+1 of the paper */
            const double* lj = L + (int64_t)j * n;
            orc_op_apply(A, lj, u);           /* u = A l_j */
            if (!none) sketch_apply(&S2, u, Z + (int64_t)j * s);   /* z_j = S2 u */
            for (int i = 0; i <= j; ++i) {    /* gathers + axpys, no inner products */
                double h = u[tp[i]];
                HH(i, j) = h;
                const double* li = L + (int64_t)i * n;
                for (int64_t r = 0; r < n; ++r) u[r] = u[r] - h * li[r];
            }
            k_done = j + 1;
            int64_t piv = (j + 1 < n) ? pivot_search_sampled(u, n, used_m, ms, sd, (uint32_t)(j + 1), 0u) : -1;
            if (piv < 0) { HH(j + 1, j) = 0.0; if (j + 1 < k) st = ORC_BREAKDOWN; break; }
            double hp = u[piv];
            HH(j + 1, j) = hp;
            double* lnext = L + (int64_t)(j + 1) * n;
            for (int64_t r = 0; r < n; ++r) lnext[r] = u[r] / hp;
            tp[j + 1] = piv; used_m[piv] = 1; nt = j + 2;
            if (P->lam > 0.0 && j + 1 < k && !none) sketch_apply(&S1, lnext, F + (int64_t)(j + 1) * s);
        }
    } else {
        /* ---- sLSLU: generalized Hessenberg process ---- */
        int64_t p = pivot_search_sampled(b, m, used_m, ms, sd, 0u, 0u);
        if (p < 0) goto small_ls;
        double beta = b[p];
        beta0 = beta;
        for (int64_t r = 0; r < m; ++r) D[r] = b[r] / beta;
        tp[0] = p; used_m[p] = 1; nt = 1;
        orc_op_apply_t(A, b, q);              /* v0 = A^T r0 */
        int64_t p2 = pivot_search_sampled(q, n, used_n, ms, sd, 0u, 1u);
        if (p2 < 0) goto small_ls;
        double alpha = q[p2];
        for (int64_t r = 0; r < n; ++r) L[r] = q[r] / alpha;
        gp[0] = p2; used_n[p2] = 1; ng = 1;
        orc_op_apply_t(A, D, q);              /* r = A^T d1; W(1,1) = r(g(1)) */
        if (out->W) WW(0, 0) = q[p2];
        if (P->lam > 0.0 && !none) sketch_apply(&S1, L, F);
        for (int j = 0; j < k; ++j) {
            const double* lj = L + (int64_t)j * n;
            orc_op_apply(A, lj, u);           /* u = A l_j */
            if (!none) sketch_apply(&S2, u, Z + (int64_t)j * s);
            for (int i = 0; i <= j; ++i) {
                double h = u[tp[i]];
                HH(i, j) = h;
                const double* di = D + (int64_t)i * m;
                for (int64_t r = 0; r < m; ++r) u[r] = u[r] - h * di[r];
            }
            k_done = j + 1;
            int64_t piv = (j + 1 < m) ? pivot_search_sampled(u, m, used_m, ms, sd, (uint32_t)(j + 1), 0u) : -1;
            if (piv < 0) { HH(j + 1, j) = 0.0; if (j + 1 < k) st = ORC_BREAKDOWN; break; }
            double hp = u[piv];
            HH(j + 1, j) = hp;
            double* dnext = D + (int64_t)(j + 1) * m;
            for (int64_t r = 0; r < m; ++r) dnext[r] = u[r] / hp;
            tp[j + 1] = piv; used_m[piv] = 1; nt = j + 2;
            if (j + 1 == k) break;            /* l_{k+1} is not needed for x_k */
            orc_op_apply_t(A, dnext, q);      /* q = A^T d_{j+1} */
            for (int i = 0; i <= j; ++i) {
                double w = q[gp[i]];
                if (out->W) WW(i, j + 1) = w;
                const double* li = L + (int64_t)i * n;
                for (int64_t r = 0; r < n; ++r) q[r] = q[r] - w * li[r];
            }
            int64_t piv2 = (j + 1 < n) ? pivot_search_sampled(q, n, used_n, ms, sd, (uint32_t)(j + 1), 1u) : -1;
            if (piv2 < 0) { st = ORC_BREAKDOWN; break; }
            double wp = q[piv2];
            if (out->W) WW(j + 1, j + 1) = wp;
            double* lnext = L + (int64_t)(j + 1) * n;
            for (int64_t r = 0; r < n; ++r) lnext[r] = q[r] / wp;
            gp[j + 1] = piv2; used_n[piv2] = 1; ng = j + 2;
            if (P->lam > 0.0 && !none) sketch_apply(&S1, lnext, F + (int64_t)(j + 1) * s);
        }
    }

small_ls:
    out->k_done = k_done;
    for (int64_t r = 0; r < n; ++r) out->x[r] = 0.0;
    if (none && k_done > 0) {
        /* CMRH / LSLU (Sec. 3.1, eq. (Hessenber_LS); with Tikhonov eq. (TP)):
         * M_{k+1}^+ (b - A L_k y) = beta e_1 - H_{k+1,k} y and
         * L_k^+ L_k y = y, so the problem is eq. (TSP):
         *   min ||beta e_1 - H y||^2 + lam^2 ||y||^2,
         * the same stacked least squares with Z = H, F = [I; 0], c = beta e_1. */
        for (int j = 0; j < k; ++j)
            for (int64_t i = 0; i < s; ++i) {
                Z[(int64_t)j * s + i] = out->H[(int64_t)j * kk1 + i];
                F[(int64_t)j * s + i] = (i == j) ? 1.0 : 0.0;
            }
        for (int64_t i = 0; i < s; ++i) c[i] = 0.0;
        c[0] = beta0;
    }
    if (k_done > 0) {
        int lst = orc_small_ls(s, k_done, Z, F, P->lam, c, y, out->res);
        if (lst != ORC_OK) { st = lst; goto done; }
        for (int j = 0; j < k_done; ++j) {    /* x = L_k y */
            const double* lj = L + (int64_t)j * n;
            for (int64_t r = 0; r < n; ++r) out->x[r] += lj[r] * y[j];
        }
    } else if (st == ORC_OK) {
        st = ORC_BREAKDOWN;
    }
    for (int i = 0; i < nt; ++i) out->t[i] = tp[i];
    if (out->g) for (int i = 0; i < ng; ++i) out->g[i] = gp[i];
    out->n_t = nt;
    out->n_g = ng;
    if (out->Lb) memcpy(out->Lb, L, sizeof(double) * (size_t)(n * (k + 1)));
    if (out->Db && rect) memcpy(out->Db, D, sizeof(double) * (size_t)(m * (k + 1)));
    if (out->Z) memcpy(out->Z, Z, sizeof(double) * (size_t)(s * k));
    if (out->F) memcpy(out->F, F, sizeof(double) * (size_t)(s * k));
    if (out->c) memcpy(out->c, c, sizeof(double) * (size_t)s);
#undef HH
#undef WW
done:
    free(L); free(D); free(Z); free(F); free(c); free(u); free(q);
    free(used_m); free(used_n); free(y); free(tp); free(gp);
    sketch_free(&S1); sketch_free(&S2);
    return st;
}
