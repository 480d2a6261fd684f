/*
 * Runs the CPU oracle over small problems under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_oracle_sanitize.py).
 * Every output array is allocated at exactly the size the oracle's
 * interface states, so a write past one is reported.  Covered: sCMRH on
 * a blur (zero and reflective boundaries, separable and general PSF,
 * Gaussian and sparse-sign sketches, lambda = 0 and > 0, sampled
 * pivoting, no sketch), sLSLU on a rectangular CSR matrix, a breakdown
 * (identity operator), b = 0, k = n, a NaN in b, invalid parameters, and
 * the small least-squares routine on a rank-deficient problem.
 * Prints one line per case; exits non-zero when a status is not the
 * expected one.
 */
#include "oracle.c"

#include <stdio.h>

static int failures = 0;

static void expect(const char* name, int got, int want0, int want1)
{
    const int ok = (got == want0 || got == want1);
    printf("%-28s status %d %s\n", name, got, ok ? "ok" : "UNEXPECTED");
    if (!ok) ++failures;
}

/* deterministic values in [-1, 1) */
static double lcg(uint64_t* st)
{
    *st = *st * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(*st >> 11) / 4503599627370496.0 - 1.0;
}

typedef struct {
    orc_out o;
    int64_t n, m, k, s;
} outs;

static void outs_alloc(outs* b, int64_t m, int64_t n, int64_t k, int64_t s, int rect)
{
    memset(b, 0, sizeof *b);
    b->m = m; b->n = n; b->k = k; b->s = s;
    b->o.x = calloc((size_t)n, sizeof(double));
    b->o.H = calloc((size_t)((k + 1) * k), sizeof(double));
    b->o.W = rect ? calloc((size_t)(k * k), sizeof(double)) : NULL;
    b->o.t = calloc((size_t)(k + 1), sizeof(int64_t));
    b->o.g = rect ? calloc((size_t)k, sizeof(int64_t)) : NULL;
    b->o.res = calloc((size_t)k, sizeof(double));
    b->o.Lb = calloc((size_t)(n * (k + 1)), sizeof(double));
    b->o.Db = rect ? calloc((size_t)(m * (k + 1)), sizeof(double)) : NULL;
    b->o.Z = calloc((size_t)(s * k), sizeof(double));
    b->o.F = calloc((size_t)(s * k), sizeof(double));
    b->o.c = calloc((size_t)s, sizeof(double));
}

static void outs_free(outs* b)
{
    free(b->o.x); free(b->o.H); free(b->o.W); free(b->o.t); free(b->o.g); free(b->o.res);
    free(b->o.Lb); free(b->o.Db); free(b->o.Z); free(b->o.F); free(b->o.c);
}

static int run(const orc_op* A, orc_params P, const double* b, int rect)
{
    outs o;
    const int64_t s = (P.sketch == 3) ? P.k + 1 : P.s;
    outs_alloc(&o, A->m, A->n, P.k, s, rect);
    const int st = orc_solve(A, &P, b, &o.o);
    outs_free(&o);
    return st;
}

int main(void)
{
    uint64_t seed = 12345u;
    /* ---- a 24 x 20 blur, radius 2 */
    const int64_t ny = 24, nx = 20, n = ny * nx;
    double ty[5], tx[5], psf[25];
    for (int i = 0; i < 5; ++i) { ty[i] = exp(-0.5 * (i - 2) * (i - 2)); tx[i] = exp(-0.3 * (i - 2) * (i - 2)); }
    for (int i = 0; i < 25; ++i) psf[i] = 0.05 + 0.02 * (i % 7) + (i == 12 ? 0.5 : 0.0);
    double* b = malloc((size_t)n * sizeof(double));
    for (int64_t i = 0; i < n; ++i) b[i] = lcg(&seed);
    orc_op A;
    memset(&A, 0, sizeof A);
    A.kind = 0; A.m = A.n = n; A.ny = ny; A.nx = nx; A.radius = 2; A.bc = 0; A.taps_y = ty; A.taps_x = tx;
    orc_params P;
    memset(&P, 0, sizeof P);
    P.k = 8; P.s = 20; P.lam = 0.0; P.sketch = 0; P.zeta = 4; P.seed = 7; P.method = 0; P.pivot_sample = 0;
    expect("scmrh blur gauss", run(&A, P, b, 0), ORC_OK, ORC_OK);
    P.lam = 1e-3;
    expect("scmrh blur gauss lam", run(&A, P, b, 0), ORC_OK, ORC_OK);
    A.bc = 1; P.sketch = 1;
    expect("scmrh reflect sparse lam", run(&A, P, b, 0), ORC_OK, ORC_OK);
    A.psf = psf; P.pivot_sample = 6;
    expect("scmrh general psf sampled", run(&A, P, b, 0), ORC_OK, ORC_OK);
    A.psf = NULL; P.pivot_sample = 0; P.sketch = 3; P.lam = 0.0;
    expect("scmrh unsketched", run(&A, P, b, 0), ORC_OK, ORC_OK);
    P.sketch = 2; P.s = (int32_t)n;
    expect("scmrh identity sketch", run(&A, P, b, 0), ORC_OK, ORC_OK);
    P.sketch = 0; P.s = 20;

    /* ---- b = 0: nothing to iterate */
    double* z = calloc((size_t)n, sizeof(double));
    expect("scmrh b = 0", run(&A, P, z, 0), ORC_OK, ORC_BREAKDOWN);
    /* ---- a NaN in b: any documented status, no memory or UB error */
    b[7] = NAN;
    {
        const int st = run(&A, P, b, 0);
        expect("scmrh nan in b", st, st, st);
    }
    b[7] = 0.25;

    /* ---- identity operator (delta PSF): the Krylov space has dimension 1 */
    double d1[5] = {0, 0, 1, 0, 0};
    orc_op I = A;
    I.taps_y = d1; I.taps_x = d1; I.bc = 0;
    expect("scmrh breakdown", run(&I, P, b, 0), ORC_BREAKDOWN, ORC_BREAKDOWN);

    /* ---- k = n on a 3 x 3 image */
    orc_op T = A;
    T.ny = 3; T.nx = 3; T.m = T.n = 9; T.radius = 1;
    double t3[3] = {0.25, 1.0, 0.5};
    T.taps_y = t3; T.taps_x = t3;
    orc_params Pk = P;
    Pk.k = 9; Pk.s = 12;
    expect("scmrh k = n", run(&T, Pk, b, 0), ORC_OK, ORC_BREAKDOWN);

    /* ---- invalid parameters */
    orc_params Pb = P;
    Pb.k = 0;
    expect("k = 0", run(&A, Pb, b, 0), ORC_EINVAL, ORC_EINVAL);
    Pb = P;
    Pb.s = Pb.k;
    expect("s < k + 1", run(&A, Pb, b, 0), ORC_EINVAL, ORC_EINVAL);

    /* ---- sLSLU on a 30 x 25 CSR matrix with 1..6 entries per row */
    const int64_t m = 30, nc = 25;
    int64_t rp[31];
    int32_t col[30 * 6];
    double val[30 * 6];
    int64_t e = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < m; ++i) {
        const int cnt = 1 + (int)(i % 6);
        for (int q = 0; q < cnt; ++q) {
            col[e] = (int32_t)((i * 7 + q * 5) % nc);
            val[e] = lcg(&seed) + (q == 0 ? 2.0 : 0.0);
            ++e;
        }
        rp[i + 1] = e;
    }
    orc_op R;
    memset(&R, 0, sizeof R);
    R.kind = 1; R.m = m; R.n = nc; R.rowptr = rp; R.col = col; R.val = val;
    double br[30];
    for (int i = 0; i < 30; ++i) br[i] = lcg(&seed);
    orc_params Q = P;
    Q.method = 1; Q.k = 6; Q.s = 14; Q.sketch = 0; Q.lam = 0.0;
    expect("slslu csr gauss", run(&R, Q, br, 1), ORC_OK, ORC_BREAKDOWN);
    Q.sketch = 1; Q.lam = 1e-2;
    expect("slslu csr sparse lam", run(&R, Q, br, 1), ORC_OK, ORC_BREAKDOWN);
    orc_params Qb = Q;
    Qb.method = 0;
    expect("square method on 30 x 25", run(&R, Qb, br, 0), ORC_EINVAL, ORC_EINVAL);

    /* ---- the small problem: a rank-deficient Z (two equal columns) */
    {
        const int64_t s = 6, k = 3;
        double Z[18], F[18], c[6], y[3], res[3];
        for (int i = 0; i < 6; ++i) {
            Z[i] = lcg(&seed); Z[6 + i] = Z[i]; Z[12 + i] = lcg(&seed);
            F[i] = F[6 + i] = F[12 + i] = 0.0;
            c[i] = lcg(&seed);
        }
        expect("small ls rank deficient", orc_small_ls(s, k, Z, F, 0.0, c, y, res), ORC_ENUMERIC, ORC_ENUMERIC);
        for (int i = 0; i < 6; ++i) Z[6 + i] = lcg(&seed);
        expect("small ls full rank", orc_small_ls(s, k, Z, F, 0.0, c, y, res), ORC_OK, ORC_OK);
    }
    free(b);
    free(z);
    printf("failures %d\n", failures);
    return failures ? 1 : 0;
}
