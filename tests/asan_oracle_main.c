/*
 * Host AddressSanitizer / UndefinedBehaviorSanitizer driver for the CPU oracle
 * (test infrastructure).  Compiled together with oracle/oracle.c into one
 * executable by tests/test_oracle_asan.py; exercises every oracle routine on a
 * small operator with projector blocks, including the edge cases of a ragged
 * grid (nx = ny = nf), a single plane and an iteration cap, and checks that the
 * results are finite and that a converged column has a small true residual.
 */
#include <stdio.h>

#include "../oracle/oracle.c"

static int check_finite(const cplx *v, int64_t n, const char *what)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(creal(v[i])) || !isfinite(cimag(v[i]))) {
            fprintf(stderr, "%s: non-finite entry %lld\n", what, (long long)i);
            return 1;
        }
    return 0;
}

static int run(int64_t nx, int64_t ny, int64_t nz, int nf, int n_atoms)
{
    const int64_t n = nx * ny * nz;
    const int np = 4;
    double coef[3 * 5];
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k <= nf; ++k) coef[a * (nf + 1) + k] = (k == 0 ? 2.5 : -1.0 / (k * k + 1.0));
    double *vloc = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) vloc[i] = -0.3 * sin(0.7 * (double)i);
    /* atoms: entries at a stride through the grid, no repeated index within an atom */
    int64_t ptr[8] = {0};
    int64_t per = n / 3 < 9 ? n / 3 : 9;
    for (int a = 0; a < n_atoms; ++a) ptr[a + 1] = ptr[a] + per;
    int64_t *idx = malloc(sizeof(int64_t) * (ptr[n_atoms] + 1));
    double *P = malloc(sizeof(double) * (ptr[n_atoms] * np + 1));
    double D[8 * 4];
    for (int a = 0; a < n_atoms; ++a) {
        for (int64_t e = ptr[a]; e < ptr[a + 1]; ++e) {
            idx[e] = (a * 5 + 3 * (e - ptr[a])) % n;
            for (int l = 0; l < np; ++l) P[e * np + l] = 0.1 * cos(0.3 * (double)(e * np + l));
        }
        for (int l = 0; l < np; ++l) D[a * np + l] = 0.5 - 0.25 * l;
    }
    oracle_op op = {nx, ny, nz, nf, np, coef, vloc, n_atoms, ptr, idx, P, D};
    int bad = 0;
    cplx *x = malloc(sizeof(cplx) * n), *y = malloc(sizeof(cplx) * n), *b = calloc(n, sizeof(cplx));
    for (int64_t i = 0; i < n; ++i) x[i] = cos((double)i) + I * sin(2.0 * (double)i);
    oracle_apply_h(&op, x, y);
    bad |= check_finite(y, n, "apply_h");
    /* conventional COCG with the full history and a snapshot */
    const cplx z = 0.1 + 0.05 * I;
    b[n / 2] = 1.0;
    int64_t it = 0;
    const int64_t cap = 400;
    double *h[5];
    for (int q = 0; q < 5; ++q) h[q] = malloc(sizeof(double) * cap);
    cplx *snap = malloc(sizeof(cplx) * n);
    int st = oracle_cocg(&op, &z, b, 1e-12, cap, x, &it, h[0], h[1], h[2], h[3], h[4], 3, snap);
    bad |= check_finite(x, n, "cocg");
    if (st == OR_CONVERGED) {
        /* true residual of the converged column */
        oracle_apply_h(&op, x, y);
        double s = 0;
        for (int64_t i = 0; i < n; ++i) {
            const cplx t = b[i] - (z * x[i] - y[i]);
            s += creal(t) * creal(t) + cimag(t) * cimag(t);
        }
        if (sqrt(s) > 1e-9) {
            fprintf(stderr, "cocg true residual %g\n", sqrt(s));
            bad = 1;
        }
    }
    /* iteration cap: must stop at the cap with status max-iter */
    st = oracle_cocg(&op, &z, b, 1e-30, 5, x, &it, NULL, NULL, NULL, NULL, NULL, -1, NULL);
    if (st != OR_MAXITER || it != 5) {
        fprintf(stderr, "cap: status %d iters %lld\n", st, (long long)it);
        bad = 1;
    }
    /* batch of unit columns, rows = every point */
    const int64_t ns = 3;
    cplx zs[3] = {0.1 + 0.05 * I, -0.4 + 0.02 * I, 1.5 + 0.1 * I};
    int64_t rhs[3] = {0, n - 1, n / 3};
    int64_t *rows = malloc(sizeof(int64_t) * n);
    for (int64_t i = 0; i < n; ++i) rows[i] = i;
    cplx *out = malloc(sizeof(cplx) * ns * n), *xf = malloc(sizeof(cplx) * ns * n);
    int64_t its[3];
    int32_t sts[3];
    if (oracle_cocg_unit_batch(&op, ns, zs, rhs, rows, n, 1e-11, 2000, out, its, sts, xf)) bad = 1;
    bad |= check_finite(out, ns * n, "unit batch");
    /* shifted COCG with and without switching */
    const int32_t K = 3;
    cplx *xs = malloc(sizeof(cplx) * K * n);
    int64_t itk[3];
    int32_t stk[3], nsw = 0, sf = 0;
    double est[3];
    for (int sw = 0; sw <= 1; ++sw) {
        oracle_shifted_cocg(&op, K, zs, b, 0, sw, 1e-11, 2000, xs, itk, stk, est, &nsw, &sf);
        bad |= check_finite(xs, K * n, "shifted");
    }
    for (int q = 0; q < 5; ++q) free(h[q]);
    free(snap); free(rows); free(out); free(xf); free(xs);
    free(x); free(y); free(b); free(vloc); free(idx); free(P);
    return bad;
}

int main(void)
{
    int bad = 0;
    bad |= run(6, 5, 7, 4, 2);   /* projectors, nf = 4 */
    bad |= run(4, 4, 1, 4, 1);   /* nx = ny = nf, a single plane */
    bad |= run(3, 5, 9, 1, 3);   /* central difference */
    bad |= run(5, 3, 4, 2, 0);   /* no projector blocks */
    if (!bad) printf("oracle sanitizer run ok\n");
    return bad;
}
