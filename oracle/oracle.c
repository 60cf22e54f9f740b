/*
 * CPU FP64 oracle for the unperturbed Green's-function columns.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The GPU library never
 * links, loads or calls it, and this file shares no code with the GPU path.
 *
 * What it computes (Sec. 3B, Eq. 17): columns of the unperturbed Green's
 * function  G(Z_k) = [Z_k - H_T]^{-1}  of the transition-region Hamiltonian,
 * i.e. the solution x^{(k)} of (Z_k - H_T) x^{(k)} = e_j.
 *
 *   H_T = H_kin + diag(V) + sum_a P_a D_a P_a^T
 *
 * H_kin is the real-space finite-difference kinetic operator (Sec. 2A, Eq. 2):
 * along each axis a symmetric stencil of half-width nf, periodic in x and y,
 * and truncated in z (the finite T block of Eq. 4: the wavefunction vanishes
 * outside planes 0..nz-1).  The nonlocal Kleinman-Bylander part is the
 * extension the paper defers to its finite-difference textbook reference; it
 * is kept as a sum of dense per-atom rank-n_proj blocks.
 *
 * Three routines, each written for checkability, not speed:
 *   oracle_apply_h      y = H x, plain loops.
 *   oracle_cocg         conventional COCG on one system, the Appendix
 *                       recurrences for x_n, r_n, p_n, alpha, beta
 *                       (Eqs. A2-A6) in the paper's order.
 *   oracle_shifted_cocg shifted COCG with collinear residuals (Eqs. A7-A12)
 *                       and seed switching (Eq. A13), storing every x^{(i)}
 *                       in full.
 *
 * Readings where the paper is silent or garbled:
 *   - Eq. A2 states x_0 = p_0 = 0; with Eq. A4 that would freeze x.  Read as
 *     x_0 = 0, p_{-1} = 0, so that p_0 = r_0 = b.
 *   - The bilinear form (u, v) is the unconjugated u^T v (A = A^T != A^H);
 *     residual norms are Euclidean, sqrt(u^H u).
 *   - sigma_i in Eq. A8 is measured from the current seed:
 *     A = Z_s - H, sigma_i = Z_i - Z_s, so Z_i - H = A + sigma_i I.
 *   - Convergence: ||r^{(i)}_n|| = ||r_n|| / |pi^{(s,i)}_n| <= tol * ||b||.
 *     A converged shift is frozen (no further updates).
 *   - Seed switching: once the seed has converged and other shifts are still
 *     active, the new seed is the active shift with the largest residual norm
 *     (smallest |pi|), ties to the lowest index.  The seed vectors r_n, r_{n-1}
 *     and the seed scalars are rebased onto the new seed with Eq. A13.
 *   - Breakdown (a zero bilinear form with a non-zero vector) is reported,
 *     not repaired.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Element-wise loops over a long vector may run on several threads: every element is
 * computed exactly as in the serial loop, so the results do not depend on the thread
 * count.  Reductions (dot products and norms) always run serially, in index order.
 * A top-level call uses every thread; inside the per-system loop of the batch routine,
 * each system gets its share (g_inner, set per system thread). */
static _Thread_local int g_inner = 1;

static int par_n(int64_t n)
{
#ifdef _OPENMP
    if (n < 65536) return 1;
    return omp_in_parallel() ? g_inner : omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

typedef double complex cplx;

/* Hamiltonian description, all arrays owned by the caller. */
typedef struct {
    int64_t nx, ny, nz;
    int32_t nf;             /* stencil half-width */
    int32_t n_proj;         /* projector channels per atom */
    const double *coef;     /* [3][nf+1] H_kin coefficients along x, y, z (Ha) */
    const double *vloc;     /* [N] local potential (Ha) */
    int32_t n_atoms;
    const int64_t *atom_ptr;/* [n_atoms+1] */
    const int64_t *atom_idx;/* [n_entries] grid index */
    const double *atom_P;   /* [n_entries][n_proj] */
    const double *atom_D;   /* [n_atoms][n_proj] */
} oracle_op;

enum { OR_CONVERGED = 0, OR_MAXITER = 1, OR_BREAKDOWN = 2 };

static int64_t wrap(int64_t i, int64_t n) { return ((i % n) + n) % n; }

/* y = H x.  Plain definition of the operator: a sum over the three axes of the
 * 1-D stencil, plus V x, plus the projector blocks.  The periodic neighbour
 * coordinates (i + k) mod n are tabulated once per call (wx, wy), so the loop does
 * no integer division. */
void oracle_apply_h(const oracle_op *op, const cplx *x, cplx *y)
{
    const int64_t nx = op->nx, ny = op->ny, nz = op->nz;
    const int nf = op->nf;
    /* wx[ix + nf + k] = (ix + k) mod nx for -nf <= k <= nf, likewise wy */
    int64_t *wx = malloc(sizeof(int64_t) * (size_t)(nx + 2 * nf));
    int64_t *wy = malloc(sizeof(int64_t) * (size_t)(ny + 2 * nf));
    for (int64_t t = 0; t < nx + 2 * nf; ++t) wx[t] = wrap(t - nf, nx);
    for (int64_t t = 0; t < ny + 2 * nf; ++t) wy[t] = wrap(t - nf, ny);
    /* every y[i] of the stencil part depends on x only: planes are independent */
#pragma omp parallel for schedule(static) num_threads(par_n(nx * ny * nz)) \
    if (par_n(nx * ny * nz) > 1)
    for (int64_t iz = 0; iz < nz; ++iz)
        for (int64_t iy = 0; iy < ny; ++iy)
            for (int64_t ix = 0; ix < nx; ++ix) {
                const int64_t i = ix + nx * (iy + ny * iz);
                cplx acc = op->vloc[i] * x[i];
                for (int k = -nf; k <= nf; ++k) {
                    const int ak = k < 0 ? -k : k;
                    /* x axis, periodic */
                    acc += op->coef[0 * (nf + 1) + ak] * x[wx[ix + nf + k] + nx * (iy + ny * iz)];
                    /* y axis, periodic */
                    acc += op->coef[1 * (nf + 1) + ak] * x[ix + nx * (wy[iy + nf + k] + ny * iz)];
                    /* z axis, zero outside the transition region */
                    if (iz + k >= 0 && iz + k < nz)
                        acc += op->coef[2 * (nf + 1) + ak] * x[ix + nx * (iy + ny * (iz + k))];
                }
                y[i] = acc;
            }
    free(wx);
    free(wy);
    const int np = op->n_proj;
    for (int32_t a = 0; a < op->n_atoms; ++a) {
        cplx c[16];
        for (int l = 0; l < np; ++l) c[l] = 0;
        for (int64_t e = op->atom_ptr[a]; e < op->atom_ptr[a + 1]; ++e)
            for (int l = 0; l < np; ++l)
                c[l] += op->atom_P[e * np + l] * x[op->atom_idx[e]];
        for (int l = 0; l < np; ++l) c[l] *= op->atom_D[a * np + l];
        for (int64_t e = op->atom_ptr[a]; e < op->atom_ptr[a + 1]; ++e)
            for (int l = 0; l < np; ++l)
                y[op->atom_idx[e]] += op->atom_P[e * np + l] * c[l];
    }
}

static int64_t op_n(const oracle_op *op) { return op->nx * op->ny * op->nz; }

/* (u, v) = u^T v, no conjugation. */
static cplx bil(int64_t n, const cplx *u, const cplx *v)
{
    cplx s = 0;
    for (int64_t i = 0; i < n; ++i) s += u[i] * v[i];
    return s;
}

static double nrm2(int64_t n, const cplx *u)
{
    double s = 0;
    for (int64_t i = 0; i < n; ++i) s += creal(u[i]) * creal(u[i]) + cimag(u[i]) * cimag(u[i]);
    return sqrt(s);
}

/* w = (z - H) v */
static void apply_a(const oracle_op *op, cplx z, const cplx *v, cplx *w)
{
    const int64_t n = op_n(op);
    oracle_apply_h(op, v, w);
#pragma omp parallel for schedule(static) num_threads(par_n(n)) if (par_n(n) > 1)
    for (int64_t i = 0; i < n; ++i) w[i] = z * v[i] - w[i];
}

/*
 * Conventional COCG for (z - H) x = b (Appendix, Eqs. A1-A6).
 *
 * Iteration n produces x_n, r_n, p_n from the (n-1)th quantities:
 *   alpha_{n-1} = (r_{n-1}, r_{n-1}) /
 *                 [ (r_{n-1}, A r_{n-1}) - beta_{n-2}/alpha_{n-2} (r_{n-1}, r_{n-1}) ]
 *   x_n = x_{n-1} + alpha_{n-1} p_{n-1}
 *   r_n = (1 + beta_{n-2} alpha_{n-1}/alpha_{n-2} - alpha_{n-1} A) r_{n-1}
 *         - beta_{n-2} alpha_{n-1}/alpha_{n-2} r_{n-2}
 *   beta_{n-1} = (r_n, r_n) / (r_{n-1}, r_{n-1})
 *   p_n = r_n + beta_{n-1} p_{n-1}
 * with x_0 = 0, p_{-1} = 0, r_{-1} = r_0 = b, alpha_{-1} = 1, beta_{-1} = 0.
 *
 * z is passed by pointer (one complex value).
 * Stops at the first n with ||r_n|| <= tol ||b|| (returns OR_CONVERGED), at
 * n = max_iter (OR_MAXITER), or on a vanishing bilinear form (OR_BREAKDOWN).
 * *iters receives n.  If hist_alpha / hist_beta / hist_res are non-NULL they
 * receive alpha_{n-1}, beta_{n-1}, ||r_n|| for n = 1..(*iters) (capacity
 * max_iter).  If snap is non-NULL, r_{snap_iter} is copied there when reached.
 */
int oracle_cocg(const oracle_op *op, const cplx *zp, const cplx *b, double tol, int64_t max_iter,
                cplx *x, int64_t *iters, double *hist_alpha_re, double *hist_alpha_im,
                double *hist_beta_re, double *hist_beta_im, double *hist_res,
                int64_t snap_iter, cplx *snap)
{
    const int64_t n = op_n(op);
    const cplx z = *zp;
    cplx *r_prev = malloc(sizeof(cplx) * n);   /* r_{n-2} */
    cplx *r = malloc(sizeof(cplx) * n);        /* r_{n-1} */
    cplx *r_next = malloc(sizeof(cplx) * n);   /* r_n */
    cplx *p = malloc(sizeof(cplx) * n);        /* p_{n-1} */
    cplx *ar = malloc(sizeof(cplx) * n);       /* A r_{n-1} */
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0;
        r_prev[i] = b[i];
        r[i] = b[i];
        p[i] = b[i];                           /* p_0 = r_0 + beta_{-1} p_{-1} = b */
    }
    cplx alpha_prev = 1.0, beta_prev = 0.0;    /* alpha_{n-2}, beta_{n-2} */
    const double bnorm = nrm2(n, b);
    int status = OR_MAXITER;
    int64_t it = 0;
    if (snap && snap_iter == 0) memcpy(snap, r, sizeof(cplx) * n);
    if (bnorm == 0.0 || nrm2(n, r) <= tol * bnorm) {
        status = OR_CONVERGED;
        goto done;
    }
    cplx rho = bil(n, r, r);                   /* (r_{n-1}, r_{n-1}) */
    for (it = 1; it <= max_iter; ++it) {
        apply_a(op, z, r, ar);
        const cplx mu = bil(n, r, ar);
        const cplx denom = mu - beta_prev / alpha_prev * rho;
        if (rho == 0.0 || denom == 0.0 || !isfinite(creal(denom)) || !isfinite(cimag(denom))) {
            status = OR_BREAKDOWN;
            it -= 1;
            break;
        }
        const cplx alpha = rho / denom;                     /* alpha_{n-1} */
        const cplx c = beta_prev * alpha / alpha_prev;      /* beta_{n-2} alpha_{n-1} / alpha_{n-2} */
#pragma omp parallel for schedule(static) num_threads(par_n(n)) if (par_n(n) > 1)
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
#pragma omp parallel for schedule(static) num_threads(par_n(n)) if (par_n(n) > 1)
        for (int64_t i = 0; i < n; ++i)
            r_next[i] = (1.0 + c) * r[i] - alpha * ar[i] - c * r_prev[i];
        const cplx rho_next = bil(n, r_next, r_next);
        const cplx beta = rho_next / rho;                   /* beta_{n-1} */
#pragma omp parallel for schedule(static) num_threads(par_n(n)) if (par_n(n) > 1)
        for (int64_t i = 0; i < n; ++i) p[i] = r_next[i] + beta * p[i];
        const double res = nrm2(n, r_next);
        if (hist_alpha_re) { hist_alpha_re[it - 1] = creal(alpha); hist_alpha_im[it - 1] = cimag(alpha); }
        if (hist_beta_re) { hist_beta_re[it - 1] = creal(beta); hist_beta_im[it - 1] = cimag(beta); }
        if (hist_res) hist_res[it - 1] = res / bnorm;
        cplx *t = r_prev; r_prev = r; r = r_next; r_next = t;
        if (snap && snap_iter == it) memcpy(snap, r, sizeof(cplx) * n);
        alpha_prev = alpha;
        beta_prev = beta;
        rho = rho_next;
        if (res <= tol * bnorm) { status = OR_CONVERGED; break; }
    }
    if (it > max_iter) it = max_iter;
done:
    *iters = it;
    free(r_prev); free(r); free(r_next); free(p); free(ar);
    return status;
}

/*
 * Many independent systems (z_k, e_{j}) at once: system s uses z[sys_k[s]] and
 * b = e_{rhs[sys_j[s]]}; its solution restricted to rows[0..n_rows) goes to
 * out[s*n_rows ...]; status and iteration count per system.  OpenMP over
 * systems (when compiled with it); with fewer systems than threads, each system's
 * element-wise loops use the threads left over.  Either way each system's
 * arithmetic is that of the sequential routine.
 */
int oracle_cocg_unit_batch(const oracle_op *op, int64_t n_sys, const cplx *zs,
                           const int64_t *rhs, const int64_t *rows, int64_t n_rows,
                           double tol, int64_t max_iter, cplx *out, int64_t *iters,
                           int32_t *status, cplx *x_full)
{
    const int64_t n = op_n(op);
    int bad = 0;
    int outer = 1, inner = 1;
#ifdef _OPENMP
    const int nt = omp_get_max_threads();
    outer = n_sys < nt ? (int)(n_sys > 0 ? n_sys : 1) : nt;
    inner = nt / outer;
    if (inner > 1 && omp_get_max_active_levels() < 2) omp_set_max_active_levels(2);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad) num_threads(outer)
    for (int64_t s = 0; s < n_sys; ++s) {
        g_inner = inner;
        cplx *b = calloc(n, sizeof(cplx));
        cplx *x = malloc(sizeof(cplx) * n);
        if (!b || !x) { bad |= 1; free(b); free(x); continue; }
        b[rhs[s]] = 1.0;
        status[s] = oracle_cocg(op, &zs[s], b, tol, max_iter, x, &iters[s], NULL, NULL, NULL,
                                NULL, NULL, -1, NULL);
        for (int64_t q = 0; q < n_rows; ++q) out[s * n_rows + q] = x[rows[q]];
        if (x_full) memcpy(x_full + s * n, x, sizeof(cplx) * n);
        free(b);
        free(x);
    }
    return bad ? -2 : 0;
}

/*
 * Shifted COCG (Appendix, Eqs. A7-A13) for (z_i - H) x^{(i)} = b, i = 0..K-1,
 * driven by one seed recurrence.  Full vectors x^{(i)}, p^{(i)} are kept
 * (x_out is [K][N]).
 *
 * Seed system: A = z_s - H with s = seed0.  sigma_i = z_i - z_s.  Per seed
 * iteration (producing r_{n+1} from r_n, r_{n-1}):
 *   alpha_n = (r_n, r_n) / [ (r_n, A r_n) - beta_{n-1}/alpha_{n-1} (r_n, r_n) ]
 *   r_{n+1} = (1 + beta_{n-1} alpha_n/alpha_{n-1} - alpha_n A) r_n
 *             - beta_{n-1} alpha_n/alpha_{n-1} r_{n-1}                      (A3)
 *   beta_n  = (r_{n+1}, r_{n+1}) / (r_n, r_n)                               (A6)
 * and for every active shift i:
 *   pi_{n+1} = (1 + beta_{n-1} alpha_n/alpha_{n-1} + alpha_n sigma_i) pi_n
 *              - beta_{n-1} alpha_n/alpha_{n-1} pi_{n-1}                    (A8)
 *   alpha^{(i)}_n = pi_n / pi_{n+1} alpha_n                                 (A9)
 *   beta^{(i)}_n  = (pi_n / pi_{n+1})^2 beta_n                              (A10)
 *   x^{(i)}_{n+1} = x^{(i)}_n + alpha^{(i)}_n p^{(i)}_n                     (A11)
 *   p^{(i)}_{n+1} = r_{n+1} / pi_{n+1} + beta^{(i)}_n p^{(i)}_n             (A7, A12)
 * Initial: pi_0 = pi_{-1} = 1, x^{(i)}_0 = 0, p^{(i)}_0 = b.
 *
 * Shift i is frozen at the first n with ||r_{n}|| / |pi^{(i)}_{n}| <= tol ||b||;
 * iters[i] = n, status[i] as in oracle_cocg.  With seed_switch != 0, when the
 * seed is frozen and shifts remain active, the seed moves to the active shift
 * s~ with the smallest |pi_{n+1}| (Eq. A13):
 *   pi^{(s~,i)}_k = pi^{(s,i)}_k / pi^{(s,s~)}_k  (k = n, n+1),
 *   r_k <- r_k / pi^{(s,s~)}_k, alpha_n <- alpha^{(s~)}_n, beta_n <- beta^{(s~)}_n,
 * and sigma_i = z_i - z_s~.  n_switch receives the number of switches and
 * seed_final the last seed index.
 */
int oracle_shifted_cocg(const oracle_op *op, int32_t K, const cplx *z, const cplx *b,
                        int32_t seed0, int32_t seed_switch, double tol, int64_t max_iter,
                        cplx *x_out, int64_t *iters, int32_t *status, double *est,
                        int32_t *n_switch, int32_t *seed_final)
{
    const int64_t n = op_n(op);
    cplx *r_prev = malloc(sizeof(cplx) * n);
    cplx *r = malloc(sizeof(cplx) * n);
    cplx *r_next = malloc(sizeof(cplx) * n);
    cplx *ar = malloc(sizeof(cplx) * n);
    cplx *p = malloc(sizeof(cplx) * n * K);
    cplx *pi_prev = malloc(sizeof(cplx) * K), *pi = malloc(sizeof(cplx) * K);
    cplx *pi_next = malloc(sizeof(cplx) * K);
    int *active = malloc(sizeof(int) * K);
    const double bnorm = nrm2(n, b);
    for (int64_t i = 0; i < n; ++i) { r_prev[i] = b[i]; r[i] = b[i]; }
    for (int32_t k = 0; k < K; ++k) {
        for (int64_t i = 0; i < n; ++i) { x_out[k * n + i] = 0; p[k * n + i] = b[i]; }
        pi_prev[k] = pi[k] = 1.0;
        active[k] = 1;
        iters[k] = 0;
        status[k] = OR_MAXITER;
        est[k] = 1.0;
    }
    int32_t s = seed0;
    cplx zs = z[s];
    cplx alpha_prev = 1.0, beta_prev = 0.0;
    cplx rho = bil(n, r, r);
    double rnorm = nrm2(n, r);
    int32_t nsw = 0;
    int n_active = K;
    if (bnorm == 0.0) {
        for (int32_t k = 0; k < K; ++k) { status[k] = OR_CONVERGED; active[k] = 0; est[k] = 0; }
        n_active = 0;
    }
    int64_t it;
    for (it = 0; it < max_iter && n_active > 0; ++it) {
        /* seed step n = it */
        apply_a(op, zs, r, ar);
        const cplx mu = bil(n, r, ar);
        const cplx denom = mu - beta_prev / alpha_prev * rho;
        if (rho == 0.0 || denom == 0.0 || !isfinite(creal(denom)) || !isfinite(cimag(denom))) {
            for (int32_t k = 0; k < K; ++k)
                if (active[k]) { status[k] = OR_BREAKDOWN; active[k] = 0; iters[k] = it; }
            n_active = 0;
            break;
        }
        const cplx alpha = rho / denom;
        const cplx c = beta_prev * alpha / alpha_prev;
        for (int64_t i = 0; i < n; ++i)
            r_next[i] = (1.0 + c) * r[i] - alpha * ar[i] - c * r_prev[i];
        const cplx rho_next = bil(n, r_next, r_next);
        cplx beta = rho_next / rho;
        const double rnorm_next = nrm2(n, r_next);
        /* shifts */
        for (int32_t k = 0; k < K; ++k) {
            if (!active[k]) continue;
            const cplx sigma = z[k] - zs;
            pi_next[k] = (1.0 + c + alpha * sigma) * pi[k] - c * pi_prev[k];
            const cplx ak = pi[k] / pi_next[k] * alpha;
            const cplx q = pi[k] / pi_next[k];
            const cplx bk = q * q * beta;
            for (int64_t i = 0; i < n; ++i) {
                x_out[k * n + i] += ak * p[k * n + i];
                p[k * n + i] = r_next[i] / pi_next[k] + bk * p[k * n + i];
            }
            est[k] = rnorm_next / cabs(pi_next[k]) / bnorm;
            if (est[k] <= tol) {
                active[k] = 0;
                status[k] = OR_CONVERGED;
                iters[k] = it + 1;
                --n_active;
            }
        }
        /* seed switch (Eq. A13) */
        cplx alpha_cur = alpha;
        if (seed_switch && !active[s] && n_active > 0) {
            int32_t t = -1;
            for (int32_t k = 0; k < K; ++k)
                if (active[k] && (t < 0 || cabs(pi_next[k]) < cabs(pi_next[t]))) t = k;
            const cplx f_next = pi_next[t], f_cur = pi[t];
            const cplx q = f_cur / f_next;
            alpha_cur = q * alpha;            /* alpha^{(s~)}_n */
            beta = q * q * beta;              /* beta^{(s~)}_n  */
            for (int32_t k = 0; k < K; ++k) {
                if (!active[k]) continue;
                pi_next[k] /= f_next;
                pi[k] /= f_cur;
            }
            for (int64_t i = 0; i < n; ++i) { r_next[i] /= f_next; r[i] /= f_cur; }
            s = t;
            zs = z[s];
            ++nsw;
        }
        /* rotate: r_{n-1} <- r_n, r_n <- r_{n+1} */
        cplx *tmp = r_prev; r_prev = r; r = r_next; r_next = tmp;
        for (int32_t k = 0; k < K; ++k) { pi_prev[k] = pi[k]; pi[k] = pi_next[k]; }
        rho = bil(n, r, r);
        rnorm = nrm2(n, r);
        (void)rnorm;
        alpha_prev = alpha_cur;
        beta_prev = beta;
    }
    for (int32_t k = 0; k < K; ++k)
        if (active[k]) iters[k] = it;
    *n_switch = nsw;
    *seed_final = s;
    free(r_prev); free(r); free(r_next); free(ar); free(p);
    free(pi_prev); free(pi); free(pi_next); free(active);
    return 0;
}
