/*
 * Shifted-COCG oracle: a plain, slow, FP64 CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  It shares no code, header, table or helper with the GPU
 * path; only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  Nothing in the product links it.
 *
 * What it computes (paper: Sec. 3.1 eq. lin_eq, Sec. 3.3 eq. shift_lin_eq):
 * for a real-symmetric sparse H, a right-hand side b and complex shifts z_k,
 *     x_k = (z_k 1 - H)^{-1} b         for every k.
 * The systems are complex symmetric, so COCG (CG with the unconjugated
 * bilinear form u.v = sum_i u_i v_i) applies to each (Sec. 3.3).  One seed
 * system is iterated; every other shift follows from the seed's scalars because
 * the Krylov subspace is shift invariant (Sec. 3.1 eq. inv_KS) and the shifted
 * residuals stay collinear with the seed residual, r_k = r / pi_k (Sec. 3.3).
 * When the seed has converged the iteration continues from another shift as
 * the new seed, keeping everything computed so far (seed switching, Sec. 3.3).
 * Convergence is judged from the residual norm (Sec. 3.4 eq. residual).
 *
 * The paper states these ideas in prose only.  The scalar recurrences used
 * here follow from COCG's residual polynomial R_n:
 *     R_{n+1}(l) = (1 + a_n b_{n-1}/a_{n-1} - a_n l) R_n(l)
 *                  - (a_n b_{n-1}/a_{n-1}) R_{n-1}(l),
 * with the seed matrix A = z_s 1 - H and A + s 1 the shifted matrix
 * (s = z_k - z_s).  Collinearity with R_n^k(0) = 1 forces pi_n^k = R_n(-s):
 *     pi_{n+1} = (1 + a_n s) pi_n + (a_n b_{n-1}/a_{n-1}) (pi_n - pi_{n-1}),
 *     alpha^k_n = (pi_n / pi_{n+1}) a_n,   beta^k_n = (pi_n / pi_{n+1})^2 b_n,
 *     p^k_n = r_n / pi_n + beta^k_{n-1} p^k_{n-1},
 *     x^k_{n+1} = x^k_n + alpha^k_n p^k_n.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

enum { OR_OK = 0, OR_BREAKDOWN = 4, OR_NOCONV = 5 };

/* q = (z 1 - H) p, H in CSR. */
static void apply_shifted(int64_t n, const int64_t *rp, const int64_t *ci, const double *v,
                          cplx z, const cplx *p, cplx *q)
{
    for (int64_t i = 0; i < n; i++) {
        cplx acc = z * p[i];
        for (int64_t k = rp[i]; k < rp[i + 1]; k++)
            acc -= v[k] * p[ci[k]];
        q[i] = acc;
    }
}

/* Unconjugated bilinear form u.v (the COCG inner product). */
static cplx dotu(int64_t n, const cplx *u, const cplx *w)
{
    cplx s = 0;
    for (int64_t i = 0; i < n; i++)
        s += u[i] * w[i];
    return s;
}

static double norm2(int64_t n, const cplx *u)
{
    double s = 0;
    for (int64_t i = 0; i < n; i++)
        s += creal(u[i]) * creal(u[i]) + cimag(u[i]) * cimag(u[i]);
    return sqrt(s);
}

/*
 * Plain COCG for one shift: (z 1 - H) x = b, x_0 = 0.
 * fixed_iter > 0 runs exactly that many iterations with no stopping test.
 * Returns OR_OK / OR_BREAKDOWN / OR_NOCONV; *iters receives the iteration count
 * and *res the final recursive relative residual ||r|| / ||b||.
 */
int oracle_cocg(int64_t n, const int64_t *rp, const int64_t *ci, const double *v, double zr, double zi,
                const double *b_ri, double tol, int max_iter, int fixed_iter, double *x_ri, int *iters,
                double *res)
{
    cplx z = zr + I * zi;
    const cplx *b = (const cplx *)b_ri;
    cplx *x = (cplx *)x_ri;
    cplx *r = malloc(sizeof(cplx) * n), *p = malloc(sizeof(cplx) * n), *q = malloc(sizeof(cplx) * n);
    int status = OR_NOCONV;
    double nb = norm2(n, b);
    for (int64_t i = 0; i < n; i++) {
        x[i] = 0;
        r[i] = b[i];
        p[i] = b[i];
    }
    cplx rho = dotu(n, r, r);
    int limit = fixed_iter > 0 ? fixed_iter : max_iter;
    int it = 0;
    double rel = nb > 0 ? 1.0 : 0.0;
    if (nb == 0) status = OR_OK;
    for (it = 0; it < limit && status != OR_OK; it++) {
        apply_shifted(n, rp, ci, v, z, p, q);
        cplx pq = dotu(n, p, q);
        if (pq == 0 || rho == 0) {
            status = OR_BREAKDOWN;
            break;
        }
        cplx alpha = rho / pq;
        for (int64_t i = 0; i < n; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        cplx rho_new = dotu(n, r, r);
        rel = norm2(n, r) / nb;
        if (fixed_iter <= 0 && rel < tol) {
            status = OR_OK;
            it++;
            break;
        }
        cplx beta = rho_new / rho;
        for (int64_t i = 0; i < n; i++)
            p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    if (fixed_iter > 0 && status != OR_BREAKDOWN) status = OR_OK;
    *iters = it;
    *res = rel;
    free(r);
    free(p);
    free(q);
    return status;
}

/* Options of the shifted solve (mirrored by a ctypes structure in oracle.py). */
typedef struct {
    double tol;
    int max_iter;
    int seed_index;        /* >= 0: the initial seed shift; < 0: the default rule */
    int switching;         /* switch seed when the seed converges */
    int fixed_iter;        /* > 0: exactly this many iterations, no freezing, no automatic switch */
    int force_switch_iter; /* >= 0: switch at the end of this iteration ... */
    int force_switch_to;   /* ... to this shift (test hook for seed independence) */
} oracle_opts;

/*
 * Default initial seed: the shift with the smallest Im z (slowest to converge);
 * ties broken by |Re z - Tr(H)/n| (closest to the spectral centre), then by the
 * lowest index.
 */
int oracle_default_seed(int64_t n, const int64_t *rp, const int64_t *ci, const double *v, int64_t m,
                        const double *z_ri)
{
    double tr = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t k = rp[i]; k < rp[i + 1]; k++)
            if (ci[k] == i) tr += v[k];
    double centre = n > 0 ? tr / (double)n : 0.0;
    int best = 0;
    for (int64_t k = 1; k < m; k++) {
        double ik = z_ri[2 * k + 1], ib = z_ri[2 * best + 1];
        double dk = fabs(z_ri[2 * k] - centre), db = fabs(z_ri[2 * best] - centre);
        if (ik < ib || (ik == ib && dk < db)) best = (int)k;
    }
    return best;
}

/*
 * Shifted COCG with seed switching for one right-hand side b (length n) and
 * m shifts z[k].  Outputs:
 *   X_ri      [m][n] complex: the solutions x_k (frozen when converged)
 *   iters     [m]  iterations after which shift k was frozen (or the total)
 *   status    [m]  0 converged, 4 breakdown, 5 not converged
 *   res       [m]  recursive relative residual ||r|| / (|pi_k| ||b||) at exit
 *   r_ri      [n]  final seed residual r (complex), may be NULL
 *   pi_ri     [m]  final collinearity factors pi_k relative to the final seed, may be NULL
 *   switch_log[2*max_log] pairs (iteration, new seed), *n_switch entries written
 *   *final_seed  the seed shift at exit
 * Returns the worst status (breakdown > not converged > ok).
 */
int oracle_shifted_cocg(int64_t n, const int64_t *rp, const int64_t *ci, const double *v, int64_t m,
                        const double *z_ri, const double *b_ri, const oracle_opts *o, double *X_ri, int *iters,
                        int *status, double *res, double *r_ri, double *pi_ri, int *switch_log, int max_log,
                        int *n_switch, int *final_seed, int *total_iters)
{
    const cplx *z = (const cplx *)z_ri;
    const cplx *b = (const cplx *)b_ri;
    cplx *X = (cplx *)X_ri;
    cplx *P = calloc((size_t)m * n, sizeof(cplx));
    cplx *r = malloc(sizeof(cplx) * n), *p = calloc(n, sizeof(cplx)), *q = malloc(sizeof(cplx) * n);
    cplx *pi = malloc(sizeof(cplx) * m), *pi_prev = malloc(sizeof(cplx) * m);
    cplx *pi_new = malloc(sizeof(cplx) * m), *beta_k = malloc(sizeof(cplx) * m);
    cplx *alpha_k = malloc(sizeof(cplx) * m), *sig = malloc(sizeof(cplx) * m);
    int *active = malloc(sizeof(int) * m);
    int ret = OR_OK;
    int ns = 0;

    int s = o->seed_index >= 0 ? o->seed_index : oracle_default_seed(n, rp, ci, v, m, z_ri);
    double nb = norm2(n, b);
    memset(X, 0, sizeof(cplx) * (size_t)m * n);
    for (int64_t i = 0; i < n; i++)
        r[i] = b[i];
    for (int64_t k = 0; k < m; k++) {
        pi[k] = 1;
        pi_prev[k] = 1;
        beta_k[k] = 0;
        active[k] = 1;
        sig[k] = z[k] - z[s];
        iters[k] = 0;
        status[k] = OR_NOCONV;
        res[k] = 1.0;
    }
    if (nb == 0) {
        for (int64_t k = 0; k < m; k++) {
            active[k] = 0;
            status[k] = OR_OK;
            res[k] = 0;
        }
    }
    cplx alpha_prev = 1, beta_prev = 0;
    cplx rho = dotu(n, r, r);
    int fixed = o->fixed_iter > 0;
    int limit = fixed ? o->fixed_iter : o->max_iter;
    int it;
    int any_active = nb != 0;

    for (it = 0; it < limit && any_active; it++) {
        /* seed direction and seed matrix-vector product */
        for (int64_t i = 0; i < n; i++)
            p[i] = r[i] + beta_prev * p[i];
        apply_shifted(n, rp, ci, v, z[s], p, q);
        cplx pq = dotu(n, p, q);
        if (pq == 0 || rho == 0) {
            ret = OR_BREAKDOWN;
            for (int64_t k = 0; k < m; k++)
                if (active[k]) status[k] = OR_BREAKDOWN;
            break;
        }
        cplx alpha = rho / pq;
        /* shifted scalars and vectors for every active shift */
        int bad_pi = 0;
        for (int64_t k = 0; k < m; k++) {
            if (!active[k]) continue;
            pi_new[k] = (1.0 + alpha * sig[k]) * pi[k] + (alpha * beta_prev / alpha_prev) * (pi[k] - pi_prev[k]);
            if (pi_new[k] == 0) bad_pi = 1;
        }
        if (bad_pi) {
            ret = OR_BREAKDOWN;
            for (int64_t k = 0; k < m; k++)
                if (active[k]) status[k] = OR_BREAKDOWN;
            break;
        }
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < m; k++) {
            if (!active[k]) continue;
            alpha_k[k] = (pi[k] / pi_new[k]) * alpha;
            cplx inv_pi = 1.0 / pi[k];
            cplx *Pk = P + (size_t)k * n, *Xk = X + (size_t)k * n;
            for (int64_t i = 0; i < n; i++) {
                Pk[i] = r[i] * inv_pi + beta_k[k] * Pk[i];
                Xk[i] += alpha_k[k] * Pk[i];
            }
        }
        /* seed residual update (the seed solution itself is X[s], since pi_s = 1) */
        for (int64_t i = 0; i < n; i++)
            r[i] -= alpha * q[i];
        cplx rho_new = dotu(n, r, r);
        double rn = norm2(n, r);
        cplx beta = rho_new / rho;
        any_active = 0;
        for (int64_t k = 0; k < m; k++) {
            if (!active[k]) continue;
            cplx ratio = pi[k] / pi_new[k];
            beta_k[k] = ratio * ratio * beta;
            pi_prev[k] = pi[k];
            pi[k] = pi_new[k];
            iters[k] = it + 1;
            res[k] = rn / (cabs(pi[k]) * nb);
            if (!fixed && res[k] < o->tol) {
                active[k] = 0;
                status[k] = OR_OK;
            }
            any_active |= active[k];
        }
        alpha_prev = alpha;
        beta_prev = beta;
        rho = rho_new;
        if (!any_active) {
            it++;
            break;
        }
        /* seed switching (Sec. 3.3): when the seed has converged, or on request */
        int t = -1;
        if (!fixed && o->switching && !active[s]) {
            double worst = -1;
            for (int64_t k = 0; k < m; k++)
                if (active[k] && res[k] > worst) {
                    worst = res[k];
                    t = (int)k;
                }
        }
        if (o->force_switch_iter == it) t = o->force_switch_to;
        if (t >= 0 && t != s) {
            cplx pt = pi[t], ppt = pi_prev[t];
            cplx inv_pt = 1.0 / pt;
            for (int64_t i = 0; i < n; i++) {
                r[i] = r[i] * inv_pt;
                p[i] = P[(size_t)t * n + i];
            }
            rho = dotu(n, r, r);
            alpha_prev = alpha_prev * ppt / pt;
            beta_prev = beta_k[t];
            for (int64_t k = 0; k < m; k++) {
                pi[k] = pi[k] / pt;
                pi_prev[k] = pi_prev[k] / ppt;
                sig[k] = z[k] - z[t];
            }
            s = t;
            if (ns < max_log) {
                switch_log[2 * ns] = it;
                switch_log[2 * ns + 1] = t;
            }
            ns++;
        }
    }
    if (ret == OR_OK)
        for (int64_t k = 0; k < m; k++)
            if (status[k] != OR_OK) {
                if (fixed) status[k] = OR_OK;
                else ret = OR_NOCONV;
            }
    if (r_ri) memcpy(r_ri, r, sizeof(cplx) * n);
    if (pi_ri) memcpy(pi_ri, pi, sizeof(cplx) * m);
    *n_switch = ns;
    *final_seed = s;
    *total_iters = it;
    free(P);
    free(r);
    free(p);
    free(q);
    free(pi);
    free(pi_prev);
    free(pi_new);
    free(beta_k);
    free(alpha_k);
    free(sig);
    free(active);
    return ret;
}

/* True residual b - (z 1 - H) x and its relative norm (Sec. 3.4 eq. residual, sign flipped). */
double oracle_true_residual(int64_t n, const int64_t *rp, const int64_t *ci, const double *v, double zr,
                            double zi, const double *x_ri, const double *b_ri)
{
    const cplx *x = (const cplx *)x_ri, *b = (const cplx *)b_ri;
    cplx *q = malloc(sizeof(cplx) * n);
    apply_shifted(n, rp, ci, v, zr + I * zi, x, q);
    double s = 0;
    for (int64_t i = 0; i < n; i++) {
        cplx d = b[i] - q[i];
        s += creal(d) * creal(d) + cimag(d) * cimag(d);
    }
    free(q);
    double nb = norm2(n, b);
    return nb > 0 ? sqrt(s) / nb : sqrt(s);
}
