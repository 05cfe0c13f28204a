/*
 * ldo.c -- oracle for the stochastic Chebyshev log-determinant estimator
 * (Han, Malioutov & Shin, arXiv 1503.06394).
 *
 * TEST INFRASTRUCTURE ONLY: plain, slow, single-threaded FP64 C, written from the
 * paper and checked against closed forms, library routines and brute force in the
 * test suite.  Nothing in the GPU library includes, links or calls this file.
 *
 * Readings of the paper taken here:
 *  - Algorithm 1 computes coefficients of f o g with g(x) = ((1 - 2 delta) x + 1)/2 mapping
 *    [-1, 1] onto [delta, 1 - delta] (Section 4.1), so its recurrence runs on the mapped
 *    matrix X = g^{-1}(A) = (2A - I)/(1 - 2 delta), whose spectrum lies in [-1, 1].
 *  - The branch "n > 1" of Algorithm 1 is read as n >= 1 (otherwise n = 1 drops c_1).
 *  - A positive definite matrix with spectrum in [a, b] enters Algorithm 1 as
 *    B/(a + b) with delta = a/(a + b), and d log(a + b) is added back (the same
 *    normalise-and-shift step Algorithm 2 uses).
 */
#include "ldo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Chebyshev interpolation, Section 2.1                                       */
/* ------------------------------------------------------------------------- */

void ldo_cheb_nodes(int n, double *x)
{
    const double pi = 3.14159265358979323846;
    for (int k = 0; k <= n; ++k)
        x[k] = cos(pi * (k + 0.5) / (n + 1));
}

/* eq. (1): c_0 = 1/(n+1) sum_k f(x_k) T_0(x_k), c_i = 2/(n+1) sum_k f(x_k) T_i(x_k),
 * with T_0 = 1, T_1 = x, T_{i+1} = 2 x T_i - T_{i-1} (eq. (2)). */
void ldo_cheb_coeffs_from_values(int n, const double *fx, double *c)
{
    double *x = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *tprev = (double *)malloc(sizeof(double) * (size_t)(n + 1)); /* T_{i-1}(x_k) */
    double *tcur = (double *)malloc(sizeof(double) * (size_t)(n + 1));  /* T_i(x_k) */
    ldo_cheb_nodes(n, x);
    for (int k = 0; k <= n; ++k) {
        tprev[k] = 0.0;
        tcur[k] = 1.0; /* T_0 */
    }
    for (int i = 0; i <= n; ++i) {
        double sum = 0.0;
        for (int k = 0; k <= n; ++k)
            sum += fx[k] * tcur[k];
        c[i] = (i == 0 ? 1.0 : 2.0) / (n + 1) * sum;
        /* advance T_i -> T_{i+1} at every node */
        for (int k = 0; k <= n; ++k) {
            double tnext = (i == 0) ? x[k] : 2.0 * x[k] * tcur[k] - tprev[k];
            tprev[k] = tcur[k];
            tcur[k] = tnext;
        }
    }
    free(x);
    free(tprev);
    free(tcur);
}

int ldo_cheb_coeffs_alg1(double delta, int n, double *c)
{
    if (n < 0 || !(delta > 0.0) || !(delta < 0.5))
        return -1;
    double *x = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *fx = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!x || !fx) {
        free(x);
        free(fx);
        return -2;
    }
    ldo_cheb_nodes(n, x);
    for (int k = 0; k <= n; ++k)
        fx[k] = log(1.0 - ((1.0 - 2.0 * delta) * x[k] + 1.0) / 2.0);
    ldo_cheb_coeffs_from_values(n, fx, c);
    free(x);
    free(fx);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Rademacher probes (Section 2.2) from a counter-based hash                  */
/* ------------------------------------------------------------------------- */

/* SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014), applied to the
 * generator state seed + (ctr + 1) * golden-gamma. */
static uint64_t splitmix64_at(uint64_t seed, uint64_t ctr)
{
    uint64_t z = seed + (ctr + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int ldo_probe_sign(uint64_t seed, int64_t j, int64_t r)
{
    uint64_t ctr = ((uint64_t)r << 16) | ((uint64_t)j >> 6);
    uint64_t word = splitmix64_at(seed, ctr);
    return ((word >> ((uint64_t)j & 63u)) & 1u) ? -1 : 1;
}

void ldo_probe(uint64_t seed, int64_t j, int64_t d, double *v)
{
    for (int64_t r = 0; r < d; ++r)
        v[r] = (double)ldo_probe_sign(seed, j, r);
}

static void get_probe(const ldo_probes *p, int64_t i, int64_t d, double *v)
{
    if (p->V) {
        memcpy(v, p->V + i * d, sizeof(double) * (size_t)d);
    } else {
        ldo_probe(p->seed, p->ids ? p->ids[i] : i, d, v);
    }
}

/* ------------------------------------------------------------------------- */
/* Sparse products                                                            */
/* ------------------------------------------------------------------------- */

/* y = B x */
static void csr_mv(const ldo_csr *B, const double *x, double *y)
{
    for (int64_t i = 0; i < B->d; ++i) {
        double acc = 0.0;
        for (int64_t t = B->row_ptr[i]; t < B->row_ptr[i + 1]; ++t)
            acc += B->val[t] * x[B->col[t]];
        y[i] = acc;
    }
}

/* y = C^T x, by scattering the rows of C (no explicit transpose). */
static void csr_mv_t(const ldo_csr *C, const double *x, double *y)
{
    for (int64_t i = 0; i < C->d; ++i)
        y[i] = 0.0;
    for (int64_t i = 0; i < C->d; ++i)
        for (int64_t t = C->row_ptr[i]; t < C->row_ptr[i + 1]; ++t)
            y[C->col[t]] += C->val[t] * x[i];
}

static double dot(int64_t d, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < d; ++i)
        s += x[i] * y[i];
    return s;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1                                                                */
/* ------------------------------------------------------------------------- */

/* X w = g^{-1}(A) w = (2 A w - w) / (1 - 2 delta), with A w = w - B w. */
static void apply_X(int64_t d, ldo_matvec_fn matvec, const void *ctx, double delta,
                    const double *w, double *Aw_scratch, double *out)
{
    matvec(ctx, w, Aw_scratch); /* B w */
    for (int64_t i = 0; i < d; ++i) {
        double Aw = w[i] - Aw_scratch[i];
        out[i] = (2.0 * Aw - w[i]) / (1.0 - 2.0 * delta);
    }
}

int ldo_alg1(int64_t d, ldo_matvec_fn matvec, const void *ctx, double delta, int n, int m,
             const ldo_probes *probes, double *gamma, double *s, double *mom)
{
    if (d < 0 || n < 0 || m < 1 || !matvec || !probes || !gamma || !(delta > 0.0) || !(delta < 0.5))
        return -1;
    double *c = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *u = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *w0 = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *w1 = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *w2 = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    int rc = 0;
    if (!c || !v || !u || !w0 || !w1 || !w2 || !tmp) {
        rc = -2;
        goto done;
    }
    ldo_cheb_coeffs_alg1(delta, n, c);

    double G = 0.0;
    for (int i = 0; i < m; ++i) {
        get_probe(probes, i, d, v);
        for (int64_t r = 0; r < d; ++r)
            u[r] = c[0] * v[r];
        if (mom)
            mom[(int64_t)i * (n + 1) + 0] = dot(d, v, v);
        if (n >= 1) {
            memcpy(w0, v, sizeof(double) * (size_t)d);
            apply_X(d, matvec, ctx, delta, v, tmp, w1);
            for (int64_t r = 0; r < d; ++r)
                u[r] += c[1] * w1[r];
            if (mom)
                mom[(int64_t)i * (n + 1) + 1] = dot(d, v, w1);
            for (int j = 2; j <= n; ++j) {
                apply_X(d, matvec, ctx, delta, w1, tmp, w2); /* w2 = X w1 ...      */
                for (int64_t r = 0; r < d; ++r)
                    w2[r] = 2.0 * w2[r] - w0[r];             /* ... = 2 X w1 - w0 */
                for (int64_t r = 0; r < d; ++r)
                    u[r] += c[j] * w2[r];
                if (mom)
                    mom[(int64_t)i * (n + 1) + j] = dot(d, v, w2);
                double *t = w0; /* w0 <- w1, w1 <- w2 */
                w0 = w1;
                w1 = w2;
                w2 = t;
            }
        }
        double sv = dot(d, v, u);
        if (s)
            s[i] = sv;
        G += sv / m;
    }
    *gamma = G;
done:
    free(c);
    free(v);
    free(u);
    free(w0);
    free(w1);
    free(w2);
    free(tmp);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Positive definite matrices with spectrum in [a, b]                         */
/* ------------------------------------------------------------------------- */

typedef struct {
    const ldo_csr *B;
    double shift;
    double scale; /* 1/(a + b) */
} pd_ctx;

/* y = (B + shift I) x / (a + b) */
static void pd_matvec(const void *vctx, const double *x, double *y)
{
    const pd_ctx *p = (const pd_ctx *)vctx;
    csr_mv(p->B, x, y);
    for (int64_t i = 0; i < p->B->d; ++i)
        y[i] = (y[i] + p->shift * x[i]) * p->scale;
}

/* y = (B + shift I)^T x / (a + b): the transposed operator, which the reverse-mode
 * recurrence of the gradient applies. */
static void pd_matvec_t(const void *vctx, const double *x, double *y)
{
    const pd_ctx *p = (const pd_ctx *)vctx;
    csr_mv_t(p->B, x, y);
    for (int64_t i = 0; i < p->B->d; ++i)
        y[i] = (y[i] + p->shift * x[i]) * p->scale;
}

static int check_csr(const ldo_csr *B)
{
    if (!B || B->d < 0 || B->nnz < 0 || !B->row_ptr || (B->nnz > 0 && (!B->col || !B->val)))
        return -1;
    if (B->row_ptr[0] != 0 || B->row_ptr[B->d] != B->nnz)
        return -1;
    for (int64_t i = 0; i < B->d; ++i)
        if (B->row_ptr[i + 1] < B->row_ptr[i])
            return -1;
    for (int64_t t = 0; t < B->nnz; ++t)
        if (B->col[t] < 0 || B->col[t] >= B->d)
            return -1;
    return 0;
}

int ldo_logdet(const ldo_csr *B, double shift, double a, double b, int n, int m,
               const ldo_probes *probes, double *gamma, double *s, double *mom)
{
    if (check_csr(B) || !(a > 0.0) || !(b > a) || !isfinite(b) || !gamma)
        return -1;
    pd_ctx ctx = {B, shift, 1.0 / (a + b)};
    double delta = a / (a + b);
    double g = 0.0;
    int rc = ldo_alg1(B->d, pd_matvec, &ctx, delta, n, m, probes, &g, s, mom);
    if (rc)
        return rc;
    double lift = (double)B->d * log(a + b);
    *gamma = g + lift;
    if (s)
        for (int i = 0; i < m; ++i)
            s[i] += lift;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Taylor-series comparator (Section 5.1's accuracy comparison)               */
/* ------------------------------------------------------------------------- */

/* With the normalisation of Section 3.1, B' = (B + shift I)/(a + b) has spectrum in
 * [delta, 1 - delta] and A = I - B' in [delta, 1 - delta] as well, so
 *     log det B' = log det(I - A) = tr log(I - A) = - sum_{k>=1} tr(A^k) / k.
 * Truncate after degree n, estimate every trace with the same probe (Hutchinson), and add back
 * d log(a + b).  Not the paper's method: the series it is compared against. */
int ldo_logdet_taylor(const ldo_csr *B, double shift, double a, double b, int n, int m,
                      const ldo_probes *probes, double *gamma, double *s)
{
    if (check_csr(B) || !(a > 0.0) || !(b > a) || !isfinite(b) || n < 0 || m < 1 || !probes || !gamma)
        return -1;
    const int64_t d = B->d;
    pd_ctx ctx = {B, shift, 1.0 / (a + b)};
    double *v = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *bw = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    if (!v || !w || !bw) {
        free(v);
        free(w);
        free(bw);
        return -2;
    }
    const double lift = (double)d * log(a + b);
    double G = 0.0;
    for (int i = 0; i < m; ++i) {
        get_probe(probes, i, d, v);
        memcpy(w, v, sizeof(double) * (size_t)d);
        double series = 0.0; /* sum_k v^T A^k v / k */
        for (int k = 1; k <= n; ++k) {
            pd_matvec(&ctx, w, bw); /* B' w */
            for (int64_t r = 0; r < d; ++r)
                w[r] = w[r] - bw[r]; /* w <- A w = A^k v */
            series += dot(d, v, w) / (double)k;
        }
        const double sv = lift - series;
        if (s)
            s[i] = sv;
        G += sv / m;
    }
    *gamma = G;
    free(v);
    free(w);
    free(bw);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 2                                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
    const ldo_csr *C;
    double scale; /* 1/(smin^2 + smax^2) */
    double *tmp;
} ns_ctx;

/* y = C^T C x / (smin^2 + smax^2) */
static void ns_matvec(const void *vctx, const double *x, double *y)
{
    const ns_ctx *p = (const ns_ctx *)vctx;
    csr_mv(p->C, x, p->tmp);
    csr_mv_t(p->C, p->tmp, y);
    for (int64_t i = 0; i < p->C->d; ++i)
        y[i] *= p->scale;
}

int ldo_logabsdet(const ldo_csr *C, double smin, double smax, int n, int m,
                  const ldo_probes *probes, double *gamma, double *s)
{
    if (check_csr(C) || !(smin > 0.0) || !(smax > smin) || !isfinite(smax) || !gamma)
        return -1;
    double nrm = smin * smin + smax * smax;
    ns_ctx ctx = {C, 1.0 / nrm, (double *)malloc(sizeof(double) * (size_t)(C->d + 1))};
    if (!ctx.tmp)
        return -2;
    double delta = smin * smin / nrm;
    double g = 0.0;
    int rc = ldo_alg1(C->d, ns_matvec, &ctx, delta, n, m, probes, &g, s, NULL);
    free(ctx.tmp);
    if (rc)
        return rc;
    double lift = (double)C->d * log(nrm);
    *gamma = (g + lift) / 2.0;
    if (s)
        for (int i = 0; i < m; ++i)
            s[i] = (s[i] + lift) / 2.0;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Gradient (not in the paper; reverse mode through Algorithm 1)              */
/* ------------------------------------------------------------------------- */
/* The recurrence evaluates v^T p(X) v for any square X, so this is the derivative with
 * respect to independent entries, for symmetric and non-symmetric B alike; at a symmetric X
 * it is itself symmetric, i.e. it is also the derivative along symmetric perturbations. */
/*
 * Per probe v the estimate is s = v^T u with u = sum_k c_k w_k, w_0 = v, w_1 = X v and
 * w_k = 2 X w_{k-1} - w_{k-2}.  w_k enters s directly (c_k v^T w_k), through w_{k+1} (via 2X)
 * and through w_{k+2} (via -1), so the adjoints y_k = ds/dw_k obey
 *   y_n = c_n v,  y_{n-1} = c_{n-1} v + 2 X^T y_n,  y_k = c_k v + 2 X^T y_{k+1} - y_{k+2},
 * and ds/dX = y_1 v^T + sum_{k=2}^{n} 2 y_k w_{k-1}^T.
 * X = ((a + b) I - 2 (B + shift I)) / (b - a), so dX/dB_ij = -2/(b - a) e_i e_j^T and
 * dX/dshift = -2/(b - a) I.  The lift d log(a + b) does not depend on B (a, b fixed).
 */
int ldo_logdet_grad(const ldo_csr *B, double shift, double a, double b, int n, int m,
                    const ldo_probes *probes, double *grad, double *grad_shift, double *gamma)
{
    if (check_csr(B) || !(a > 0.0) || !(b > a) || !isfinite(b) || n < 0 || m < 1 || !probes || !grad)
        return -1;
    const int64_t d = B->d;
    pd_ctx ctx = {B, shift, 1.0 / (a + b)};
    const double delta = a / (a + b);
    double *c = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *W = (double *)malloc(sizeof(double) * (size_t)(n + 1) * (size_t)(d + 1)); /* w_0..w_n */
    double *Y = (double *)malloc(sizeof(double) * (size_t)(n + 2) * (size_t)(d + 1)); /* y_0..y_{n+1} */
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *tmp2 = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *acc = (double *)calloc((size_t)(B->nnz + 1), sizeof(double));
    int rc = 0;
    if (!c || !W || !Y || !tmp || !tmp2 || !acc) {
        rc = -2;
        goto done;
    }
    ldo_cheb_coeffs_alg1(delta, n, c);
    double accshift = 0.0, G = 0.0;
    for (int i = 0; i < m; ++i) {
        double *v = W; /* w_0 = v */
        get_probe(probes, i, d, v);
        /* forward: store every w_k and the estimate s */
        double sv = c[0] * dot(d, v, v);
        if (n >= 1) {
            apply_X(d, pd_matvec, &ctx, delta, v, tmp, W + (d + 1));
            sv += c[1] * dot(d, v, W + (d + 1));
        }
        for (int k = 2; k <= n; ++k) {
            double *wk = W + (int64_t)k * (d + 1);
            apply_X(d, pd_matvec, &ctx, delta, W + (int64_t)(k - 1) * (d + 1), tmp, wk);
            for (int64_t r = 0; r < d; ++r)
                wk[r] = 2.0 * wk[r] - W[(int64_t)(k - 2) * (d + 1) + r];
            sv += c[k] * dot(d, v, wk);
        }
        G += sv / m;
        if (n == 0)
            continue;
        /* backward: y_{n+1} = 0, y_n = c_n v, y_k = c_k v + 2 X^T y_{k+1} - y_{k+2} */
        double *ynp1 = Y + (int64_t)(n + 1) * (d + 1);
        for (int64_t r = 0; r < d; ++r)
            ynp1[r] = 0.0;
        double *yn = Y + (int64_t)n * (d + 1);
        for (int64_t r = 0; r < d; ++r)
            yn[r] = c[n] * v[r];
        for (int k = n - 1; k >= 1; --k) {
            double *yk = Y + (int64_t)k * (d + 1);
            apply_X(d, pd_matvec_t, &ctx, delta, Y + (int64_t)(k + 1) * (d + 1), tmp2, yk); /* X^T y */
            for (int64_t r = 0; r < d; ++r)
                yk[r] = c[k] * v[r] + 2.0 * yk[r] - Y[(int64_t)(k + 2) * (d + 1) + r];
        }
        /* ds/dX restricted to the pattern: y_1 v^T + sum_{k=2}^n 2 y_k w_{k-1}^T */
        for (int64_t r = 0; r < d; ++r) {
            for (int64_t t = B->row_ptr[r]; t < B->row_ptr[r + 1]; ++t) {
                int64_t col = B->col[t];
                double g = Y[(d + 1) + r] * v[col];
                for (int k = 2; k <= n; ++k)
                    g += 2.0 * Y[(int64_t)k * (d + 1) + r] * W[(int64_t)(k - 1) * (d + 1) + col];
                acc[t] += g;
            }
            double gd = Y[(d + 1) + r] * v[r];
            for (int k = 2; k <= n; ++k)
                gd += 2.0 * Y[(int64_t)k * (d + 1) + r] * W[(int64_t)(k - 1) * (d + 1) + r];
            accshift += gd;
        }
    }
    {
        const double chain = -2.0 / (b - a) / m;
        for (int64_t t = 0; t < B->nnz; ++t)
            grad[t] = chain * acc[t];
        if (grad_shift)
            *grad_shift = chain * accshift;
        if (gamma)
            *gamma = G + (double)d * log(a + b);
    }
done:
    free(c);
    free(W);
    free(Y);
    free(tmp);
    free(tmp2);
    free(acc);
    return rc;
}

/* Directional derivative of the ldo_logdet estimate along B -> B + h E, where E has the values
 * e_val on B's pattern and e_shift on the diagonal, at fixed a, b and probes: forward-mode
 * differentiation of Algorithm 1's recurrence.  With X = (I - 2 (B + shift I)/(a + b))/(1 - 2 delta)
 * its tangent is dX = -2 (E + e_shift I)/((a + b)(1 - 2 delta)), and
 *     dw_0 = 0,  dw_1 = dX v,  dw_k = 2 (dX w_{k-1} + X dw_{k-1}) - dw_{k-2},
 *     d s = sum_k c_k v^T dw_k,  d Gamma = (1/m) sum_probes d s.
 * Three sparse products per degree and five vectors per probe, whatever the degree. */
int ldo_logdet_dir(const ldo_csr *B, double shift, double a, double b, int n, int m,
                   const ldo_probes *probes, const double *e_val, double e_shift, double *dgamma)
{
    if (check_csr(B) || !(a > 0.0) || !(b > a) || !isfinite(b) || n < 0 || m < 1 || !probes || !e_val ||
        !dgamma)
        return -1;
    const int64_t d = B->d;
    pd_ctx ctx = {B, shift, 1.0 / (a + b)};
    const double delta = a / (a + b);
    ldo_csr E = *B;
    E.val = e_val;
    const double dxs = -2.0 / ((a + b) * (1.0 - 2.0 * delta)); /* dX = dxs (E + e_shift I) */
    double *c = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    double *v = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *w0 = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *w1 = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *t0 = (double *)malloc(sizeof(double) * (size_t)(d + 1)); /* tangents dw_{k-2}, dw_{k-1} */
    double *t1 = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *xw = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *xt = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *ew = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    int rc = 0;
    if (!c || !v || !w0 || !w1 || !t0 || !t1 || !xw || !xt || !ew || !tmp) {
        rc = -2;
        goto done;
    }
    ldo_cheb_coeffs_alg1(delta, n, c);
    double D = 0.0;
    for (int i = 0; i < m; ++i) {
        get_probe(probes, i, d, v);
        double ds = 0.0; /* c_0 v^T dw_0 = 0 */
        if (n >= 1) {
            memcpy(w0, v, sizeof(double) * (size_t)d); /* w_0 */
            apply_X(d, pd_matvec, &ctx, delta, v, tmp, w1); /* w_1 = X v */
            csr_mv(&E, v, ew);
            for (int64_t r = 0; r < d; ++r) {
                t0[r] = 0.0;                                    /* dw_0 */
                t1[r] = dxs * (ew[r] + e_shift * v[r]);         /* dw_1 = dX v */
            }
            ds += c[1] * dot(d, v, t1);
            for (int k = 2; k <= n; ++k) {
                apply_X(d, pd_matvec, &ctx, delta, w1, tmp, xw); /* X w_{k-1} */
                apply_X(d, pd_matvec, &ctx, delta, t1, tmp, xt); /* X dw_{k-1} */
                csr_mv(&E, w1, ew);                              /* E w_{k-1} */
                for (int64_t r = 0; r < d; ++r) {
                    const double wk = 2.0 * xw[r] - w0[r];
                    const double tk = 2.0 * (dxs * (ew[r] + e_shift * w1[r]) + xt[r]) - t0[r];
                    w0[r] = w1[r];
                    w1[r] = wk;
                    t0[r] = t1[r];
                    t1[r] = tk;
                }
                ds += c[k] * dot(d, v, t1);
            }
        }
        D += ds / m;
    }
    *dgamma = D;
done:
    free(c);
    free(v);
    free(w0);
    free(w1);
    free(t0);
    free(t1);
    free(xw);
    free(xt);
    free(ew);
    free(tmp);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* Spectral interval and stated bounds                                        */
/* ------------------------------------------------------------------------- */

int ldo_gershgorin(const ldo_csr *B, double shift, double *a, double *b)
{
    if (check_csr(B) || !a || !b || B->d == 0)
        return -1;
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = 0; i < B->d; ++i) {
        double diag = 0.0, off = 0.0;
        for (int64_t t = B->row_ptr[i]; t < B->row_ptr[i + 1]; ++t) {
            if (B->col[t] == i)
                diag += B->val[t];
            else
                off += fabs(B->val[t]);
        }
        diag += shift;
        if (diag - off < lo)
            lo = diag - off;
        if (diag + off > hi)
            hi = diag + off;
    }
    *a = lo;
    *b = hi;
    return 0;
}

double ldo_lemma_bound(double delta, int n, int64_t d)
{
    double K = (sqrt(2.0 - delta) + sqrt(delta)) / (sqrt(2.0 - delta) - sqrt(delta));
    return 20.0 * (double)d * log(2.0 * (1.0 / delta - 1.0)) / ((K - 1.0) * pow(K, n));
}
