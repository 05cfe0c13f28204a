/*
 * ldo.h -- oracle for the stochastic Chebyshev log-determinant estimator of
 * Han, Malioutov & Shin, "Large-scale Log-determinant Computation through
 * Stochastic Chebyshev Expansions" (arXiv 1503.06394).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 C
 * implementation written to be checked against the paper by eye.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * All pointers are HOST pointers.  Functions return 0 on success and a negative
 * value on invalid arguments (-1) or allocation failure (-2); outputs are then
 * left untouched.
 *
 * Parity status of every function: pinned (see the test suite), except where a
 * comment says "parity unpinned".
 */
#ifndef LDO_H
#define LDO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Square sparse matrix in CSR form; values in FP64.  Columns need not be sorted. */
typedef struct {
    int64_t d;              /* rows == columns */
    int64_t nnz;
    const int64_t *row_ptr; /* d+1 entries, row_ptr[0] == 0, row_ptr[d] == nnz */
    const int32_t *col;     /* nnz entries in [0, d) */
    const double  *val;     /* nnz entries */
} ldo_csr;

/* Where the probe vectors come from.  If V is non-NULL, probe i is V[i*d .. i*d+d-1]
 * (entries +1/-1 for Rademacher probes, though any values are accepted).  Otherwise
 * probe i is the counter-hash Rademacher vector with index ids[i] (or i when ids is
 * NULL) under seed `seed`, see ldo_probe_sign. */
typedef struct {
    const double  *V;
    uint64_t       seed;
    const int64_t *ids;
} ldo_probes;

/* Chebyshev nodes x_k = cos(pi (k + 1/2) / (n + 1)), k = 0..n (Section 2.1, eq. (1)). */
void ldo_cheb_nodes(int n, double *x);

/* Chebyshev interpolation coefficients c_0..c_n of eq. (1) from the values f(x_k) at the
 * nodes above; T_i(x_k) is evaluated with the three-term recurrence of eq. (2). */
void ldo_cheb_coeffs_from_values(int n, const double *fx, double *c);

/* Coefficients for Algorithm 1: f(x) = log(1 - ((1 - 2 delta) x + 1) / 2) on [-1, 1]. */
int ldo_cheb_coeffs_alg1(double delta, int n, double *c);

/* Rademacher probe entry v_j[r] in {+1, -1} under the counter-hash spec:
 *   ctr  = (r << 16) | (j >> 6)
 *   word = SplitMix64 output function applied to seed + (ctr + 1) * 0x9E3779B97F4A7C15
 *   v    = +1 if bit (j & 63) of word is 0, else -1.
 * SplitMix64 as published by Steele, Lea & Flood (OOPSLA 2014). */
int ldo_probe_sign(uint64_t seed, int64_t j, int64_t r);

/* Fill v[0..d) with probe j. */
void ldo_probe(uint64_t seed, int64_t j, int64_t d, double *v);

/* Matrix-vector product callback: y = B x, for the normalised B of Algorithm 1. */
typedef void (*ldo_matvec_fn)(const void *ctx, const double *x, double *y);

/* Algorithm 1 (Section 3.1) for a positive definite B (given through `matvec`) with
 * eigenvalues in [delta, 1 - delta], m probes and degree n.
 * gamma  : the estimate of log det B.
 * s      : (nullable, m) per-probe values v^T u.
 * mom    : (nullable, m*(n+1)) per-probe moments v^T w_k, k = 0..n, of the mapped
 *          recurrence (diagnostic, not in the paper).
 */
int ldo_alg1(int64_t d, ldo_matvec_fn matvec, const void *ctx, double delta, int n, int m,
             const ldo_probes *probes, double *gamma, double *s, double *mom);

/* log det of a symmetric positive definite (B + shift I) whose spectrum lies in [a, b],
 * by Algorithm 1 applied to (B + shift I)/(a + b) with delta = a/(a + b), plus
 * d log(a + b).  s (nullable, m): per-probe estimates, each including d log(a + b).
 * mom: as in ldo_alg1. */
int ldo_logdet(const ldo_csr *B, double shift, double a, double b, int n, int m,
               const ldo_probes *probes, double *gamma, double *s, double *mom);

/* Taylor-series comparator for the accuracy comparison of Section 5.1 (not the paper's method):
 * with A = I - (B + shift I)/(a + b), log det(B + shift I) = d log(a + b) - sum_{k>=1} tr(A^k)/k,
 * truncated after degree n, each trace estimated with the probes.  s (nullable, m): per-probe
 * values. */
int ldo_logdet_taylor(const ldo_csr *B, double shift, double a, double b, int n, int m,
                      const ldo_probes *probes, double *gamma, double *s);

/* Algorithm 2 (Section 3.2): log|det C| for a non-singular C with singular values in
 * [smin, smax].  s (nullable, m): per-probe values of the final output formula. */
int ldo_logabsdet(const ldo_csr *C, double smin, double smax, int n, int m,
                  const ldo_probes *probes, double *gamma, double *s);

/* Gradient of the ldo_logdet estimate with respect to every stored entry of B (and to the
 * diagonal shift), at fixed a, b and probes, by reverse-mode differentiation of Algorithm 1's
 * recurrence: the adjoint recurrence applies X^T, so the result is the derivative with respect
 * to each stored entry on its own, for any square B (for symmetric B it is symmetric).
 * grad: nnz entries; grad_shift: nullable; gamma: nullable. */
int ldo_logdet_grad(const ldo_csr *B, double shift, double a, double b, int n, int m,
                    const ldo_probes *probes, double *grad, double *grad_shift, double *gamma);

/* Directional derivative of the ldo_logdet estimate along B -> B + h E (E: values e_val on B's
 * pattern, nnz of them, plus e_shift on the diagonal), at fixed a, b and probes, by forward-mode
 * differentiation of Algorithm 1's recurrence (no stored vectors: usable at any size).
 * Equals sum_t grad[t] e_val[t] + grad_shift e_shift of ldo_logdet_grad. */
int ldo_logdet_dir(const ldo_csr *B, double shift, double a, double b, int n, int m,
                   const ldo_probes *probes, const double *e_val, double e_shift, double *dgamma);

/* Gershgorin interval of B + shift I: a = min_i (B_ii + shift - sum_{j!=i} |B_ij|),
 * b = max_i (B_ii + shift + sum_{j!=i} |B_ij|). */
int ldo_gershgorin(const ldo_csr *B, double shift, double *a, double *b);

/* Right-hand side of Lemma 7 (matrix version of the interpolation bound):
 * 20 d log(2 (1/delta - 1)) / ((K - 1) K^n), K = (sqrt(2-delta)+sqrt(delta))/(sqrt(2-delta)-sqrt(delta)). */
double ldo_lemma_bound(double delta, int n, int64_t d);

#ifdef __cplusplus
}
#endif
#endif /* LDO_H */
