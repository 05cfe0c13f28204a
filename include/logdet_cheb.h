/*
 * logdet_cheb.h -- C ABI of the MI355X (gfx950) stochastic Chebyshev log-determinant
 * library, liblogdet_cheb.so.
 *
 * Method: Han, Malioutov & Shin, "Large-scale Log-determinant Computation through
 * Stochastic Chebyshev Expansions" (arXiv 1503.06394).  For a symmetric positive
 * definite B with spectrum inside [a, b] the library maps B onto
 *     At = (2 B - (a + b) I) / (b - a)               (spectrum in [-1, 1], Section 4.1),
 * interpolates f(x) = log(((b - a) x + (a + b)) / 2) at the n + 1 first-kind Chebyshev
 * nodes (eq. (1), FP64 on the host), runs the three-term recurrence
 *     W_1 = At V,   W_{k+1} = 2 At W_k - W_{k-1}     (eq. (2); Section 2.2)
 * over a block V of M Rademacher probes (Section 2.2) and accumulates the moments
 * mu[j][k] = v_j^T W_k[:, j]; the estimate is
 *     Gamma = (1/M) sum_j sum_k c_k mu[j][k]         (Algorithm 1, final step),
 * which equals Algorithm 1's v^T u by linearity.
 *
 * Conventions shared by every entry point:
 *  - All matrix and vector pointers are DEVICE pointers owned by the caller, on the
 *    current HIP device.  The library never frees caller memory.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on it and
 *    the call synchronises it before returning, because results are host doubles.
 *  - Return value: 0 success; negative = error, outputs untouched, message available
 *    from ld_last_error(); positive = warning with the result filled in.
 *  - CSR: row_ptr monotone with row_ptr[0] = 0 and row_ptr[rows] = nnz, column
 *    indices in [0, cols), no duplicates.  These are trusted, not checked on device.
 *  - Probe j (0 <= j < M) has entry v_j[r] = +1 or -1 at row r from the counter hash
 *        ctr  = (r << 16) | (j >> 6)
 *        word = SplitMix64 output function of (seed + (ctr + 1) * 0x9E3779B97F4A7C15)
 *        v_j[r] = (bit (j & 63) of word) ? -1 : +1
 *    (SplitMix64: Steele, Lea & Flood, OOPSLA 2014).  Matrix i of a batch uses seed + i.
 *  - Nothing here throws or aborts.
 */
#ifndef LOGDET_CHEB_H
#define LOGDET_CHEB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LD_OK 0
#define LD_EINVAL (-1)     /* null pointer, rows != cols, n < 0, M < 1, bad bounds, ... */
#define LD_EDTYPE (-2)     /* unsupported value / vector type combination */
#define LD_EWORKSPACE (-3) /* caller workspace smaller than ld_workspace_bytes() */
#define LD_EHIP (-4)       /* HIP runtime error (message in ld_last_error) */
#define LD_ENOMEM (-5)     /* device allocation failed */
#define LD_WBOUNDS 1       /* warning: some |mu[j][k]| > d (1 + 1e-6): [a, b] misses the spectrum */

/* value types of ld_csr.values */
#define LD_F64 0
#define LD_F32 1
#define LD_BF16 2

/* Square sparse matrix on the device.  The effective matrix is values + diag_shift * I;
 * the shift is kept as an FP64 scalar so that small shifts survive low-precision
 * storage (e.g. 4 + 0.01 is not representable in BF16). */
typedef struct {
    int64_t rows, cols, nnz;
    const int64_t *row_ptr; /* rows + 1 */
    const int32_t *col_idx; /* nnz */
    const void *values;     /* nnz elements of type `dtype` */
    int32_t dtype;          /* LD_F64 | LD_F32 | LD_BF16 */
    int32_t reserved;       /* must be 0 */
    double diag_shift;
} ld_csr;

typedef struct {
    double logdet;          /* Gamma */
    double std_err;         /* sample standard deviation of the per-probe estimates / sqrt(M) */
    double poly_bound;      /* Lemma 7 bound on |log det - tr p_n| for delta = a / (a + b) */
    double grad_shift;      /* d Gamma / d diag_shift (gradient entry point only) */
    double kernel_ms;       /* with ld_opts.timing: summed duration of the recurrence-step kernels */
    double adjoint_ms;      /* with ld_opts.timing: summed duration of the adjoint steps (gradient;
                               product + SDDMM launches, not the closing SDDMM of y_1 w_0^T) */
    int32_t kernel_launches;/* with ld_opts.timing: number of recurrence-step kernels timed */
    int32_t adjoint_launches;
    int32_t n, M;
    uint32_t flags;         /* bit 0: LD_WBOUNDS seen */
    int32_t adjoint_form;   /* gradient entry point: how its adjoint ran (LD_ADJ_*); 0 elsewhere */
    int32_t plane_tiles;    /* gradient entry point: 0 when the general kernels walked the row tiles
                               in row order; > 0 when they walked them plane by plane (a lattice in
                               natural order whose planes span more vector rows than an XCD's L2:
                               each XCD takes one column of every plane, planes in turn), this many
                               tiles per plane.  The results do not depend on the order. */
    int32_t staged_steps;   /* ld_logdet_cheb, the gradient and the Taylor comparator: recurrence steps
                               that ran on vector tiles staged in LDS (stencil patterns, FP32 vectors,
                               FP32 or BF16 values, one probe tile: every step); 0 elsewhere */
} ld_result;

/* ld_result.adjoint_form.  The product-identity forward (symmetric pattern) has two adjoints:
 * the explicit one streams w_{k-1}, w_k, w_{k+1} for its seed and gathers one row of y_{k+1} per
 * stored entry; the shifted one carries y_k + eps_k w_{k-1} instead, which cancels the w_{k-1}
 * and w_{k+1} terms, and reads rows of both y_{k+1} and w_k per entry: two vector blocks less per
 * step.  The shifted form runs by default on stencil patterns, from vector tiles staged in LDS;
 * elsewhere the explicit form runs (LD_GRAD_FORM=shifted|explicit in the environment forces one). */
#define LD_ADJ_EXPLICIT_SINGLE 1 /* explicit seed, one gather per entry (transposed-entry trick) */
#define LD_ADJ_EXPLICIT_TWO 2    /* explicit seed, two gathers per entry */
#define LD_ADJ_SHIFTED 3         /* shifted form, two gathers per entry from global memory */
#define LD_ADJ_PLAIN 4           /* plain recurrence: single-gather adjoint on B^T */
#define LD_ADJ_SHIFTED_STAGED 5  /* shifted form on vector tiles staged in LDS (stencil patterns:
                                    the rows a tile reaches are its own and a fixed offset list) */

typedef struct {
    void *workspace;          /* device scratch, 256-byte aligned (LD_EINVAL otherwise), or NULL:
                                 then the library takes one of its own device buffers, kept for
                                 reuse until ld_clear_cache */
    size_t workspace_bytes;
    int32_t vec_f64;          /* recurrence vectors: 0 = FP64 for FP64 values, else FP32;
                                 1 = FP64; 2 = FP32 */
    int32_t ckpt_stride;      /* gradient: checkpoint every s steps; 0 = automatic: keep every
                                 W_k when that fits (the workspace given, or half of the free
                                 device memory), else every ceil(sqrt(steps)) */
    int32_t tile;             /* kernel shape: 0 = autotuned, > 0 = rows per workgroup */
    int32_t probe_tile;       /* kernel shape: 0 = autotuned, > 0 = probes per pass over the matrix
                                 (the estimators; the gradient's passes are fixed) */
    int32_t timing;           /* 1 = time recurrence-step kernels with HIP events on `stream` */
    int32_t plain_recurrence; /* 1 = one sparse product per degree (Algorithm 1's loop as written;
                                 the gradient then assumes no symmetry);
                                 0 = ceil(n/2) products: moments 2k and 2k+1 from the Chebyshev
                                 product identities T_2k = 2 T_k^2 - T_0, T_2k+1 = 2 T_k+1 T_k - T_1
                                 (needs a symmetric matrix; same estimate up to rounding) */
    double *moments_out;      /* host, nullable: M x (n+1) moments mu[j][k] = v_j^T T_k(At) v_j */
    double *probe_out;        /* host, nullable: M per-probe estimates s_j = sum_k c_k mu[j][k] */
} ld_opts;

/* Algorithm 1 in the [a, b] form: estimate log det(B + diag_shift I) for a symmetric B.
 * Requires 0 < a < b finite, n >= 0, 1 <= M <= 4096.  With vec_f64 = 0 the recurrence runs
 * in FP32 and the moments, coefficients and final sum in FP64.  By default the moments
 * v^T T_k(At) v come from ceil(n/2) sparse products (see ld_opts.plain_recurrence), which
 * assumes B = B^T (not checked); plain_recurrence = 1 evaluates Algorithm 1's recurrence as
 * written, the same v^T p(At) v for any square B. */
int ld_logdet_cheb(const ld_csr *B, double a, double b, int n, int M, uint64_t seed,
                   const ld_opts *opt, void *stream, ld_result *out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): ld_logdet_cheb with the same arguments, results and
 * errors, whose workspace is a fixed device array of the library, LD_NOALLOC_SCRATCH_BYTES
 * (64 MiB) per GPU, held by each GPU the library runs on until the process ends.  The call makes
 * no hipMalloc, hipFree or other allocating call: the kernel shape is the planner's default (no
 * autotuning) and opt->timing is ignored.  opt->workspace must be NULL (LD_EINVAL otherwise).  A
 * problem whose ld_workspace_bytes(B, n, M, 0, ...) exceeds the array gets LD_EWORKSPACE, before
 * any work.  Every call on a GPU shares that GPU's array and leaves its contents behind (nothing in
 * it needs clearing: each step writes every partial it later reads): calls that overlap on one
 * GPU, from several threads or on several streams, race and must be serialised by the caller. */
#define LD_NOALLOC_SCRATCH_BYTES (64ull << 20)
int ld_logdet_cheb_noalloc(const ld_csr *B, double a, double b, int n, int M, uint64_t seed,
                           const ld_opts *opt, void *stream, ld_result *out);

/* Algorithm 2: estimate log|det C| for a non-singular C with singular values in
 * [smin, smax], via log|det C| = (1/2) log det(C^T C).  The recurrence applies C^T (C w)
 * with two sparse products per step.  Ct (nullable) is C^T in CSR form with the same
 * dtype; if NULL the library builds it on the device for the duration of the call.
 * C's diag_shift must be 0. */
int ld_logabsdet_cheb(const ld_csr *C, const ld_csr *Ct, double smin, double smax, int n, int M,
                      uint64_t seed, const ld_opts *opt, void *stream, ld_result *out);

/* Taylor-series comparator, for the accuracy comparison of Section 5.1 (not the paper's method).
 * With the normalisation of Section 3.1, A = I - (B + diag_shift I)/(a + b) has spectrum in
 * [delta, 1 - delta], delta = a/(a + b), and
 *     log det(B + diag_shift I) = d log(a + b) - sum_{k>=1} tr(A^k) / k.
 * The series is truncated after degree n and every trace is estimated with the same M probes as
 * ld_logdet_cheb: Gamma = d log(a + b) - (1/M) sum_j sum_{k=1..n} v_j^T A^k v_j / k, one sparse
 * product per degree.  out->poly_bound is the truncation bound d q^(n+1) / ((n+1)(1-q)),
 * q = b/(a + b); moments_out receives v_j^T A^k v_j (k = 0..n).  Arguments and errors as for
 * ld_logdet_cheb (plain_recurrence does not apply). */
int ld_logdet_taylor(const ld_csr *B, double a, double b, int n, int M, uint64_t seed,
                     const ld_opts *opt, void *stream, ld_result *out);

/* Gradient of the ld_logdet_cheb estimate (same B, a, b, n, M, seed, with a and b held
 * fixed) with respect to every stored entry of B, scaled by grad_output (not in the paper: a
 * reverse-mode derivation of Algorithm 1's recurrence).  Two forms:
 *  - default, pattern holding its transpose: B is taken as symmetric (Algorithm 1's premise; the
 *    values are not checked), the forward uses the product identities, and each stored entry
 *    receives the derivative along symmetric perturbations,
 *        grad_values[t] = grad_output * (dGamma/dB_ij + dGamma/dB_ji) / 2,  (i, j) = entry t,
 *    which at a symmetric B equals dGamma/dB_ij;
 *  - a pattern without its transpose, or opt->plain_recurrence = 1: no symmetry is assumed.  The
 *    forward runs Algorithm 1's recurrence as written and the adjoint
 *    y_k = c_k v + 2 At^T y_{k+1} - y_{k+2} runs on B^T, so that
 *        grad_values[t] = grad_output * dGamma/dB_ij   for each stored entry on its own.
 * The adjoint runs backwards over segments recomputed from checkpoints every ckpt_stride steps.
 * Probes run in passes of at most 128 (FP32 vectors) or 64 (FP64), whose contributions add up;
 * 1 <= M <= 4096 as for ld_logdet_cheb, with the same probes.  grad_values is a device array of
 * nnz elements of type grad_dtype (LD_F64 or LD_F32).  out->grad_shift receives
 * grad_output * dGamma/d diag_shift and out->logdet the forward estimate.
 * Pattern analysis: the first call on a pattern (keyed by device, row_ptr, col_idx, rows, nnz)
 * learns whether it holds its transpose, and keeps the transposed-entry index (or the pattern of
 * B^T) in library device memory until ld_clear_cache (at most 8 patterns, least recently used
 * dropped); only that first call synchronises before the forward.  Every call also hashes the
 * pattern on the device; if the hash no longer matches (the arrays were rewritten in place), the
 * pattern is analysed again and the call repeated before it returns. */
int ld_logdet_cheb_grad(const ld_csr *B, double a, double b, int n, int M, uint64_t seed,
                        double grad_output, void *grad_values, int grad_dtype,
                        const ld_opts *opt, void *stream, ld_result *out);

/* Batched Algorithm 1: matrix i (count of them, uneven sizes) uses its own bounds
 * [a[i], b[i]], degree n[i] and probe seed seed + i, all with M probes.  The whole batch
 * runs as one captured HIP graph, cached per batch signature (device pointers, sizes, bounds,
 * degrees, seed; at most 8 graphs, least recently used dropped).  Without opt->tile, the first
 * call on a signature whose members total 65536 rows or more captures one graph per candidate
 * shape and keeps the fastest replay (LD_AUTOTUNE=0 in the environment skips that).
 * a, b, n, outs are host arrays of `count` entries;
 * Bs is a host array of descriptors pointing at device data.  a and b may both be NULL:
 * then every member gets its Gershgorin interval (ld_gershgorin_batched).  opt->moments_out
 * and opt->probe_out are ignored. */
int ld_logdet_cheb_batched(int count, const ld_csr *Bs, const double *a, const double *b,
                           const int *n, int M, uint64_t seed, const ld_opts *opt, void *stream,
                           ld_result *outs);

/* Gershgorin interval of B + diag_shift I (FP64), an interval [a, b] holding the spectrum, the
 * input Algorithm 1 needs (Section 3.2 discusses how such bounds are obtained):
 * a = min_i (B_ii + shift - sum_{j != i} |B_ij|), b = max_i (B_ii + shift + sum_{j != i} |B_ij|).
 * a and b are host doubles; LD_EINVAL for an empty matrix. */
int ld_gershgorin(const ld_csr *B, double *a, double *b, void *stream);

/* Gershgorin intervals of `count` matrices (host array of descriptors of device data, one
 * dtype, none empty) in one pass: a[i], b[i] (host) as ld_gershgorin would give them, bit for
 * bit (the bounds of a1 for a batch). */
int ld_gershgorin_batched(int count, const ld_csr *Bs, double *a, double *b, void *stream);

/* Estimates of the extreme eigenvalues of B + diag_shift I (gram = 0, B symmetric) or of
 * C^T C (gram = 1; Ct nullable, built on the device if NULL) by `iters` steps of the Lanczos
 * process in FP64 from a Rademacher start vector (probe 0 of `seed`), without
 * reorthogonalisation.  *lo and *hi receive the extreme Ritz values: *hi <= lambda_max and
 * *lo >= lambda_min, converging from inside the spectrum, so they are ESTIMATES, not bounds;
 * callers pad them (Section 3.2 suggests power / inverse power iteration for these bounds).
 * 2 <= iters <= 2000. */
int ld_spectral_estimate(const ld_csr *B, const ld_csr *Ct, int gram, int iters, uint64_t seed,
                         void *stream, double *lo, double *hi);

/* Spanning-tree counting (Section 3.3).  By Kirchhoff's matrix-tree theorem the number of
 * spanning trees of a graph G is tau(G) = det L(hub), where L(hub) is the Laplacian D - A of G
 * with the row and column of one vertex removed.  When that vertex is adjacent to every other
 * vertex, every row of L(hub) has diagonal deg(i) and deg(i) - 1 off-diagonal entries -1, so its
 * spectrum lies in [1, 2 Delta_max - 1], Delta_max being the largest degree among the other
 * vertices (the hub's edge included).
 *
 * ld_laplacian_minor builds L(hub) from the adjacency pattern `adj` of a simple undirected graph
 * (device CSR with both orientations of every edge, sorted columns, no self loops; values
 * ignored).  Output, all device arrays owned by the caller: row_ptr_out (rows entries, i.e. the
 * rows - 1 rows of the minor plus one), col_out and val_out (adj->nnz - (rows - 1) entries,
 * columns sorted, values of type val_dtype: LD_F64 or LD_F32, exact integers).  Row r of the
 * minor is vertex r + (r >= hub); columns above the hub shift down by one.  *max_degree receives
 * Delta_max.  LD_EINVAL if the hub's degree is not rows - 1, or if some vertex misses the hub,
 * has a self loop or repeats a neighbour (outputs then undefined, but no write leaves them). */
int ld_laplacian_minor(const ld_csr *adj, int64_t hub, int64_t *row_ptr_out, int32_t *col_out,
                       void *val_out, int32_t val_dtype, int64_t *max_degree, void *stream);

/* log tau(G) for a graph whose vertex `hub` is adjacent to every other vertex (Section 3.3):
 * method 1 runs Algorithm 2 with C = L(hub) and singular values in [1, 2 Delta_max - 1], as the
 * spanning-tree corollary states; method 0 runs Algorithm 1 on the symmetric positive definite
 * L(hub) with spectrum in [1, 2 Delta_max - 1].  The minor is built on the device in one of the
 * library's internal buffers (opt->workspace only serves the estimator); values and
 * vectors are FP64 when opt->vec_f64 = 1, else FP32.  out->logdet is the estimate of log tau(G).
 * When Delta_max = 1 the minor is the identity and 0 is returned exactly (probe_out zeroed,
 * moments_out untouched).  Errors as for ld_laplacian_minor and ld_logdet_cheb. */
int ld_log_spanning_trees(const ld_csr *adj, int64_t hub, int n, int M, uint64_t seed, int method,
                          const ld_opts *opt, void *stream, ld_result *out);

/* Quadratic form x^T (B + diag_shift I) x in FP64 for a device FP64 vector x of B->rows
 * entries: the data term of a Gaussian log-likelihood, -x^T J x / 2 (Section 5.2).  One sparse
 * product into library scratch and a fixed-order FP64 dot; *out is a host double. */
int ld_quadratic_form(const ld_csr *B, const double *x, void *stream, double *out);

/* The Rademacher probes of Hutchinson's estimator (Section 2.2) as every kernel regenerates them:
 * out[r * M + j] = v_j[r] (int8, +1/-1) for r < rows, j < M, out a caller-owned device array of
 * rows * M bytes.  For tests and inspection; the estimators never store probes. */
int ld_probes(uint64_t seed, int M, int64_t rows, int8_t *out, void *stream);

/* C^T of a square CSR matrix (Algorithm 2 applies C^T (C w), Section 3.2) into caller-owned
 * device buffers: row_ptr_t (rows + 1), col_t and val_t (nnz, C's dtype).  Rows of the result have
 * ascending column indices; the result is deterministic. */
int ld_transpose(const ld_csr *C, int64_t *row_ptr_t, int32_t *col_t, void *val_t, void *stream);

/* Device bytes the entry point `mode` (0 logdet, 1 logabsdet, 2 grad, 3 taylor) needs as
 * workspace; vec_f64: 1 = FP64 recurrence vectors, 0 = FP32.  The estimators' figure covers every
 * shape their autotuner may pick; the gradient's assumes the default tile height (a smaller
 * opt->tile needs more room for per-tile partials, and a short workspace gives LD_EWORKSPACE). */
size_t ld_workspace_bytes(const ld_csr *B, int n, int M, int mode, int vec_f64);

/* Device-to-device streaming copy with the library's own kernel (HBM bandwidth probe);
 * returns the kernel duration in milliseconds through *ms (nullable).  dst and src must be
 * 16-byte aligned (LD_EINVAL otherwise); any byte count is copied exactly. */
int ld_copy(void *dst, const void *src, size_t bytes, void *stream, double *ms);

/* Release the library's cached batched graphs (with their device memory), its idle internal
 * workspaces, the gradient's pattern analyses and its autotuning results.  Not safe to call while
 * another thread is inside the library. */
int ld_clear_cache(void);

/* Message for the last non-zero status returned on this thread. */
const char *ld_last_error(void);

/* Library version string. */
const char *ld_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LOGDET_CHEB_H */
