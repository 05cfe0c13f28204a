// Internal interfaces of liblogdet_cheb: step descriptors, kernel launchers and the host
// planner's helpers.  Not part of the public C ABI (include/logdet_cheb.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ld {

// Where an operand of the fused recurrence step comes from.
enum Src : int {
  SRC_NONE = 0,  // operand absent (coefficient treated as 0)
  SRC_BUF = 1,   // device vector block, d x M row-major (probe index contiguous)
  SRC_HASH = 2,  // the Rademacher probe block V, regenerated from the counter hash
  SRC_SAME = 3,  // (diagonal operand only) same as the gathered operand: the diagonal
                 // coefficient is folded into the matrix entry with col == row
};

// One matrix's share of one recurrence step:
//   out[r, :] = ag * sum_t val[t] * G[col[t], :] + bd * D[r, :] + cp * P[r, :] + cv * V[r, :]
// for every row r, plus (optionally) per-tile partial sums of V[r, p] * out[r, p].
// `out` may alias `P` (in-place update); it never aliases G or D.
struct StepDesc {
  const int64_t* row_ptr;
  const int32_t* col;
  const void* val;
  const void* G;
  const void* D;
  const void* P;
  void* out;
  double ag, bd, cp, cv;
  uint64_t seed;
  int64_t d;
  double* mu_part;   // [tiles of this matrix][M] doubles for this step, or nullptr
  double* mu_part2;  // second inner product (MU_PAIR), same layout
  int64_t tile0;    // global index of this matrix's first tile
  int32_t active;   // 0: skip this matrix at this step
  int32_t pad_;
};

// Kernel shape chosen by the planner (or the autotuner).
struct Shape {
  int vpl;          // vector elements per lane (1, 2 or 4; divides M)
  int lpr_log2;     // log2 lanes per row (LPR * vpl >= min(M, 64 * vpl))
  int tile_rows;    // rows per workgroup tile (multiple of 4 * (64 / LPR))
  int probe_tiles;  // gridDim.y: ceil(M / (LPR * vpl))
  int plane = 0;    // tiles per plane of the plane-major tile order (general step and adjoint kernels;
                    // a multiple of 8 dividing the tile count), 0: tiles in row order
};

// Launch configuration for a whole step over a tile list.
struct StepLaunch {
  StepDesc d0;              // the matrix when descs == nullptr (single-matrix launches)
  const StepDesc* descs;    // device array, one per matrix, or nullptr
  int nmat;
  const int32_t* tile_mat;  // device [ntiles] matrix of each tile, or nullptr (single matrix)
  const int64_t* tile_row0; // device [ntiles] first row of each tile, or nullptr
  int64_t ntiles;
  int64_t tile_rows;
  int M;
  Shape shape;
};

// Capacity of the LDS copy of a row tile's CSR slice (rows, nonzeros).  Tiles larger than
// this still work but read their slice from global memory.
constexpr int kStageRows = 1024;
constexpr int kStageNnz = 2048;

// Value type tags
enum ValT : int { VAL_F64 = 0, VAL_F32 = 1, VAL_BF16 = 2 };

// Moment epilogue of a step that produces W_{k+1} from W_k:
enum Mu : int {
  MU_NONE = 0,   // none
  MU_PROBE = 1,  // mu_part  <- per-tile sums of v_j^T W_{k+1}          (moment k+1)
  MU_PAIR = 2,   // mu_part  <- per-tile sums of W_k^T W_{k+1},  mu_part2 <- W_{k+1}^T W_{k+1}
};

// Launch one fused step.  gsrc/dsrc/psrc select the operand sources (uniform across
// matrices), mu the moment epilogue.  Returns a hipError_t.
hipError_t launch_step(const StepLaunch& L, int vec_f64, int valt, int gsrc, int dsrc, int psrc, int mu,
                       hipStream_t s);

// Adjoint step (gradient): for row r with y1 = Y_{k+1}:
//   if spmm: out[r,:] = cv * V[r,:] + ag * sum_t val[t] y1[col[t],:] + bd * y1[r,:] + cp * Y2[r,:]
//   G[t] += gw * sum_p y1[r,p] * W[col[t],p]    (SDDMM on the pattern of the matrix)
//   gdiag_part[tile] += gw * sum_p y1[r,p] * W[r,p]
//   with spmm the new vector also takes the seed  cw * W[r,:] + cwm * Wm[r,:] + cwp * Wp[r,:]
//   (Wm, Wp nullable): the direct derivative of the estimate with respect to w_k.
// Two-gather form only (sym off), the shifted adjoint: Y1 holds yh = y + ce * W (yh_{k+1} =
// y_{k+1} + eps_{k+1} w_k), and the product runs on z = Y1 + ck * W:
//   out[r,:] = ag * sum_t val[t] z[col[t],:] + bd * z[r,:] + cp * Y2[r,:] + cw * W[r,:] + ...
//   G[t] += gw * sum_p (Y1[r,p] - ce * W[r,p]) * W[col[t],p]
// (ck = ce = 0 is the plain two-gather form).
struct AdjDesc {
  const int64_t* row_ptr;
  const int32_t* col;
  const void* val;
  const void* Y1;  // y_{k+1}
  const void* Y2;  // y_{k+2} (or nullptr)
  void* out;       // y_k (may alias Y2), or nullptr when spmm is off
  const void* W;   // w_k (nullptr => probe hash, k = 0)
  const void* Wm;  // w_{k-1} for the seed, or nullptr
  const void* Wp;  // w_{k+1} for the seed, or nullptr
  void* Gacc;      // nnz accumulators (float for FP32 vectors, double for FP64)
  double* gdiag_part;  // [tiles] doubles
  double ag, bd, cp, cv, gw, cw, cwm, cwp;
  double ck, ce;  // shifted adjoint (two-gather form): z = Y1 + ck W in the product, y = Y1 - ce W in G
  uint64_t seed;
  int64_t d;
};

// Vector tiles staged in LDS (the shifted adjoint on stencil patterns).  Tiles are one row pass of
// a block, TR = 4 * 64 / LPR consecutive rows.  A pattern is a stencil pattern for TR when the rows
// that tile t's entries reach outside the tile are always among r0 + ofs[j] for one short list of
// offsets (grids and lattices in their natural order) and every row stores its diagonal: the block
// then copies the rows of y_{k+1} and w_k for its own rows and r0 + ofs[j] (those inside [0, d))
// into LDS, and every entry reads its operands from there.  Entries are kept in a padded layout, K
// slots per row in tile order (slot (tile * TR + lr) * K + k), so that no address in the kernel
// depends on a load: the packed entries (LDS slot of the column -- own row r0 + c at c, offset
// ofs[j] at TR + j -- with its value) and the gradient accumulators live in that layout, and emap
// carries a slot back to its stored entry (-1: padding).
constexpr int kStencilRuns = 8;   // the offset list as at most this many runs of consecutive offsets
struct StencilDesc {
  const void* ent;  // [ntiles * TR * K] packed entries: BF16 values: uint32 (value bits << 16 | slot);
                    // FP32: (slot, value bits) as 2 x uint32; FP64: (slot, 0, value) as 16 bytes
  void* hacc;       // [ntiles * TR * K] gradient accumulators (vector type) per entry slot
  int K, nofs, nruns;
  int run_base[kStencilRuns];   // first LDS halo index of each run (prefix sums of the run lengths)
  int run_delta[kStencilRuns];  // offset of halo index j in run q: j + run_delta[q]
};
constexpr int kStencilRows = 64;  // largest staged tile
constexpr int kStencilK = 8;      // most entries per row (K of 5 and 7, the 2-D and 3-D grids, run exactly)
constexpr int kStencilLdsBytes = 48 << 10;  // LDS for the two staged vector tiles (y_{k+1}, w_k)
inline int stencil_tile_rows(int lpr_log2) { return 4 * (64 >> lpr_log2); }
inline size_t stencil_entry_bytes(int valt) { return valt == VAL_BF16 ? 4 : (valt == VAL_F32 ? 8 : 16); }

// The shifted adjoint step (spmm, ck/ce, no Wm/Wp) on staged stencil tiles; the SDDMM accumulates
// into S.hacc (the diagonal entries' accumulators carry the shift's derivative; no gdiag partials).
// sddmm: the closing term y_1 w_0^T alone (A.Y1 = yh_1, A.ce = eps_1, w_0 from the probe hash of
// A.seed; no product, no output), for the forms adjoint_stencil_sddmm_supported admits.
hipError_t launch_adjoint_stencil(const AdjDesc& A, const StencilDesc& S, int M, const Shape& sh, int vec_f64,
                                  int valt, bool y2, bool sddmm, hipStream_t s);
bool adjoint_stencil_sddmm_supported(int vec_f64, int valt, const Shape& sh, const StencilDesc& S);
// The recurrence step (launch_step's operands) on staged stencil tiles, for the combinations
// step_stencil_supported accepts: FP32 vectors, FP32/BF16 values, the diagonal folded into the product,
// W_k from a buffer (W_{k-1} from a buffer or the probe hash, or none with probe moments) or from the
// probe hash (no W_{k-1}), MU_PAIR, MU_PROBE or MU_NONE, one probe tile, tiles a whole number of
// stencil tiles.  S's plan must be for the launch shape's stencil tile.
bool step_stencil_supported(const StepLaunch& L, int vec_f64, int valt, int gsrc, int dsrc, int psrc, int mu);
hipError_t launch_step_stencil(const StepLaunch& L, const StencilDesc& S, int valt, int gsrc, int psrc, int mu,
                               hipStream_t s);
// ent[i] = packed (lcol[i], emap[i] >= 0 ? val[emap[i]] : 0), i < n.
hipError_t launch_stencil_pack(const void* val, int valt, const int32_t* emap, const uint16_t* lcol, int64_t n,
                               void* ent, hipStream_t s);
// acc[emap[i]] += hacc[i] for emap[i] >= 0 (every stored entry appears once), i < n.
hipError_t launch_stencil_unpack(const void* hacc, int vec_f64, const int32_t* emap, int64_t n, void* acc,
                                 hipStream_t s);
// part[b] += fixed-order partial sums of hacc[dslot[i]] over rows i (blocks b < 256): the staged
// steps' share of d Gamma / d shift.
hipError_t launch_stencil_diag_sum(const void* hacc, int vec_f64, const int64_t* dslot, int64_t d, double* part,
                                   hipStream_t s);

// out[r,:] = cv * V[r,:] + cw * W[r,:] + cwm * Wm[r,:] + cwp * Wp[r,:] (W, Wm, Wp nullable):
// the adjoint's starting vector.
hipError_t launch_seed(void* out, int vec_f64, const void* W, const void* Wm, const void* Wp, double cv, double cw,
                       double cwm, double cwp, uint64_t seed, int64_t d, int M, hipStream_t s);

// sym: the pattern is symmetric and A.Gacc accumulates the transposed entries (see the kernel).
hipError_t launch_adjoint(const AdjDesc& A, int M, const Shape& sh, int vec_f64, int valt, bool spmm,
                          bool w_hash, bool y2, bool sym, hipStream_t s);

// perm[t] = index of the stored entry (col[t], row(t)); *missing |= 1 if some is absent.
hipError_t launch_transpose_index(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t nnz, int64_t* perm,
                                  int* missing, hipStream_t s);

// hist[b] += count of stored entries (i, j) with bit_length(|i - j|) = b, b < kDistBins (hist zeroed
// by the caller; d <= 2^31 keeps b <= 32).
constexpr int kDistBins = 33;
hipError_t launch_distance_hist(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t nnz,
                                unsigned long long* hist, hipStream_t s);

// out[0] = max(out[0], largest |i - j| of a stored entry); with band > 0 also out[1] += the entries
// farther than band / 16 from both the diagonal and distance `band` (out zeroed by the caller).
hipError_t launch_plane_fit(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t band,
                            unsigned long long* out, hipStream_t s);

// out[t] = scale * (a[t] + a[perm[t]]) / 2
hipError_t launch_sym_scale(const void* a, int a_f64, const int64_t* perm, int64_t n, double scale, void* out,
                            int out_f64, hipStream_t s);

// Deterministic reduction of per-tile partials:
// mu[j * ldmu + k] = sum_{t < ntiles} part[k][t][j] for k in [k_lo, k_hi].
// part is laid out as part + (k - k_lo) * kstride + t * M + j.
// tmp: reduce_scratch_bytes(k_hi - k_lo + 1, M) bytes of device scratch.
hipError_t launch_reduce_moments(const double* part, int64_t ntiles, int M, int k_lo, int k_hi, int64_t kstride,
                                 double* mu, int ldmu, double* tmp, hipStream_t s);
size_t reduce_scratch_bytes(int nk, int M);

// Batched reduction: for matrix i, tiles [tile_range[2i], tile_range[2i+1]) of degree k (k <= n[i])
// into mu[i][j][k].  part[(k-1) * kstride + tile * M + j].
hipError_t launch_reduce_batched(const double* part, const int64_t* tile_range, const int* n, int count, int M,
                                 int kmax, int64_t kstride, double* mu, hipStream_t s);

hipError_t launch_sum_doubles(const double* x, int64_t n, double* out, hipStream_t s);

hipError_t launch_gershgorin(const int64_t* row_ptr, const int32_t* col, const void* val, int valt, double shift,
                             int64_t d, double* lo_part, double* hi_part, int nblocks, hipStream_t s);

// One workgroup's share of a batched Gershgorin pass: rows [row0, row1) of one matrix.
struct GershItem {
  const int64_t* row_ptr;
  const int32_t* col;
  const void* val;
  double shift;
  int64_t row0, row1;
};
hipError_t launch_gershgorin_batched(const GershItem* items, int nitems, int valt, double* lo_part, double* hi_part,
                                     hipStream_t s);

// Laplacian minor L(hub) of a graph given by its adjacency pattern (see the kernel); valt is
// VAL_F64 or VAL_F32.  max_part / bad_part: nblocks partial maxima of the degree and counts of rows
// that miss the hub or carry a self loop.
hipError_t launch_laplacian_minor(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t hub, int64_t deg_hub,
                                  int64_t* rp_out, int32_t* col_out, void* val_out, int valt, int64_t* max_part,
                                  int64_t* bad_part, int nblocks, hipStream_t s);

hipError_t launch_probes(uint64_t seed, int M, int64_t rows, int8_t* out, hipStream_t s);

// C^T in CSR form with ascending columns.  val/val_t may be null (pattern only); src_t (nullable)
// receives, for every entry of C^T, the index of the entry of C it came from.
hipError_t launch_transpose(const int64_t* row_ptr, const int32_t* col, const void* val, int valt, int64_t d,
                            int64_t nnz, int64_t* row_ptr_t, int32_t* col_t, void* val_t, int64_t* cursor,
                            void* scan_tmp, size_t scan_tmp_bytes, hipStream_t s, int64_t* src_t = nullptr);
size_t transpose_scratch_bytes(int64_t d);

// out[u] = val[src[u]] for u < n (values of type valt): the values of C^T from its source map.
hipError_t launch_gather_values(const void* val, int valt, const int64_t* src, int64_t n, void* out, hipStream_t s);

// Gradient output through an index map: scatter = 0: out[u] = scale * a[idx[u]];
// scatter = 1: out[idx[u]] = scale * a[u] (idx a permutation of [0, n)).
hipError_t launch_perm_scale(const void* a, int a_f64, const int64_t* idx, int64_t n, double scale, void* out,
                             int out_f64, int scatter, hipStream_t s);

// *out (device) = an order-independent 64-bit hash of a CSR pattern (row_ptr[0..d], col[0..nnz)):
// the sum mod 2^64 of a mixing function of (position, value) over both arrays.
hipError_t launch_pattern_hash(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t nnz, uint64_t* out,
                               hipStream_t s);

hipError_t launch_scale_grad(const void* Gacc, int acc_f64, int64_t nnz, double scale, void* out, int out_f64,
                             hipStream_t s);

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// FP64 dot product into device memory: *out = x^T y (part: 512 doubles of scratch).
hipError_t launch_dot(const double* x, const double* y, int64_t n, double* part, double* out, hipStream_t s);

// Lanczos steps with coefficients that stay in device memory (no host round trip per step):
// w <- w - (*alpha) v - sqrt(*bb_prev) u (bb_prev null: no u term);  y <- x / sqrt(*bb).
hipError_t launch_lanczos_update(double* w, const double* v, const double* u, const double* alpha,
                                 const double* bb_prev, int64_t n, hipStream_t s);
hipError_t launch_lanczos_scale(const double* x, const double* bb, int64_t n, double* y, hipStream_t s);


hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace ld
