// Preparation kernels for gfx950 that run once per matrix, before the estimator's loop (Han,
// Malioutov & Shin, arXiv 1503.06394): Gershgorin bounds for a whole batch of matrices in one
// launch, the Lanczos steps of the spectral estimate (the bounds Section 3.2 asks for), the
// Laplacian minor used to count spanning trees (Section 3.3), and the pattern analysis of the
// gradient (values of B^T through a source map, outputs through an index map, a pattern hash).
#include <algorithm>

#include "ld_internal.h"

namespace ld {

// Stored value t of a CSR value array of type VALT, widened to double.
template <int VALT>
__device__ __forceinline__ double value_at(const void* p, int64_t t) {
  if constexpr (VALT == VAL_F64) return static_cast<const double*>(p)[t];
  if constexpr (VALT == VAL_F32) return (double)static_cast<const float*>(p)[t];
  return (double)__uint_as_float((uint32_t)static_cast<const uint16_t*>(p)[t] << 16);  // BF16
}

// --- Gershgorin intervals of a batch ---
//
// Work item i (one per workgroup) covers rows [row0, row1) of one matrix and writes the minimum
// of B_rr + shift - sum_{c != r} |B_rc| and the maximum of B_rr + shift + sum_{c != r} |B_rc| over
// them; the host takes the min / max over a matrix's items.  Same arithmetic per row as the
// single-matrix kernel, and min / max do not depend on order, so the bounds agree bit for bit.
template <int VALT>
__global__ void __launch_bounds__(256) gershgorin_batched_kernel(const GershItem* items, double* lo_part,
                                                                 double* hi_part) {
  const GershItem it = items[blockIdx.x];
  double lo = __builtin_inf(), hi = -__builtin_inf();
  for (int64_t r = it.row0 + threadIdx.x; r < it.row1; r += 256) {
    double diag = 0.0, off = 0.0;
    for (int64_t t = it.row_ptr[r]; t < it.row_ptr[r + 1]; ++t) {
      const double v = value_at<VALT>(it.val, t);
      if (it.col[t] == r)
        diag += v;
      else
        off += fabs(v);
    }
    diag += it.shift;
    lo = fmin(lo, diag - off);
    hi = fmax(hi, diag + off);
  }
  __shared__ double sl[256], sh[256];
  sl[threadIdx.x] = lo;
  sh[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sl[threadIdx.x] = fmin(sl[threadIdx.x], sl[threadIdx.x + w]);
      sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    lo_part[blockIdx.x] = sl[0];
    hi_part[blockIdx.x] = sh[0];
  }
}

hipError_t launch_gershgorin_batched(const GershItem* items, int nitems, int valt, double* lo_part, double* hi_part,
                                     hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  if (valt == VAL_F64)
    hipLaunchKernelGGL(gershgorin_batched_kernel<VAL_F64>, dim3(nitems), dim3(256), 0, s, items, lo_part, hi_part);
  else if (valt == VAL_F32)
    hipLaunchKernelGGL(gershgorin_batched_kernel<VAL_F32>, dim3(nitems), dim3(256), 0, s, items, lo_part, hi_part);
  else
    hipLaunchKernelGGL(gershgorin_batched_kernel<VAL_BF16>, dim3(nitems), dim3(256), 0, s, items, lo_part, hi_part);
  return hipGetLastError();
}

// --- Laplacian minor for spanning-tree counting (Kirchhoff's matrix-tree theorem) ---
//
// Output row r' is graph vertex r = r' + (r' >= hub).  It holds -1 for every neighbour other than the
// hub (columns above the hub shift down by one) and deg(r) on the diagonal, inserted in column order.
// When every vertex is adjacent to the hub, row r' has exactly deg(r) entries and starts at
// row_ptr[r] - (r > hub ? deg(hub) : 0).  A row that misses the hub or has a self loop is counted in
// bad_part; its writes are clipped to its own deg(r) slots, so no write leaves the output arrays.
template <typename OT>
__global__ void __launch_bounds__(256) laplacian_minor_kernel(const int64_t* row_ptr, const int32_t* col, int64_t d,
                                                              int64_t hub, int64_t deg_hub, int64_t* rp_out,
                                                              int32_t* col_out, OT* val_out, int64_t* max_part,
                                                              int64_t* bad_part) {
  int64_t mx = 0, bad = 0;
  const int64_t m = d - 1;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < m; q += (int64_t)gridDim.x * 256) {
    const int64_t r = q + (q >= hub ? 1 : 0);
    const int64_t b = row_ptr[r], e = row_ptr[r + 1], deg = e - b;
    const int64_t ob = b - (r > hub ? deg_hub : 0), oend = ob + deg;
    rp_out[q] = ob;
    int64_t o = ob;
    bool diag_done = false, saw_hub = false, loop = false;
    for (int64_t t = b; t < e; ++t) {
      const int64_t c = col[t];
      if (c == hub) {
        saw_hub = true;
        continue;
      }
      if (c == r) {
        loop = true;
        continue;
      }
      const int64_t cc = c - (c > hub ? 1 : 0);
      if (!diag_done && cc > q) {
        if (o < oend) {
          col_out[o] = (int32_t)q;
          val_out[o] = (OT)deg;
        }
        ++o;
        diag_done = true;
      }
      if (o < oend) {
        col_out[o] = (int32_t)cc;
        val_out[o] = (OT)(-1);
      }
      ++o;
    }
    if (!diag_done) {
      if (o < oend) {
        col_out[o] = (int32_t)q;
        val_out[o] = (OT)deg;
      }
      ++o;
    }
    if (!saw_hub || loop || o != oend) ++bad;
    mx = deg > mx ? deg : mx;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) rp_out[m] = row_ptr[d] - deg_hub;
  __shared__ int64_t smx[256], sbad[256];
  smx[threadIdx.x] = mx;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smx[threadIdx.x] = smx[threadIdx.x] > smx[threadIdx.x + w] ? smx[threadIdx.x] : smx[threadIdx.x + w];
      sbad[threadIdx.x] += sbad[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    max_part[blockIdx.x] = smx[0];
    bad_part[blockIdx.x] = sbad[0];
  }
}

hipError_t launch_laplacian_minor(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t hub, int64_t deg_hub,
                                  int64_t* rp_out, int32_t* col_out, void* val_out, int valt, int64_t* max_part,
                                  int64_t* bad_part, int nblocks, hipStream_t s) {
  if (valt == VAL_F64)
    hipLaunchKernelGGL(laplacian_minor_kernel<double>, dim3(nblocks), dim3(256), 0, s, row_ptr, col, d, hub, deg_hub,
                       rp_out, col_out, static_cast<double*>(val_out), max_part, bad_part);
  else
    hipLaunchKernelGGL(laplacian_minor_kernel<float>, dim3(nblocks), dim3(256), 0, s, row_ptr, col, d, hub, deg_hub,
                       rp_out, col_out, static_cast<float*>(val_out), max_part, bad_part);
  return hipGetLastError();
}

// --- Lanczos steps with device-resident coefficients ---
//
// alpha_j = w^T v and beta_j^2 = w^T w are written to device memory by the dot-product kernel;
// these kernels read them there, so a whole run of steps is queued without waiting for the host.
// The arithmetic is that of host-side coefficients: w - alpha v - beta u with beta = sqrt(bb), and
// (1 / sqrt(bb)) x, every operation IEEE-rounded in FP64.
__global__ void __launch_bounds__(256) lanczos_update_kernel(double* w, const double* v, const double* u,
                                                             const double* alpha, const double* bb_prev, int64_t n) {
  const double a = *alpha;
  const double b = bb_prev ? sqrt(*bb_prev) : 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256)
    w[t] = w[t] - a * v[t] - b * u[t];
}

__global__ void __launch_bounds__(256) lanczos_scale_kernel(const double* x, const double* bb, int64_t n, double* y) {
  const double c = 1.0 / sqrt(*bb);
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) y[t] = c * x[t];
}

static unsigned lanczos_grid(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

hipError_t launch_lanczos_update(double* w, const double* v, const double* u, const double* alpha,
                                 const double* bb_prev, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lanczos_update_kernel, dim3(lanczos_grid(n)), dim3(256), 0, s, w, v, u, alpha, bb_prev, n);
  return hipGetLastError();
}

hipError_t launch_lanczos_scale(const double* x, const double* bb, int64_t n, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lanczos_scale_kernel, dim3(lanczos_grid(n)), dim3(256), 0, s, x, bb, n, y);
  return hipGetLastError();
}

// --- pattern analysis for the gradient ---

template <typename T>
__global__ void __launch_bounds__(256) gather_values_kernel(const T* val, const int64_t* src, int64_t n, T* out) {
  for (int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x; u < n; u += (int64_t)gridDim.x * 256) out[u] = val[src[u]];
}

hipError_t launch_gather_values(const void* val, int valt, const int64_t* src, int64_t n, void* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = lanczos_grid(n);
  if (valt == VAL_F64)
    hipLaunchKernelGGL(gather_values_kernel<double>, dim3(g), dim3(256), 0, s, static_cast<const double*>(val), src, n,
                       static_cast<double*>(out));
  else if (valt == VAL_F32)
    hipLaunchKernelGGL(gather_values_kernel<float>, dim3(g), dim3(256), 0, s, static_cast<const float*>(val), src, n,
                       static_cast<float*>(out));
  else
    hipLaunchKernelGGL(gather_values_kernel<uint16_t>, dim3(g), dim3(256), 0, s, static_cast<const uint16_t*>(val), src,
                       n, static_cast<uint16_t*>(out));
  return hipGetLastError();
}

template <typename TA, typename TO>
__global__ void __launch_bounds__(256) perm_scale_kernel(const TA* a, const int64_t* idx, int64_t n, double scale,
                                                         TO* out, int scatter) {
  for (int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x; u < n; u += (int64_t)gridDim.x * 256) {
    if (scatter)
      out[idx[u]] = (TO)((double)a[u] * scale);
    else
      out[u] = (TO)((double)a[idx[u]] * scale);
  }
}

hipError_t launch_perm_scale(const void* a, int a_f64, const int64_t* idx, int64_t n, double scale, void* out,
                             int out_f64, int scatter, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = lanczos_grid(n);
  if (a_f64 && out_f64)
    hipLaunchKernelGGL((perm_scale_kernel<double, double>), dim3(g), dim3(256), 0, s, static_cast<const double*>(a), idx,
                       n, scale, static_cast<double*>(out), scatter);
  else if (a_f64)
    hipLaunchKernelGGL((perm_scale_kernel<double, float>), dim3(g), dim3(256), 0, s, static_cast<const double*>(a), idx,
                       n, scale, static_cast<float*>(out), scatter);
  else if (out_f64)
    hipLaunchKernelGGL((perm_scale_kernel<float, double>), dim3(g), dim3(256), 0, s, static_cast<const float*>(a), idx,
                       n, scale, static_cast<double*>(out), scatter);
  else
    hipLaunchKernelGGL((perm_scale_kernel<float, float>), dim3(g), dim3(256), 0, s, static_cast<const float*>(a), idx, n,
                       scale, static_cast<float*>(out), scatter);
  return hipGetLastError();
}

// Order-independent pattern hash: every (position, value) pair of row_ptr and col goes through the
// SplitMix64 finaliser (a generic 64-bit mixer here) with a different salt per array; the terms are
// summed modulo 2^64 (per-workgroup sums, then one integer atomic each), so the result does not
// depend on the order of the additions.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256) pattern_hash_kernel(const int64_t* row_ptr, const int32_t* col, int64_t d,
                                                           int64_t nnz, unsigned long long* out) {
  uint64_t h = 0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r <= d; r += stride)
    h += mix64(((uint64_t)r * 0x9E3779B97F4A7C15ull) ^ (uint64_t)row_ptr[r] ^ 0x5851F42D4C957F2Dull);
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < nnz; t += stride)
    h += mix64(((uint64_t)t * 0xD1B54A32D192ED03ull) ^ (uint64_t)(uint32_t)col[t]);
  for (int o = 32; o >= 1; o >>= 1) h += (uint64_t)__shfl_xor((unsigned long long)h, o, 64);
  __shared__ uint64_t sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = h;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, (unsigned long long)(sh[0] + sh[1] + sh[2] + sh[3]));
}

hipError_t launch_pattern_hash(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t nnz, uint64_t* out,
                               hipStream_t s) {
  hipError_t e = launch_fill_zero(out, sizeof(uint64_t), s);
  if (e != hipSuccess) return e;
  const int64_t work = std::max<int64_t>(d + 1, nnz);
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 2047) / 2048, 2048));
  hipLaunchKernelGGL(pattern_hash_kernel, dim3(g), dim3(256), 0, s, row_ptr, col, d, nnz,
                     reinterpret_cast<unsigned long long*>(out));
  return hipGetLastError();
}

}  // namespace ld
