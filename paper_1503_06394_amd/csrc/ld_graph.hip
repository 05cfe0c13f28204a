// Graph kernels for gfx950: the Laplacian minor used to count spanning trees (Section 3.3 of
// Han, Malioutov & Shin, arXiv 1503.06394).  Built once per graph, outside the estimator's loop.
#include "ld_internal.h"

namespace ld {

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

}  // namespace ld
