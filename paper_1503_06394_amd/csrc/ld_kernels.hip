// HIP kernels for gfx950 (CDNA4) of the stochastic Chebyshev log-determinant estimator
// (Han, Malioutov & Shin, arXiv 1503.06394).
//
// The hot loop is the three-term recurrence W_{k+1} = 2 At W_k - W_{k-1} (Section 2.2,
// eq. (2)) over a block of M Rademacher probes: a sparse-matrix x dense-block product
// whose arithmetic intensity (about 1-2 flop/byte) puts it far below the MFMA and even
// the FP32-vector ridge points, so nothing here uses matrix cores.  Design points:
//  * Vector blocks are d x M row-major (probe index contiguous): the LPR lanes of a row
//    group read a whole row of W_k (M * 4 bytes) as VPL-wide vector loads, so every
//    gathered row is one fully coalesced segment.
//  * Each workgroup stages its row tile's CSR slice (row offsets, columns, values) in LDS
//    once, so a row pass waits on a single global round trip: its gathers.
//  * The diagonal term of 2 At = alpha B + beta I is folded into the coefficient of the
//    stored diagonal entry, so W_k[r] is not read twice.
//  * Probes are never stored: v_j[r] is regenerated from a SplitMix64 counter hash.
//  * Moments are fused into the step's epilogue: v_j^T W_{k+1}, or W_k^T W_{k+1} and
//    W_{k+1}^T W_{k+1} for the Chebyshev product identities (half the products).  Lanes
//    sum their rows in the vector type; from the wave butterfly on everything is FP64: a
//    fixed-order sum over waves, one partial per tile, a fixed-order reduction over tiles
//    (deterministic, no floating-point atomics).
//  * One workgroup per row tile; workgroup ids are remapped so that each of the eight
//    XCDs walks a contiguous range of tiles in order, which keeps the W_k rows that
//    banded patterns reuse (neighbours at +-N, +-N^2) inside that XCD's L2.
#include <algorithm>
#include <type_traits>

#include "ld_internal.h"

#ifndef LD_UNROLL
#define LD_UNROLL 4
#endif
#ifndef LD_NT
#define LD_NT 1
#endif

namespace ld {

// ------------------------------------------------------------------------------------
// small device helpers
// ------------------------------------------------------------------------------------

// SplitMix64 output function at generator state seed + (ctr + 1) * gamma, with
// ctr = (row << 16) | (probe >> 6); bit (probe & 63) is the probe's sign bit.
__device__ __forceinline__ uint64_t probe_word(uint64_t seed, uint64_t row, uint32_t blk) {
  uint64_t ctr = (row << 16) | (uint64_t)blk;
  uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The signs of probes p0 .. p0 + N - 1 (within one 64-probe block) from their probe word.
template <typename VT, int N>
__device__ __forceinline__ void word_signs(uint64_t w, int p0, VT* r) {
  const uint32_t bits = (uint32_t)(w >> (p0 & 63));
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = ((bits >> i) & 1u) ? VT(-1) : VT(1);
}

template <typename VT, int N>
__device__ __forceinline__ void probe_signs(uint64_t seed, int64_t row, int p0, VT* r) {
  word_signs<VT, N>(probe_word(seed, (uint64_t)row, (uint32_t)(p0 >> 6)), p0, r);
}

template <int VALT>
struct Val;
template <>
struct Val<VAL_F64> {
  typedef double T;
  __device__ static double get(const void* p, int64_t t) { return static_cast<const double*>(p)[t]; }
};
template <>
struct Val<VAL_F32> {
  typedef float T;
  __device__ static float get(const void* p, int64_t t) { return static_cast<const float*>(p)[t]; }
};
template <>
struct Val<VAL_BF16> {
  typedef float T;
  __device__ static float get(const void* p, int64_t t) {
    const uint32_t u = static_cast<const uint16_t*>(p)[t];
    return __uint_as_float(u << 16);
  }
};

template <typename VT, int N>
__device__ __forceinline__ void vload(const VT* p, VT* r) {
  if constexpr (N == 1) {
    r[0] = p[0];
  } else {
    typedef VT vec_t __attribute__((ext_vector_type(N)));
    const vec_t x = *reinterpret_cast<const vec_t*>(p);
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = x[i];
  }
}

template <typename VT, int N>
__device__ __forceinline__ void vstore(VT* p, const VT* r) {
  if constexpr (N == 1) {
    p[0] = r[0];
  } else {
    typedef VT vec_t __attribute__((ext_vector_type(N)));
    vec_t x;
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = r[i];
    *reinterpret_cast<vec_t*>(p) = x;
  }
}

// Non-temporal variants for the streamed operands (read or written once per step), so that
// they do not displace the gathered W_k rows from L2 and the Infinity Cache.
template <typename VT, int N>
__device__ __forceinline__ void vload_nt(const VT* p, VT* r) {
#if LD_NT
  if constexpr (N == 1) {
    r[0] = __builtin_nontemporal_load(p);
  } else {
    typedef VT vec_t __attribute__((ext_vector_type(N)));
    const vec_t x = __builtin_nontemporal_load(reinterpret_cast<const vec_t*>(p));
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = x[i];
  }
#else
  vload<VT, N>(p, r);
#endif
}

template <typename VT, int N>
__device__ __forceinline__ void vstore_nt(VT* p, const VT* r) {
#if LD_NT
  if constexpr (N == 1) {
    __builtin_nontemporal_store(r[0], p);
  } else {
    typedef VT vec_t __attribute__((ext_vector_type(N)));
    vec_t x;
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = r[i];
    __builtin_nontemporal_store(x, reinterpret_cast<vec_t*>(p));
  }
#else
  vstore<VT, N>(p, r);
#endif
}

// Physical workgroup id -> logical tile: XCD x (= id mod 8) walks tiles
// [x * per, (x + 1) * per) in dispatch order.
__device__ __forceinline__ int64_t xcd_tile(int64_t ntiles) {
  const int64_t per = (ntiles + 7) >> 3;
  const int64_t b = blockIdx.x;
  return (b & 7) * per + (b >> 3);
}

// Plane-major order (plane > 0 tiles per plane; the launcher checks that plane is a multiple of 8
// and divides ntiles): the tiles form ntiles / plane planes of `plane` consecutive tiles, XCD x
// owns the x-th eighth of every plane and walks its share plane after plane.  On a lattice whose
// plane is the pattern's reach, the rows a tile gathers one plane up or down were read a plane
// earlier by the same XCD and are still in its L2.
__device__ __forceinline__ int64_t block_tile(int64_t ntiles, int64_t plane) {
  if (plane == 0) return xcd_tile(ntiles);
  const int64_t b = blockIdx.x, k = b >> 3, bu = plane >> 3;
  return (k / bu) * plane + (b & 7) * bu + k % bu;
}

constexpr int kBlock = 256;  // 4 waves of 64
constexpr int kWaves = kBlock / 64;
constexpr int kUnroll = LD_UNROLL;  // nonzeros whose gathers are in flight together per row group
#ifndef LD_UNROLL_STEP
#define LD_UNROLL_STEP LD_UNROLL
#endif
constexpr int kUnrollStep = LD_UNROLL_STEP;  // the same for the recurrence step

// ------------------------------------------------------------------------------------
// fused recurrence step
// ------------------------------------------------------------------------------------

// The CSR slice of a row tile (row offsets, column indices, values) is staged in LDS once
// per workgroup: after that a row pass waits on a single global round trip, its gathers.
// Tiles whose slice does not fit (unusually long rows) read the slice from global memory.
template <int VALT>
struct TileCsr {
  typedef typename Val<VALT>::T MV;
  int rp[kStageRows + 1];
  int col[kStageNnz];
  MV val[kStageNnz];
};

// Loads the tile's slice into LDS if it fits; returns whether it did.  All threads call it.
template <int VALT>
__device__ __forceinline__ bool stage_tile(TileCsr<VALT>& T, const int64_t* rp, const int32_t* ci, const void* val,
                                           int64_t row0, int64_t row_end, int64_t& nz0) {
  nz0 = rp[row0];
  const int64_t nz1 = rp[row_end];
  const int nrows = (int)(row_end - row0);
  const bool fits = (nz1 - nz0) <= kStageNnz && nrows <= kStageRows;
  if (fits) {
    // every load of the thread's share in flight before the first LDS write (a loop that wrote each
    // value before loading the next waited one round trip per value)
    constexpr int kRpPer = (kStageRows + 1 + kBlock - 1) / kBlock, kNzPer = (kStageNnz + kBlock - 1) / kBlock;
    const int nnz = (int)(nz1 - nz0);
    int64_t rv[kRpPer];
    int cv[kNzPer];
    typename Val<VALT>::T vv[kNzPer];
#pragma unroll
    for (int q = 0; q < kRpPer; ++q) {
      const int i = (int)threadIdx.x + q * kBlock;
      rv[q] = i <= nrows ? rp[row0 + i] : 0;
    }
#pragma unroll
    for (int q = 0; q < kNzPer; ++q) {
      const int i = (int)threadIdx.x + q * kBlock;
      cv[q] = 0;
      vv[q] = 0;
      if (i < nnz) {
        cv[q] = ci[nz0 + i];
        vv[q] = Val<VALT>::get(val, nz0 + i);
      }
    }
#pragma unroll
    for (int q = 0; q < kRpPer; ++q) {
      const int i = (int)threadIdx.x + q * kBlock;
      if (i <= nrows) T.rp[i] = (int)(rv[q] - nz0);
    }
#pragma unroll
    for (int q = 0; q < kNzPer; ++q) {
      const int i = (int)threadIdx.x + q * kBlock;
      if (i < nnz) {
        T.col[i] = cv[q];
        T.val[i] = vv[q];
      }
    }
  }
  __syncthreads();
  return fits;
}

template <typename VT, int VALT, int VPL, int GSRC, int DSRC, int PSRC, int MU>
__global__ void __launch_bounds__(kBlock) step_kernel(StepLaunch L) {
  typedef typename Val<VALT>::T MV;
  const int64_t tile = block_tile(L.ntiles, L.shape.plane);
  if (tile >= L.ntiles) return;
  const int mat = L.tile_mat ? L.tile_mat[tile] : 0;
  const StepDesc& D = L.descs ? L.descs[mat] : L.d0;
  if (!D.active) return;
  const int64_t row0 = L.tile_row0 ? L.tile_row0[tile] : tile * L.tile_rows;
  const int64_t row_end = min(D.d, row0 + L.tile_rows);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lg = L.shape.lpr_log2;
  const int LPR = 1 << lg;
  const int RPW = 64 >> lg;
  const int sub = lane & (LPR - 1);
  const int grp = lane >> lg;
  const int M = L.M;
  const int tile_probes = LPR * VPL;
  int p0 = (int)blockIdx.y * tile_probes + sub * VPL;
  const bool pact = p0 < M;
  if (!pact) p0 = 0;  // keep addresses valid; results of these lanes are discarded

  const VT ag = (VT)D.ag, bd = (VT)D.bd, cp = (VT)D.cp;
  const VT* __restrict__ G = static_cast<const VT*>(D.G);
  const VT* __restrict__ Dv = static_cast<const VT*>(D.D);
  const VT* P = static_cast<const VT*>(D.P);
  VT* out = static_cast<VT*>(D.out);
  const int64_t* __restrict__ rp = D.row_ptr;
  const int32_t* __restrict__ ci = D.col;

  __shared__ TileCsr<VALT> T;
  int64_t nz0;
  const bool staged = stage_tile<VALT>(T, rp, ci, D.val, row0, row_end, nz0);

  // MU_PROBE: mu = v^T W_{k+1}.  MU_PAIR: mu = W_k^T W_{k+1} and mu2 = W_{k+1}^T W_{k+1}, the two
  // inner products the Chebyshev product identities turn into moments 2k+1 and 2k+2.  A lane
  // sums over its few rows of the tile in the vector type; everything after that is FP64.
  VT mu[VPL], mu2[VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) mu[i] = mu2[i] = VT(0);

  // the row passes, compiled once for the staged slice and once for the global one (one code path
  // each: a runtime choice per entry left loads of both kinds in flight and forced full waits)
  auto row_passes = [&](auto stg) {
    constexpr bool STG = decltype(stg)::value;
    for (int64_t base = row0 + wave * RPW; base < row_end; base += (int64_t)kWaves * RPW) {
      const int64_t row = base + grp;
      const bool has = row < row_end;
      const int lr = (int)(row - row0);
      int64_t s = 0, e = 0;  // entry range relative to nz0
      if (has) {
        if constexpr (STG) {
          s = T.rp[lr];
          e = T.rp[lr + 1];
        } else {
          s = rp[row] - nz0;
          e = rp[row + 1] - nz0;
        }
      }
      const int64_t off = (has ? row : row0) * (int64_t)M + p0;
      // streamed operands first, so their latency overlaps the gathers
      VT pv[VPL];
      if constexpr (PSRC == SRC_BUF) {
        if (has) vload_nt<VT, VPL>(P + off, pv);
      } else if constexpr (PSRC == SRC_HASH) {
        probe_signs<VT, VPL>(D.seed, row, p0, pv);
      }
      VT dv[VPL];
      if constexpr (DSRC == SRC_BUF) {
        if (has) vload<VT, VPL>(Dv + off, dv);
      } else if constexpr (DSRC == SRC_HASH) {
        probe_signs<VT, VPL>(D.seed, row, p0, dv);
      }

      VT acc[VPL];
      VT wk[VPL];  // own row of the gathered operand (MU_PAIR with the diagonal folded in)
  #pragma unroll
      for (int i = 0; i < VPL; ++i) acc[i] = wk[i] = VT(0);
      bool hd = false;
      for (int64_t t = s; t < e; t += kUnrollStep) {
        int cc[kUnrollStep];
        VT aa[kUnrollStep];
        bool ok[kUnrollStep];
  #pragma unroll
        for (int u = 0; u < kUnrollStep; ++u) {
          ok[u] = t + u < e;
          int cu = 0;
          MV vu = MV(0);
          if (ok[u]) {
            if constexpr (STG) {
              cu = T.col[t + u];
              vu = T.val[t + u];
            } else {
              cu = ci[nz0 + t + u];
              vu = Val<VALT>::get(D.val, nz0 + t + u);
            }
          }
          VT a = ag * (VT)vu;
          if constexpr (DSRC == SRC_SAME) {
            if (ok[u] && cu == row) {
              a += bd;
              hd = true;
            }
          }
          aa[u] = a;
          cc[u] = cu;
        }
        VT gg[kUnrollStep][VPL];
  #pragma unroll
        for (int u = 0; u < kUnrollStep; ++u) {
          if (ok[u]) {
            if constexpr (GSRC == SRC_BUF)
              vload<VT, VPL>(G + (int64_t)cc[u] * M + p0, gg[u]);
            else
              probe_signs<VT, VPL>(D.seed, cc[u], p0, gg[u]);
          } else {
  #pragma unroll
            for (int i = 0; i < VPL; ++i) gg[u][i] = VT(0);
          }
        }
  #pragma unroll
        for (int u = 0; u < kUnrollStep; ++u)
  #pragma unroll
          for (int i = 0; i < VPL; ++i) acc[i] = fma(aa[u], gg[u][i], acc[i]);
        if constexpr (MU == MU_PAIR && DSRC == SRC_SAME) {
  #pragma unroll
          for (int u = 0; u < kUnrollStep; ++u)
            if (ok[u] && cc[u] == row)
  #pragma unroll
              for (int i = 0; i < VPL; ++i) wk[i] = gg[u][i];
        }
      }

      if (has) {
        if constexpr (DSRC == SRC_SAME) {
          if (!hd) {  // pattern without a stored diagonal in this row
            VT g[VPL];
            if constexpr (GSRC == SRC_BUF)
              vload<VT, VPL>(G + off, g);
            else
              probe_signs<VT, VPL>(D.seed, row, p0, g);
  #pragma unroll
            for (int i = 0; i < VPL; ++i) {
              acc[i] = fma(bd, g[i], acc[i]);
              wk[i] = g[i];
            }
          }
        } else if constexpr (DSRC != SRC_NONE) {
  #pragma unroll
          for (int i = 0; i < VPL; ++i) wk[i] = dv[i];
  #pragma unroll
          for (int i = 0; i < VPL; ++i) acc[i] = fma(bd, dv[i], acc[i]);
        }
        if constexpr (PSRC != SRC_NONE) {
  #pragma unroll
          for (int i = 0; i < VPL; ++i) acc[i] = fma(cp, pv[i], acc[i]);
        }
        if (pact) {
          vstore_nt<VT, VPL>(out + off, acc);
          if constexpr (MU == MU_PROBE) {
            const uint64_t w = probe_word(D.seed, (uint64_t)row, (uint32_t)(p0 >> 6));
            const uint32_t bits = (uint32_t)(w >> (p0 & 63));
  #pragma unroll
            for (int i = 0; i < VPL; ++i) mu[i] += ((bits >> i) & 1u) ? -acc[i] : acc[i];
          } else if constexpr (MU == MU_PAIR) {
  #pragma unroll
            for (int i = 0; i < VPL; ++i) {
              mu[i] = fma(acc[i], wk[i], mu[i]);
              mu2[i] = fma(acc[i], acc[i], mu2[i]);
            }
          }
        }
      }
    }
  };
  if (staged)
    row_passes(std::integral_constant<bool, true>{});
  else
    row_passes(std::integral_constant<bool, false>{});

  if constexpr (MU != MU_NONE) {
    // fixed-order reduction: wave butterfly, then waves summed in order through LDS that
    // the tile's CSR slice no longer needs
    constexpr int NQ = MU == MU_PAIR ? 2 : 1;
    double m1[VPL], m2[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      m1[i] = (double)mu[i];
      m2[i] = (double)mu2[i];
    }
    for (int o = LPR; o < 64; o <<= 1)
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        m1[i] += __shfl_xor(m1[i], o, 64);
        if constexpr (NQ == 2) m2[i] += __shfl_xor(m2[i], o, 64);
      }
    __syncthreads();
    double* red = reinterpret_cast<double*>(&T);  // [NQ][kWaves][256]
    static_assert(sizeof(TileCsr<VAL_BF16>) >= 2 * kWaves * 256 * sizeof(double), "LDS reuse too small");
    if (grp == 0)
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        red[wave * 256 + sub * VPL + i] = m1[i];
        if constexpr (NQ == 2) red[(kWaves + wave) * 256 + sub * VPL + i] = m2[i];
      }
    __syncthreads();
    for (int q = 0; q < NQ; ++q) {
      double* dst = (q == 0 ? D.mu_part : D.mu_part2) + (tile - D.tile0) * (int64_t)M;
      for (int j = threadIdx.x; j < tile_probes; j += kBlock) {
        const int pj = (int)blockIdx.y * tile_probes + j;
        if (pj < M) {
          double sum = 0.0;
#pragma unroll
          for (int w = 0; w < kWaves; ++w) sum += red[(q * kWaves + w) * 256 + j];
          dst[pj] = sum;
        }
      }
    }
  }
}

// ------------------------------------------------------------------------------------
// adjoint step (gradient): Clenshaw-type backward recurrence fused with the SDDMM
// ------------------------------------------------------------------------------------

// DPP lane exchange within a row of 16 lanes (a VALU operand modifier: no LDS traffic).
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, typename VT>
__device__ __forceinline__ VT dpp_x(VT v) {
  if constexpr (sizeof(VT) == 4)
    return dpp_f32<CTRL>(v);
  else
    return dpp_f64<CTRL>(v);
}

// Two forms of the SDDMM term G_ij += gw * sum_p y1[i,p] w[j,p] for stored (i, j):
//  * general pattern: gather w[j] next to y1[j] (two gathers per nonzero);
//  * symmetric pattern (SYM): row i computes, for each stored (i, j), the value of the
//    TRANSPOSED entry, H_t = gw * sum_p y1[j,p] w[i,p] = G_ji contribution, from the y1[j]
//    row that the SpMM gathers anyway and the row's own w[i]; H is permuted once at the end
//    (entry (i, j) takes H at the index of (j, i)).  One gather per nonzero.
template <typename VT, int VALT, int VPL, bool SPMM, bool WHASH, bool Y2, bool SYM>
// FP32 vectors, single-gather form, FP32 or BF16 values: fit five waves per SIMD (96 VGPRs, no
// spills).  The two-gather form (a second gathered row per nonzero), FP64 values and FP64
// vectors would spill at that budget: those keep the compiler's choice.
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((sizeof(VT) == 4 && SYM && VALT != VAL_F64) ? 5 : 1)))
adjoint_kernel(AdjDesc A, int M, int lpr_log2, int64_t tile_rows, int64_t ntiles, int64_t plane) {
  typedef typename Val<VALT>::T MV;
  const int64_t tile = block_tile(ntiles, plane);
  if (tile >= ntiles) return;
  const int64_t row0 = tile * tile_rows;
  const int64_t row_end = min(A.d, row0 + tile_rows);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int LPR = 1 << lpr_log2;
  const int RPW = 64 >> lpr_log2;
  const int sub = lane & (LPR - 1);
  const int grp = lane >> lpr_log2;
  int p0 = sub * VPL;
  const bool pact = p0 < M;
  if (!pact) p0 = 0;

  const VT ag = (VT)A.ag, bd = (VT)A.bd, cp = (VT)A.cp, cv = (VT)A.cv, gw = (VT)A.gw;
  const VT ck = (VT)A.ck, ce = (VT)A.ce;  // shifted adjoint (two-gather form); zero otherwise
  const VT* __restrict__ Y1 = static_cast<const VT*>(A.Y1);
  const VT* Y2p = static_cast<const VT*>(A.Y2);
  VT* out = static_cast<VT*>(A.out);
  const VT* __restrict__ W = static_cast<const VT*>(A.W);
  VT* __restrict__ Hacc = static_cast<VT*>(A.Gacc);
  const int64_t* __restrict__ rp = A.row_ptr;
  const int32_t* __restrict__ ci = A.col;

  __shared__ TileCsr<VALT> T;
  int64_t nz0;
  const bool staged = stage_tile<VALT>(T, rp, ci, A.val, row0, row_end, nz0);

  double gdiag = 0.0;
  for (int64_t base = row0 + wave * RPW; base < row_end; base += (int64_t)kWaves * RPW) {
    const int64_t row = base + grp;
    const bool has = row < row_end;
    int64_t s = 0, e = 0;  // entry range relative to nz0
    if (has) {
      if (staged) {
        s = T.rp[row - row0];
        e = T.rp[row - row0 + 1];
      } else {
        s = rp[row] - nz0;
        e = rp[row + 1] - nz0;
      }
    }
    const int64_t roff = (has ? row : row0) * (int64_t)M + p0;
    VT yown[VPL], wown[VPL];
    vload<VT, VPL>(Y1 + roff, yown);
    if constexpr (WHASH)
      probe_signs<VT, VPL>(A.seed, has ? row : row0, p0, wown);
    else
      vload_nt<VT, VPL>(W + roff, wown);
    if (!pact || !has) {
#pragma unroll
      for (int i = 0; i < VPL; ++i) yown[i] = wown[i] = VT(0);
    }
    // y_{k+1} of the row (Y1 less the shift ce * w_k) for the SDDMM and the diagonal term; the
    // single-gather form has no shift and keeps no copy (its register budget is tight)
    VT ysd[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) ysd[i] = SYM ? VT(0) : fma(-ce, wown[i], yown[i]);
    VT acc[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) acc[i] = VT(0);
    // the row's streamed seed operands, issued ahead of the gathers so their latency overlaps
    VT xm[VPL], xp[VPL], x2[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) xm[i] = xp[i] = x2[i] = VT(0);
    if constexpr (SPMM) {
      if (has && A.Wm) vload_nt<VT, VPL>(static_cast<const VT*>(A.Wm) + roff, xm);
      if (has && A.Wp) vload_nt<VT, VPL>(static_cast<const VT*>(A.Wp) + roff, xp);
      if constexpr (Y2)
        if (has) vload_nt<VT, VPL>(Y2p + roff, x2);
    }

    for (int64_t t = s; t < e; t += kUnroll) {
      int cc[kUnroll];
      MV vv[kUnroll];
      bool ok[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        ok[u] = t + u < e;
        cc[u] = 0;
        vv[u] = MV(0);
        if (ok[u]) {
          if (staged) {
            cc[u] = T.col[t + u];
            vv[u] = T.val[t + u];
          } else {
            cc[u] = ci[nz0 + t + u];
            vv[u] = Val<VALT>::get(A.val, nz0 + t + u);
          }
        }
      }
      // accumulator slot this lane will own after the transposing reduction (wide groups),
      // read before the gathers so its latency overlaps them
      const bool wide = LPR >= kUnroll;
      const int myu = wide ? (sub / (LPR / kUnroll)) & (kUnroll - 1) : 0;
      const bool writer = wide && (sub & (LPR / kUnroll - 1)) == 0 && t + myu < e;
      VT hold = VT(0);
      if (writer) hold = Hacc[nz0 + t + myu];
      VT dot[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        VT yg[VPL], wg[VPL];
        if (ok[u]) {
          if constexpr (SPMM || SYM) vload<VT, VPL>(Y1 + (int64_t)cc[u] * M + p0, yg);
          if constexpr (!SYM) {
            if constexpr (WHASH)
              probe_signs<VT, VPL>(A.seed, cc[u], p0, wg);
            else
              vload<VT, VPL>(W + (int64_t)cc[u] * M + p0, wg);
          }
        } else {
#pragma unroll
          for (int i = 0; i < VPL; ++i) yg[i] = wg[i] = VT(0);
        }
        if constexpr (SPMM) {
          const VT a = ag * (VT)vv[u];
          if constexpr (SYM) {
#pragma unroll
            for (int i = 0; i < VPL; ++i) acc[i] = fma(a, yg[i], acc[i]);
          } else {  // product on z = Y1 + ck w_k
#pragma unroll
            for (int i = 0; i < VPL; ++i) acc[i] = fma(a, fma(ck, wg[i], yg[i]), acc[i]);
          }
        }
        VT dp = VT(0);
#pragma unroll
        for (int i = 0; i < VPL; ++i) dp = SYM ? fma(yg[i], wown[i], dp) : fma(ysd[i], wg[i], dp);
        dot[u] = dp;
      }
      if (wide) {
        // transposing butterfly: each exchange hands half of the live values to the partner
        // lane, so after log2(kUnroll) exchanges every lane holds one nonzero's partial;
        // the remaining exchanges (offsets below LPR/kUnroll) add up the copies.
        int o = LPR >> 1;
#pragma unroll
        for (int h = kUnroll; h > 1; h >>= 1, o >>= 1) {
          const bool up = (sub & o) != 0;
#pragma unroll
          for (int i = 0; i < h / 2; ++i) {
            const VT send = up ? dot[i] : dot[i + h / 2];
            const VT keep = up ? dot[i + h / 2] : dot[i];
            dot[i] = keep + __shfl_xor(send, o, 64);
          }
        }
        for (; o >= 1; o >>= 1) dot[0] += __shfl_xor(dot[0], o, 64);
        if (writer) Hacc[nz0 + t + myu] = hold + gw * dot[0];
      } else {
        for (int o = 1; o < LPR; o <<= 1)
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) dot[u] += __shfl_xor(dot[u], o, 64);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
          if (ok[u] && sub == (u & (LPR - 1))) Hacc[nz0 + t + u] += gw * dot[u];
      }
    }
    if (has) {
      double dd = 0.0;
#pragma unroll
      for (int i = 0; i < VPL; ++i) dd += (double)(SYM ? yown[i] : ysd[i]) * (double)wown[i];
      gdiag += (double)A.gw * dd;
      if constexpr (SPMM) {
        VT vv[VPL];
        probe_signs<VT, VPL>(A.seed, row, p0, vv);
        const VT cw = (VT)A.cw;
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
          VT o = fma(bd, SYM ? yown[i] : fma(ck, wown[i], yown[i]), acc[i]);
          o = fma(cw, wown[i], o);
          acc[i] = fma(cv, vv[i], o);
        }
        if (A.Wm) {
          const VT c = (VT)A.cwm;
#pragma unroll
          for (int i = 0; i < VPL; ++i) acc[i] = fma(c, xm[i], acc[i]);
        }
        if (A.Wp) {
          const VT c = (VT)A.cwp;
#pragma unroll
          for (int i = 0; i < VPL; ++i) acc[i] = fma(c, xp[i], acc[i]);
        }
        if constexpr (Y2) {
#pragma unroll
          for (int i = 0; i < VPL; ++i) acc[i] = fma(cp, x2[i], acc[i]);
        }
        if (pact) vstore_nt<VT, VPL>(out + roff, acc);
      }
    }
  }
  // tile partial of the diagonal term (fixed-order block reduction)
  __shared__ double sg[kWaves];
  for (int o = 1; o < 64; o <<= 1) gdiag += __shfl_xor(gdiag, o, 64);
  if (lane == 0) sg[wave] = gdiag;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < kWaves; ++w) sum += sg[w];
    A.gdiag_part[tile] += sum;
  }
}

// ------------------------------------------------------------------------------------
// shifted adjoint step on vector tiles staged in LDS (stencil patterns)
// ------------------------------------------------------------------------------------

// Sum over the LPR consecutive lanes of a row group (LPR a power of two), every lane receiving
// the total: exchanges within quads, then the mirrored half-row and row, then (LPR >= 32) shuffles.
// N independent sums at once: one uniform branch per exchange level for all of them, and the N
// exchanges of a level back to back.
template <typename VT, int N>
__device__ __forceinline__ void row_sums(VT (&v)[N], int LPR) {
  if (LPR >= 2)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_x<0xB1>(v[k]);   // quad_perm [1,0,3,2]
  if (LPR >= 4)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_x<0x4E>(v[k]);   // quad_perm [2,3,0,1]
  if (LPR >= 8)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_x<0x141>(v[k]);  // row_half_mirror: lane i of 8 <- lane 7 - i
  if (LPR >= 16)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += dpp_x<0x140>(v[k]);  // row_mirror: lane i of 16 <- lane 15 - i
  for (int o = 16; o < LPR; o <<= 1)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += __shfl_xor(v[k], o, 64);
}

// Packed entry of the stencil layout: LDS slot of the column and the value.
template <int VALT>
struct StencilEnt;
template <>
struct StencilEnt<VAL_BF16> {
  typedef uint32_t T;  // value bits << 16 | slot
  __device__ static void dec(const T& w, int& lc, float& v) {
    lc = (int)(w & 0xFFFFu);
    v = __uint_as_float(w & 0xFFFF0000u);
  }
  __device__ static void get(const void* p, int64_t i, int& lc, float& v) {
    dec(static_cast<const T*>(p)[i], lc, v);
  }
};
template <>
struct StencilEnt<VAL_F32> {
  typedef uint2 T;  // (slot, value bits)
  __device__ static void dec(const T& w, int& lc, float& v) {
    lc = (int)w.x;
    v = __uint_as_float(w.y);
  }
  __device__ static void get(const void* p, int64_t i, int& lc, float& v) {
    dec(static_cast<const T*>(p)[i], lc, v);
  }
};
template <>
struct StencilEnt<VAL_F64> {
  typedef uint4 T;  // (slot, 0, value bits low, high)
  __device__ static void dec(const T& w, int& lc, double& v) {
    lc = (int)w.x;
    v = __hiloint2double((int)w.w, (int)w.z);
  }
  __device__ static void get(const void* p, int64_t i, int& lc, double& v) {
    dec(static_cast<const T*>(p)[i], lc, v);
  }
};

constexpr int kHaloPasses = 3;  // halo rows per thread of a staged tile: the plan keeps nofs <= 3 TR

// Offset (from the tile's first row) of halo index j: run q holds indices [run_base[q], run_base[q + 1]).
__device__ __forceinline__ int halo_offset(const StencilDesc& S, int j) {
  int off = j + S.run_delta[0];
#pragma unroll
  for (int q = 1; q < kStencilRuns; ++q)
    if (q < S.nruns && j >= S.run_base[q]) off = j + S.run_delta[q];
  return off;
}

// Staged rows that are probe signs (W_0 = V) go to LDS as probe words: one hash per staged row
// and 64-probe block, spread over the block's threads, instead of one per row in every lane that
// stages it.  Word q * nblk + b holds block b of staged row q (own rows first, then the halo);
// rows outside the matrix get 0 (no entry reaches them).
__device__ __forceinline__ void stage_probe_words(uint64_t* wd, uint64_t seed, const StencilDesc& S, int64_t sr0,
                                                  int TR, int nblk_log2, int64_t d) {
  const int n = (TR + S.nofs) << nblk_log2;
  for (int i = threadIdx.x; i < n; i += kBlock) {
    const int q = i >> nblk_log2, b = i & ((1 << nblk_log2) - 1);
    const int64_t r = sr0 + (q < TR ? q : halo_offset(S, q - TR));
    wd[i] = (r >= 0 && r < d) ? probe_word(seed, (uint64_t)r, (uint32_t)b) : 0ull;
  }
}

// The shifted adjoint gathers rows of both y_{k+1} and w_k at every stored entry.  On a stencil
// pattern the rows a tile's entries reach are its own rows and r0 + ofs[j] for a short offset list
// (a few runs, passed by value), so the block copies those rows of both operands into LDS once, all
// loads in flight together and none depending on another, and every entry reads them from there: a
// vector row crosses the cache hierarchy (TR + nofs) / TR times per step instead of once per entry
// that reaches it.  Each row's KK packed entry slots and accumulators (arithmetic addresses in the
// padded layout) load together with the staged rows; after the barrier the row forms the product
// on z = y_{k+1} + ck w_k and the SDDMM dots, sums each dot over the row's lanes with DPP
// exchanges, and writes the accumulators back.  The diagonal entries' accumulators carry
// d Gamma / d shift, summed after the steps.  SD: the closing SDDMM term y_1 w_0^T alone, w_0 the
// probe block (nothing staged but the probe words of the own and offset rows), no product.
template <typename VT, int VALT, int VPL, bool Y2, int KK, bool SD = false>
__global__ void __launch_bounds__(kBlock) adjoint_stencil_kernel(AdjDesc A, StencilDesc S, int M, int lpr_log2,
                                                                 int64_t ntiles) {
  typedef typename Val<VALT>::T MV;
  const int64_t tile = xcd_tile(ntiles);
  if (tile >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int LPR = 1 << lpr_log2;
  const int RPW = 64 >> lpr_log2;
  const int TR = kWaves * RPW;  // rows of the tile: one per lane group
  const int sub = lane & (LPR - 1);
  const int grp = lane >> lpr_log2;
  const int tp = LPR * VPL;  // elements per staged row
  const int64_t row0 = tile * TR;
  const int nown = (int)min((int64_t)TR, A.d - row0);
  int p0 = sub * VPL;
  const bool pact = p0 < M;
  if (!pact) p0 = 0;
  const VT* __restrict__ Y1 = static_cast<const VT*>(A.Y1);
  const VT* __restrict__ W = static_cast<const VT*>(A.W);

  extern __shared__ __align__(16) unsigned char ld_stencil_smem[];
  VT* Ys = reinterpret_cast<VT*>(ld_stencil_smem);
  VT* Ws = Ys + (TR + S.nofs) * tp;
  uint64_t* Wd = reinterpret_cast<uint64_t*>(ld_stencil_smem);  // SD: probe words of w_0 = V
  const int nblk_log2 = tp > 128 ? 2 : (tp > 64 ? 1 : 0);

  const int lr = wave * RPW + grp;
  const bool has = lr < nown;
  const int64_t row = row0 + (has ? lr : 0);
  const int64_t roff = row * (int64_t)M + p0;

  // ---- staging: own rows and the offset rows, every load independent of the others ----
  VT yown[VPL], wown[VPL], x2[VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) yown[i] = wown[i] = x2[i] = VT(0);
  if (has && pact) {
    vload<VT, VPL>(Y1 + roff, yown);
    if constexpr (!SD) vload<VT, VPL>(W + roff, wown);
    if constexpr (Y2) vload_nt<VT, VPL>(static_cast<const VT*>(A.Y2) + roff, x2);
  }
  // Ys holds the product's operand z = y_{k+1} + ck w_k of every staged row, Ws holds w_k
  const VT ck = (VT)A.ck;
  // every halo row this thread stages (at most kHaloPasses: the plan keeps nofs <= kHaloPasses TR)
  // loaded first, all in flight together, then written to LDS
  VT hy[kHaloPasses][VPL], hw[kHaloPasses][VPL];
#pragma unroll
  for (int h = 0; h < kHaloPasses; ++h) {
    const int j = lr + h * TR;
#pragma unroll
    for (int i = 0; i < VPL; ++i) hy[h][i] = hw[h][i] = VT(0);
    const int64_t r = row0 + halo_offset(S, j);
    if constexpr (!SD) {
      if (j < S.nofs && r >= 0 && r < A.d && pact) {
        vload<VT, VPL>(Y1 + r * M + p0, hy[h]);
        vload<VT, VPL>(W + r * M + p0, hw[h]);
      }
    }
  }
  // the row's entry slots and accumulators, in flight with the staged rows (loaded after the LDS
  // writes they would cost one more round trip per block); rows past the end read the tile's first
  // row's slots (valid memory, results dropped), so that the KK consecutive loads carry no
  // predicate and merge into wide ones
  const int64_t e0 = (tile * TR + (has ? lr : 0)) * (int64_t)KK;
  VT* __restrict__ hacc = static_cast<VT*>(S.hacc) + e0;
  int lc[KK];
  VT va[KK], h[KK];
#pragma unroll
  for (int k = 0; k < KK; ++k) {
    MV v;
    StencilEnt<VALT>::get(S.ent, e0 + k, lc[k], v);
    va[k] = (VT)v;
    h[k] = hacc[k];
  }
  VT zown[VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) zown[i] = fma(ck, wown[i], yown[i]);
  if constexpr (SD) {
    stage_probe_words(Wd, A.seed, S, row0, TR, nblk_log2, A.d);
  } else {
#pragma unroll
    for (int h = 0; h < kHaloPasses; ++h) {
      const int j = lr + h * TR;
      if (j < S.nofs) {
#pragma unroll
        for (int i = 0; i < VPL; ++i) hy[h][i] = fma(ck, hw[h][i], hy[h][i]);
        vstore<VT, VPL>(Ys + (TR + j) * tp + sub * VPL, hy[h]);
        vstore<VT, VPL>(Ws + (TR + j) * tp + sub * VPL, hw[h]);
      }
    }
    vstore<VT, VPL>(Ys + lr * tp + sub * VPL, zown);
    vstore<VT, VPL>(Ws + lr * tp + sub * VPL, wown);
  }

  __syncthreads();
  if constexpr (SD) {
    if (has && pact) word_signs<VT, VPL>(Wd[(lr << nblk_log2) + (p0 >> 6)], p0, wown);
  }

  const VT ag = (VT)A.ag, ce = (VT)A.ce, gw = (VT)A.gw;
  VT ysd[VPL], acc[VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) {
    ysd[i] = fma(-ce, wown[i], yown[i]);
    acc[i] = VT(0);
  }
  VT dp[KK];
#pragma unroll
  for (int k = 0; k < KK; ++k) {
    VT zg[VPL], wg[VPL];
    if constexpr (SD) {
      word_signs<VT, VPL>(Wd[(lc[k] << nblk_log2) + (p0 >> 6)], p0, wg);
    } else {
      vload<VT, VPL>(Ys + lc[k] * tp + sub * VPL, zg);
      vload<VT, VPL>(Ws + lc[k] * tp + sub * VPL, wg);
    }
    const VT a = ag * va[k];
    dp[k] = VT(0);
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      if constexpr (!SD) acc[i] = fma(a, zg[i], acc[i]);
      dp[k] = fma(ysd[i], wg[i], dp[k]);
    }
  }
  row_sums<VT, KK>(dp, LPR);
#pragma unroll
  for (int k = 0; k < KK; ++k) h[k] = fma(gw, dp[k], h[k]);
  if (!has) return;
  // every lane of the row holds the sums: lane 0 writes the KK slots back (padding too: never read out)
  if (sub == 0)
#pragma unroll
    for (int k = 0; k < KK; ++k) hacc[k] = h[k];
  if constexpr (SD) return;
  const VT bd = (VT)A.bd, cp = (VT)A.cp, cw = (VT)A.cw;
#pragma unroll
  for (int i = 0; i < VPL; ++i) {
    VT o = fma(bd, zown[i], acc[i]);
    o = fma(cw, wown[i], o);
    acc[i] = Y2 ? fma(cp, x2[i], o) : o;
  }
  if (A.cv != 0.0) {  // the probe term (absent in the shifted form's steps)
    VT pv[VPL];
    probe_signs<VT, VPL>(A.seed, row, p0, pv);
    const VT cv = (VT)A.cv;
#pragma unroll
    for (int i = 0; i < VPL; ++i) acc[i] = fma(cv, pv[i], acc[i]);
  }
  if (pact) vstore_nt<VT, VPL>(static_cast<VT*>(A.out) + roff, acc);
}

// Recurrence step on stencil tiles: the step kernel's W_{k+1} = alpha B W_k + beta W_k + cp P with its
// moment partials, where W_k's rows reach each entry from LDS.  A block covers one row tile of the
// pass shape (so that its moment partials keep the step kernel's [tile][M] layout) as a sequence of
// stencil tiles of one row pass each: stage the own and offset rows of W_k (the rows' packed entries
// loaded with them), barrier, one row per lane group, barrier.  FP32 vectors, FP32 or BF16 values,
// a single probe tile.  W_k comes from a buffer or (k = 0) from the probe hash, for own and offset
// rows alike.
template <int VALT, int VPL, int GSRC, int PSRC, int MU, int KK>
__global__ void __launch_bounds__(kBlock) step_stencil_kernel(StepLaunch L, StencilDesc S) {
  typedef float VT;
  typedef typename Val<VALT>::T MV;
  const int64_t tile = xcd_tile(L.ntiles);
  if (tile >= L.ntiles) return;
  const StepDesc& D = L.d0;
  const int64_t row0 = tile * L.tile_rows;
  const int64_t row_end = min(D.d, row0 + L.tile_rows);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lg = L.shape.lpr_log2;
  const int LPR = 1 << lg;
  const int RPW = 64 >> lg;
  const int TR = kWaves * RPW;
  const int sub = lane & (LPR - 1);
  const int grp = lane >> lg;
  const int M = L.M;
  const int tp = LPR * VPL;
  int p0 = sub * VPL;
  const bool pact = p0 < M;
  if (!pact) p0 = 0;
  const VT ag = (VT)D.ag, bd = (VT)D.bd, cp = (VT)D.cp;
  const VT* __restrict__ G = static_cast<const VT*>(D.G);
  const VT* P = static_cast<const VT*>(D.P);
  VT* out = static_cast<VT*>(D.out);

  extern __shared__ __align__(16) unsigned char ld_step_smem[];
  VT* Ws = reinterpret_cast<VT*>(ld_step_smem);
  uint64_t* Wd = reinterpret_cast<uint64_t*>(ld_step_smem);  // probe words (W_0 from the hash)
  const int nblk_log2 = tp > 128 ? 2 : (tp > 64 ? 1 : 0);       // 64-probe blocks of the tile's probes
  const int lr = wave * RPW + grp;

  VT mu[VPL], mu2[VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) mu[i] = mu2[i] = VT(0);

  for (int64_t sr0 = row0; sr0 < row_end; sr0 += TR) {
    const int nown = (int)min((int64_t)TR, row_end - sr0);
    const bool has = lr < nown;
    const int64_t row = sr0 + (has ? lr : 0);
    const int64_t roff = row * (int64_t)M + p0;
    VT wown[VPL], pv[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) wown[i] = pv[i] = VT(0);
    if constexpr (GSRC != SRC_HASH) {
      if (has && pact) vload<VT, VPL>(G + roff, wown);
    }
    if constexpr (PSRC == SRC_BUF) {
      if (has && pact) vload_nt<VT, VPL>(P + roff, pv);
    } else if constexpr (PSRC == SRC_HASH) {
      probe_signs<VT, VPL>(D.seed, row, p0, pv);
    }
    const int64_t e0 = row * (int64_t)KK;  // slot (tile * TR + lr) * KK of the padded layout
    typedef typename StencilEnt<VALT>::T ET;
    ET ew[KK];  // packed entries: loaded with the rows, decoded where they are used
    if constexpr (GSRC == SRC_HASH) {
      // W_0 = V: the packed entries in flight while the block hashes the staged rows' probe words
#pragma unroll
      for (int k = 0; k < KK; ++k) ew[k] = static_cast<const ET*>(S.ent)[e0 + k];
      stage_probe_words(Wd, D.seed, S, sr0, TR, nblk_log2, D.d);
    } else {
      VT hw[kHaloPasses][VPL];
#pragma unroll
      for (int h = 0; h < kHaloPasses; ++h) {
        const int j = lr + h * TR;
#pragma unroll
        for (int i = 0; i < VPL; ++i) hw[h][i] = VT(0);
        const int64_t r = sr0 + halo_offset(S, j);
        if (j < S.nofs && r >= 0 && r < D.d && pact) vload<VT, VPL>(G + r * M + p0, hw[h]);
      }
#pragma unroll
      for (int k = 0; k < KK; ++k) ew[k] = static_cast<const ET*>(S.ent)[e0 + k];
#pragma unroll
      for (int h = 0; h < kHaloPasses; ++h) {
        const int j = lr + h * TR;
        if (j < S.nofs) vstore<VT, VPL>(Ws + (TR + j) * tp + sub * VPL, hw[h]);
      }
      vstore<VT, VPL>(Ws + lr * tp + sub * VPL, wown);
    }
    __syncthreads();
    if constexpr (GSRC == SRC_HASH) {
      if (has && pact) word_signs<VT, VPL>(Wd[(lr << nblk_log2) + (p0 >> 6)], p0, wown);
    }
    VT acc[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) acc[i] = bd * wown[i];
#pragma unroll
    for (int k = 0; k < KK; ++k) {
      int lck;
      MV vk;
      StencilEnt<VALT>::dec(ew[k], lck, vk);
      VT g[VPL];
      if constexpr (GSRC == SRC_HASH)
        word_signs<VT, VPL>(Wd[(lck << nblk_log2) + (p0 >> 6)], p0, g);
      else
        vload<VT, VPL>(Ws + lck * tp + sub * VPL, g);
      const VT a = ag * (VT)vk;
#pragma unroll
      for (int i = 0; i < VPL; ++i) acc[i] = fma(a, g[i], acc[i]);
    }
    if constexpr (PSRC != SRC_NONE) {
#pragma unroll
      for (int i = 0; i < VPL; ++i) acc[i] = fma(cp, pv[i], acc[i]);
    }
    if (has && pact) {
      vstore_nt<VT, VPL>(out + roff, acc);
      if constexpr (MU == MU_PAIR) {
#pragma unroll
        for (int i = 0; i < VPL; ++i) {
          mu[i] = fma(acc[i], wown[i], mu[i]);
          mu2[i] = fma(acc[i], acc[i], mu2[i]);
        }
      } else if constexpr (MU == MU_PROBE) {
        const uint64_t w = probe_word(D.seed, (uint64_t)row, (uint32_t)(p0 >> 6));
        const uint32_t bits = (uint32_t)(w >> (p0 & 63));
#pragma unroll
        for (int i = 0; i < VPL; ++i) mu[i] += ((bits >> i) & 1u) ? -acc[i] : acc[i];
      }
    }
    __syncthreads();  // the next stencil tile overwrites the staged rows
  }

  if constexpr (MU != MU_NONE) {
    constexpr int NQ = MU == MU_PAIR ? 2 : 1;
    // fixed-order reduction as in the step kernel: wave butterfly, then waves summed in order
    double m1[VPL], m2[VPL];
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      m1[i] = (double)mu[i];
      m2[i] = (double)mu2[i];
    }
    for (int o = LPR; o < 64; o <<= 1)
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        m1[i] += __shfl_xor(m1[i], o, 64);
        if constexpr (NQ == 2) m2[i] += __shfl_xor(m2[i], o, 64);
      }
    double* red = reinterpret_cast<double*>(ld_step_smem);  // [NQ][kWaves][256] (the launch sizes it)
    if (grp == 0)
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        red[wave * 256 + sub * VPL + i] = m1[i];
        if constexpr (NQ == 2) red[(kWaves + wave) * 256 + sub * VPL + i] = m2[i];
      }
    __syncthreads();
    for (int q = 0; q < NQ; ++q) {
      double* dst = (q == 0 ? D.mu_part : D.mu_part2) + (tile - D.tile0) * (int64_t)M;
      for (int j = threadIdx.x; j < tp; j += kBlock)
        if (j < M) {
          double sum = 0.0;
#pragma unroll
          for (int w = 0; w < kWaves; ++w) sum += red[(q * kWaves + w) * 256 + j];
          dst[j] = sum;
        }
    }
  }
}

template <int VALT>
__global__ void __launch_bounds__(256) stencil_pack_kernel(const void* val, const int32_t* emap, const uint16_t* lcol,
                                                           int64_t n, void* ent) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int32_t e = emap[i];
    const uint32_t lc = lcol[i];
    if constexpr (VALT == VAL_BF16) {
      const uint32_t vb = e >= 0 ? static_cast<const uint16_t*>(val)[e] : 0u;
      static_cast<uint32_t*>(ent)[i] = (vb << 16) | lc;
    } else if constexpr (VALT == VAL_F32) {
      const float v = e >= 0 ? static_cast<const float*>(val)[e] : 0.f;
      static_cast<uint2*>(ent)[i] = make_uint2(lc, __float_as_uint(v));
    } else {
      const double v = e >= 0 ? static_cast<const double*>(val)[e] : 0.0;
      static_cast<uint4*>(ent)[i] = make_uint4(lc, 0u, (uint32_t)__double2loint(v), (uint32_t)__double2hiint(v));
    }
  }
}

template <typename VT>
__global__ void __launch_bounds__(256) stencil_unpack_kernel(const VT* hacc, const int32_t* emap, int64_t n, VT* acc) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int32_t e = emap[i];
    if (e >= 0) acc[e] += hacc[i];
  }
}

// 256 blocks, block b: rows [b * chunk, (b + 1) * chunk), threads strided, then a fixed-order tree.
template <typename VT>
__global__ void __launch_bounds__(256) stencil_diag_sum_kernel(const VT* hacc, const int64_t* dslot, int64_t d,
                                                               double* part) {
  __shared__ double red[256];
  const int64_t chunk = (d + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(d, r0 + chunk);
  double sum = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) sum += (double)hacc[dslot[i]];
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] += red[0];
}

// perm[t] = index of the entry (col[t], row(t)); flag set when some transposed entry is missing.
// One thread per stored entry: its row by binary search over row_ptr, then a binary search of
// row col[t] (columns are usually sorted) with a linear scan as the fallback for rows that are
// not, so that a lookup in a long row costs log(length).
__global__ void __launch_bounds__(256) transpose_index_kernel(const int64_t* row_ptr, const int32_t* col, int64_t d,
                                                              int64_t nnz, int64_t* perm, int* missing) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * 256) {
    int64_t lo = 0, hi = d;  // row_ptr[lo] <= t < row_ptr[hi]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (row_ptr[mid] <= t)
        lo = mid;
      else
        hi = mid;
    }
    const int64_t r = lo;
    const int64_t j = col[t];
    const int64_t u0 = row_ptr[j], u1 = row_ptr[j + 1];
    lo = u0;
    hi = u1;
    while (lo < hi) {  // first u with col[u] >= r
      const int64_t mid = (lo + hi) >> 1;
      if (col[mid] < r)
        lo = mid + 1;
      else
        hi = mid;
    }
    int64_t found = (lo < u1 && col[lo] == r) ? lo : -1;
    for (int64_t u = u0; found < 0 && u < u1; ++u)
      if (col[u] == r) found = u;
    perm[t] = found;
    if (found < 0) atomicOr(missing, 1);
  }
}

// hist[b] += number of stored entries (i, j) with bit_length(|i - j|) = b (b = 0: the diagonal):
// how far from its row each entry reaches, which decides the adjoint's form.  Block-local counts
// in LDS, one atomic per bin per block (integer atomics: the result does not depend on order).
__global__ void __launch_bounds__(256) distance_hist_kernel(const int64_t* row_ptr, const int32_t* col, int64_t d,
                                                            int64_t nnz, unsigned long long* hist) {
  __shared__ unsigned int h[kDistBins];
  for (int i = threadIdx.x; i < kDistBins; i += 256) h[i] = 0u;
  __syncthreads();
  // rows of this block's share of entries: walk rows in a grid-stride loop
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < d; r += (int64_t)gridDim.x * 256) {
    for (int64_t t = row_ptr[r]; t < row_ptr[r + 1]; ++t) {
      const int64_t dist = col[t] > r ? col[t] - r : r - col[t];
      const int b = dist == 0 ? 0 : 64 - __clzll((unsigned long long)dist);
      atomicAdd(&h[b], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kDistBins; i += 256)
    if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

// out[0] = max(out[0], max |i - j| over stored entries); with band > 0 also out[1] += the entries with
// min(|i - j|, | |i - j| - band |) > band / 16: those that sit neither near the diagonal nor one
// plane of `band` rows away.
__global__ void __launch_bounds__(256) plane_fit_kernel(const int64_t* row_ptr, const int32_t* col, int64_t d,
                                                        int64_t band, unsigned long long* out) {
  __shared__ unsigned long long blk[2];
  if (threadIdx.x < 2) blk[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long mx = 0, off = 0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < d; r += (int64_t)gridDim.x * 256) {
    for (int64_t t = row_ptr[r]; t < row_ptr[r + 1]; ++t) {
      const int64_t dist = col[t] > r ? col[t] - r : r - col[t];
      mx = max(mx, (unsigned long long)dist);
      if (band > 0) {
        const int64_t to_plane = dist > band ? dist - band : band - dist;
        off += (unsigned long long)(min(dist, to_plane) * 16 > band);
      }
    }
  }
  if (mx) atomicMax(&blk[0], mx);
  if (off) atomicAdd(&blk[1], off);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (blk[0]) atomicMax(&out[0], blk[0]);
    if (blk[1]) atomicAdd(&out[1], blk[1]);
  }
}

// out[t] = scale * (a[t] + a[perm[t]]) / 2: the derivative along symmetric perturbations from
// per-entry accumulators (either orientation, since the mean is symmetric in the pair).
template <typename TA, typename TO>
__global__ void __launch_bounds__(256) sym_scale_kernel(const TA* a, const int64_t* perm, int64_t n, double scale,
                                                        TO* out) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256)
    out[t] = (TO)(0.5 * ((double)a[t] + (double)a[perm[t]]) * scale);
}

// ------------------------------------------------------------------------------------
// reductions and utilities
// ------------------------------------------------------------------------------------

// Stage 1 of the moment reduction: block (k, probe group, chunk) sums tiles
// [chunk * per, (chunk + 1) * per) with 16 slices x 4 independent accumulators per probe,
// combined in a fixed order.  Stage 2 adds the chunks in order.  Deterministic.
constexpr int kRedChunks = 16;

__global__ void __launch_bounds__(1024) reduce_moments_stage1(const double* part, int64_t ntiles, int M,
                                                              int64_t kstride, double* tmp) {
  const int kk = blockIdx.x;
  const int j = blockIdx.y * 64 + (threadIdx.x & 63);
  const int q = threadIdx.x >> 6;  // 16 slices
  const int64_t per = (ntiles + kRedChunks - 1) / kRedChunks;
  const int64_t t0 = (int64_t)blockIdx.z * per;
  const int64_t t1 = min(ntiles, t0 + per);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (j < M) {
    const double* p = part + (int64_t)kk * kstride + j;
    int64_t t = t0 + q;
    for (; t + 48 < t1; t += 64) {
      a0 += p[t * M];
      a1 += p[(t + 16) * M];
      a2 += p[(t + 32) * M];
      a3 += p[(t + 48) * M];
    }
    for (; t < t1; t += 16) a0 += p[t * M];
  }
  __shared__ double sh[16][64];
  sh[q][threadIdx.x & 63] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  if (q == 0 && j < M) {
    double sum = 0.0;
    for (int r = 0; r < 16; ++r) sum += sh[r][threadIdx.x & 63];
    tmp[((int64_t)kk * kRedChunks + blockIdx.z) * M + j] = sum;
  }
}

__global__ void __launch_bounds__(256) reduce_moments_stage2(const double* tmp, int M, int k_lo, int nk, double* mu,
                                                             int ldmu) {
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < (int64_t)nk * M; x += (int64_t)gridDim.x * 256) {
    const int kk = (int)(x / M);
    const int j = (int)(x - (int64_t)kk * M);
    double sum = 0.0;
    for (int c = 0; c < kRedChunks; ++c) sum += tmp[((int64_t)kk * kRedChunks + c) * M + j];
    mu[(int64_t)j * ldmu + k_lo + kk] = sum;
  }
}

__global__ void __launch_bounds__(1024) reduce_batched_kernel(const double* part, const int64_t* tile_range,
                                                              const int* nvec, int M, int64_t kstride, double* mu,
                                                              int kmax) {
  const int i = blockIdx.x;        // matrix
  const int k = 1 + blockIdx.y;    // degree
  const int j = blockIdx.z * 64 + (threadIdx.x & 63);
  const int q = threadIdx.x >> 6;
  if (k > nvec[i]) return;
  double s = 0.0;
  if (j < M) {
    const double* p = part + (int64_t)(k - 1) * kstride + j;
    for (int64_t t = tile_range[2 * i] + q; t < tile_range[2 * i + 1]; t += 16) s += p[t * M];
  }
  __shared__ double sh[16][64];
  sh[q][threadIdx.x & 63] = s;
  __syncthreads();
  if (q == 0 && j < M) {
    double sum = 0.0;
    for (int r = 0; r < 16; ++r) sum += sh[r][threadIdx.x & 63];
    mu[((int64_t)i * M + j) * (kmax + 1) + k] = sum;
  }
}

__global__ void __launch_bounds__(1024) sum_doubles_kernel(const double* x, int64_t n, double* out) {
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += 1024) s += x[t];
  __shared__ double sh[1024];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

template <int VALT>
__global__ void __launch_bounds__(256) gershgorin_kernel(const int64_t* row_ptr, const int32_t* col, const void* val,
                                                         double shift, int64_t d, double* lo_part, double* hi_part) {
  double lo = __builtin_inf(), hi = -__builtin_inf();
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < d; r += (int64_t)gridDim.x * 256) {
    double diag = 0.0, off = 0.0;
    for (int64_t t = row_ptr[r]; t < row_ptr[r + 1]; ++t) {
      const double v = (double)Val<VALT>::get(val, t);
      if (col[t] == r)
        diag += v;
      else
        off += fabs(v);
    }
    diag += shift;
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

// --- Lanczos helpers (FP64 vectors) ---

__global__ void __launch_bounds__(256) dot_partials_kernel(const double* x, const double* y, int64_t n, double* part) {
  double s = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) s += x[t] * y[t];
  __shared__ double sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) probes_kernel(uint64_t seed, int M, int64_t rows, int8_t* out) {
  const int64_t total = rows * (int64_t)M;
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < total; x += (int64_t)gridDim.x * 256) {
    const int64_t r = x / M;
    const int j = (int)(x - r * M);
    const uint64_t w = probe_word(seed, (uint64_t)r, (uint32_t)(j >> 6));
    out[x] = ((w >> (j & 63)) & 1u) ? (int8_t)-1 : (int8_t)1;
  }
}

// --- transpose (setup for Algorithm 2) ---

__global__ void __launch_bounds__(256) count_cols_kernel(const int32_t* col, int64_t nnz, int64_t* cnt) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < nnz; t += (int64_t)gridDim.x * 256)
    atomicAdd(reinterpret_cast<unsigned long long*>(cnt + col[t]), 1ull);
}

// exclusive scan in three passes: block sums, scan of block sums (one block), add-back
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 8;  // per thread
constexpr int64_t kScanTile = (int64_t)kScanBlock * kScanItems;

__device__ int64_t block_exclusive_scan(int64_t x, int64_t* sh, int64_t* total) {
  sh[threadIdx.x] = x;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int64_t y = ((int)threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += y;
    __syncthreads();
  }
  const int64_t incl = sh[threadIdx.x];
  *total = sh[kScanBlock - 1];
  __syncthreads();
  return incl - x;
}

__global__ void __launch_bounds__(kScanBlock) scan_tiles_kernel(const int64_t* in, int64_t n, int64_t* out,
                                                                int64_t* tile_sums) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t local = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    local += v[i];
  }
  int64_t total;
  int64_t run = block_exclusive_scan(local, sh, &total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) scan_sums_kernel(int64_t* sums, int64_t nt) {
  __shared__ int64_t sh[kScanBlock];
  int64_t carry = 0;
  for (int64_t base = 0; base < nt; base += kScanBlock) {
    const int64_t i = base + threadIdx.x;
    const int64_t x = i < nt ? sums[i] : 0;
    int64_t total;
    const int64_t ex = block_exclusive_scan(x, sh, &total);
    if (i < nt) sums[i] = carry + ex;
    carry += total;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) scan_add_kernel(int64_t* out, int64_t n, const int64_t* sums) {
  for (int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x; x < n; x += (int64_t)gridDim.x * 256)
    out[x] += sums[x / kScanTile];
}

// Row r of C scatters its entries into the rows of C^T at per-column cursors.  val_t and src_t are
// nullable: without values only the pattern is built; src_t[pos] = t records which entry of C
// landed at pos (the map from C^T's entries back to C's).
template <int VALT>
__global__ void __launch_bounds__(256) scatter_t_kernel(const int64_t* row_ptr, const int32_t* col, const void* val,
                                                        int64_t d, int64_t* cursor, int32_t* col_t, void* val_t,
                                                        int64_t* src_t) {
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < d; r += (int64_t)gridDim.x * 256) {
    for (int64_t t = row_ptr[r]; t < row_ptr[r + 1]; ++t) {
      const int c = col[t];
      const int64_t pos = (int64_t)atomicAdd(reinterpret_cast<unsigned long long*>(cursor + c), 1ull);
      col_t[pos] = (int32_t)r;
      if (src_t) src_t[pos] = t;
      if (val_t) {
        if constexpr (VALT == VAL_F64)
          static_cast<double*>(val_t)[pos] = static_cast<const double*>(val)[t];
        else if constexpr (VALT == VAL_F32)
          static_cast<float*>(val_t)[pos] = static_cast<const float*>(val)[t];
        else
          static_cast<uint16_t*>(val_t)[pos] = static_cast<const uint16_t*>(val)[t];
      }
    }
  }
}

// Sorts every row by column (the scatter's order within a row depends on timing); values and
// source indices (both nullable) move with their columns, so the result is deterministic.
template <int VALT>
__global__ void __launch_bounds__(256) sort_rows_kernel(const int64_t* row_ptr, int64_t d, int32_t* col, void* val,
                                                        int64_t* src) {
  typedef typename std::conditional<VALT == VAL_F64, double,
                                    typename std::conditional<VALT == VAL_F32, float, uint16_t>::type>::type T;
  T* v = static_cast<T*>(val);
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < d; r += (int64_t)gridDim.x * 256) {
    const int64_t s = row_ptr[r], e = row_ptr[r + 1];
    for (int64_t i = s + 1; i < e; ++i) {  // insertion sort: rows are short
      const int32_t kc = col[i];
      const T kv = v ? v[i] : T(0);
      const int64_t ks = src ? src[i] : 0;
      int64_t j = i - 1;
      while (j >= s && col[j] > kc) {
        col[j + 1] = col[j];
        if (v) v[j + 1] = v[j];
        if (src) src[j + 1] = src[j];
        --j;
      }
      col[j + 1] = kc;
      if (v) v[j + 1] = kv;
      if (src) src[j + 1] = ks;
    }
  }
}

template <typename TA, typename TO>
__global__ void __launch_bounds__(256) scale_kernel(const TA* a, int64_t n, double scale, TO* out) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256)
    out[t] = (TO)((double)a[t] * scale);
}

// out[r, j] = cv v_j[r] + cw W[r, j] + cwm Wm[r, j] + cwp Wp[r, j] (W, Wm, Wp nullable).  A thread
// takes N consecutive probes of one row (N divides M and 64, so they share one hash word); the
// (row, group) index advances by a fixed stride, so no division runs inside the loop.
template <typename VT, int N>
__global__ void __launch_bounds__(256) seed_kernel(VT* out, const VT* W, const VT* Wm, const VT* Wp, double cv,
                                                   double cw, double cwm, double cwp, uint64_t seed, int64_t d,
                                                   int M) {
  const int groups = M / N;
  const int64_t total = d * (int64_t)groups;
  const int64_t stride = (int64_t)gridDim.x * 256;
  int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t r = x / groups;
  int g = (int)(x - r * groups);
  const int64_t step_r = stride / groups;
  const int step_g = (int)(stride - step_r * groups);
  for (; x < total; x += stride) {
    const int j0 = g * N;
    const int64_t off = r * M + j0;
    VT o[N], t[N];
    probe_signs<VT, N>(seed, r, j0, o);
#pragma unroll
    for (int i = 0; i < N; ++i) o[i] *= (VT)cv;
    if (W) {
      vload_nt<VT, N>(W + off, t);
#pragma unroll
      for (int i = 0; i < N; ++i) o[i] = fma((VT)cw, t[i], o[i]);
    }
    if (Wm) {
      vload_nt<VT, N>(Wm + off, t);
#pragma unroll
      for (int i = 0; i < N; ++i) o[i] = fma((VT)cwm, t[i], o[i]);
    }
    if (Wp) {
      vload_nt<VT, N>(Wp + off, t);
#pragma unroll
      for (int i = 0; i < N; ++i) o[i] = fma((VT)cwp, t[i], o[i]);
    }
    vstore_nt<VT, N>(out + off, o);
    r += step_r;
    g += step_g;
    if (g >= groups) {
      g -= groups;
      ++r;
    }
  }
}

// Streaming copy: each workgroup moves 1024 16-byte vectors per pass, four per thread at
// a 4 KB spacing, all four loads issued before the stores, non-temporal on both sides.
__global__ void __launch_bounds__(256) copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4* s = reinterpret_cast<const u32x4*>(src);
  u32x4* d = reinterpret_cast<u32x4*>(dst);
  const int64_t stride = (int64_t)gridDim.x * 1024;
  for (int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x; base < n16; base += stride) {
    u32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (base + u * 256 < n16) v[u] = __builtin_nontemporal_load(s + base + u * 256);
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (base + u * 256 < n16) __builtin_nontemporal_store(v[u], d + base + u * 256);
  }
}

__global__ void __launch_bounds__(256) copy_tail_kernel(const uint8_t* src, uint8_t* dst, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) dst[t] = src[t];
}

__global__ void __launch_bounds__(256) zero_kernel(uint4* p, int64_t n16) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n16; t += (int64_t)gridDim.x * 256)
    p[t] = make_uint4(0, 0, 0, 0);
}

__global__ void __launch_bounds__(256) zero_tail_kernel(uint8_t* p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)gridDim.x * 256) p[t] = 0;
}

// ------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------

static unsigned grid_for(int64_t work, int per_block, unsigned cap = 65536u) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

// A plane-major order needs whole planes of a multiple of 8 tiles (then every block maps to
// one tile of [0, ntiles) and every tile to one block); single-matrix launches only.
static bool plane_fits(int64_t plane, int64_t ntiles) {
  return plane == 0 || (plane > 0 && plane % 8 == 0 && ntiles % plane == 0);
}

template <typename VT, int VALT, int VPL, int GSRC, int DSRC, int PSRC, int MU>
static hipError_t go_step(const StepLaunch& L, hipStream_t s) {
  if (!plane_fits(L.shape.plane, L.ntiles) || (L.shape.plane && (L.descs || L.tile_row0)))
    return hipErrorInvalidValue;
  const int64_t per = (L.ntiles + 7) / 8;
  dim3 grid((unsigned)(per * 8), (unsigned)L.shape.probe_tiles);
  hipLaunchKernelGGL((step_kernel<VT, VALT, VPL, GSRC, DSRC, PSRC, MU>), grid, dim3(kBlock), 0, s, L);
  return hipGetLastError();
}

template <typename VT, int VALT, int VPL>
static hipError_t step_by_src(const StepLaunch& L, int g, int d, int p, int mu, hipStream_t s) {
#define LD_CASE(G_, D_, P_, MU_) \
  if (g == G_ && d == D_ && p == P_ && mu == MU_) return go_step<VT, VALT, VPL, G_, D_, P_, MU_>(L, s);
  // Algorithm 1 forward: k = 0, k = 1, k >= 2 (MU_NONE: recomputation; MU_PAIR: product identities)
  LD_CASE(SRC_HASH, SRC_SAME, SRC_NONE, MU_PROBE)
  LD_CASE(SRC_BUF, SRC_SAME, SRC_HASH, MU_PROBE)
  LD_CASE(SRC_BUF, SRC_SAME, SRC_BUF, MU_PROBE)
  LD_CASE(SRC_HASH, SRC_SAME, SRC_NONE, MU_PAIR)
  LD_CASE(SRC_BUF, SRC_SAME, SRC_HASH, MU_PAIR)
  LD_CASE(SRC_BUF, SRC_SAME, SRC_BUF, MU_PAIR)
  LD_CASE(SRC_HASH, SRC_SAME, SRC_NONE, MU_NONE)
  LD_CASE(SRC_BUF, SRC_SAME, SRC_HASH, MU_NONE)
  LD_CASE(SRC_BUF, SRC_SAME, SRC_BUF, MU_NONE)
  // plain product (B + shift I) x, for the Lanczos estimate of the spectrum
  LD_CASE(SRC_BUF, SRC_SAME, SRC_NONE, MU_NONE)
  // Algorithm 2: T = C X, then W_{k+1} = alpha C^T T + beta W_k - W_{k-1}
  LD_CASE(SRC_HASH, SRC_NONE, SRC_NONE, MU_NONE)
  LD_CASE(SRC_BUF, SRC_NONE, SRC_NONE, MU_NONE)
  LD_CASE(SRC_BUF, SRC_HASH, SRC_NONE, MU_PROBE)
  LD_CASE(SRC_BUF, SRC_BUF, SRC_HASH, MU_PROBE)
  LD_CASE(SRC_BUF, SRC_BUF, SRC_BUF, MU_PROBE)
  LD_CASE(SRC_BUF, SRC_HASH, SRC_NONE, MU_PAIR)
  LD_CASE(SRC_BUF, SRC_BUF, SRC_HASH, MU_PAIR)
  LD_CASE(SRC_BUF, SRC_BUF, SRC_BUF, MU_PAIR)
#undef LD_CASE
  return hipErrorInvalidValue;
}

template <typename VT, int VALT>
static hipError_t step_by_vpl(const StepLaunch& L, int g, int d, int p, int mu, hipStream_t s) {
  switch (L.shape.vpl) {
    case 1: return step_by_src<VT, VALT, 1>(L, g, d, p, mu, s);
    case 2: return step_by_src<VT, VALT, 2>(L, g, d, p, mu, s);
    case 4:
      if constexpr (sizeof(VT) == 4) return step_by_src<VT, VALT, 4>(L, g, d, p, mu, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step(const StepLaunch& L, int vec_f64, int valt, int gsrc, int dsrc, int psrc, int mu,
                       hipStream_t s) {
  if (L.ntiles <= 0) return hipSuccess;
  if (vec_f64) {
    if (valt == VAL_F64) return step_by_vpl<double, VAL_F64>(L, gsrc, dsrc, psrc, mu, s);
    if (valt == VAL_F32) return step_by_vpl<double, VAL_F32>(L, gsrc, dsrc, psrc, mu, s);
    if (valt == VAL_BF16) return step_by_vpl<double, VAL_BF16>(L, gsrc, dsrc, psrc, mu, s);
  } else {
    if (valt == VAL_F64) return step_by_vpl<float, VAL_F64>(L, gsrc, dsrc, psrc, mu, s);
    if (valt == VAL_F32) return step_by_vpl<float, VAL_F32>(L, gsrc, dsrc, psrc, mu, s);
    if (valt == VAL_BF16) return step_by_vpl<float, VAL_BF16>(L, gsrc, dsrc, psrc, mu, s);
  }
  return hipErrorInvalidValue;
}

template <typename VT, int VALT, int VPL>
static hipError_t adj_by_flags(const AdjDesc& A, int M, const Shape& sh, bool spmm, bool wh, bool y2, bool sym,
                               hipStream_t s) {
  const int64_t ntiles = (A.d + sh.tile_rows - 1) / sh.tile_rows;
  if (!plane_fits(sh.plane, ntiles)) return hipErrorInvalidValue;
  const int64_t per = (ntiles + 7) / 8;
  dim3 grid((unsigned)(per * 8));
#define LD_ADJ(S_, W_, Y_, X_)                                                                                    \
  if (spmm == S_ && wh == W_ && y2 == Y_ && sym == X_) {                                                         \
    hipLaunchKernelGGL((adjoint_kernel<VT, VALT, VPL, S_, W_, Y_, X_>), grid, dim3(kBlock), 0, s, A, M,          \
                       sh.lpr_log2, (int64_t)sh.tile_rows, ntiles, (int64_t)sh.plane);                          \
    return hipGetLastError();                                                                                   \
  }
  LD_ADJ(true, false, true, false)
  LD_ADJ(true, false, false, false)
  LD_ADJ(false, true, false, false)
  LD_ADJ(true, false, true, true)
  LD_ADJ(true, false, false, true)
  LD_ADJ(false, true, false, true)
#undef LD_ADJ
  return hipErrorInvalidValue;
}

template <typename VT, int VALT>
static hipError_t adj_by_vpl(const AdjDesc& A, int M, const Shape& sh, bool spmm, bool wh, bool y2, bool sym,
                             hipStream_t s) {
  switch (sh.vpl) {
    case 1: return adj_by_flags<VT, VALT, 1>(A, M, sh, spmm, wh, y2, sym, s);
    case 2: return adj_by_flags<VT, VALT, 2>(A, M, sh, spmm, wh, y2, sym, s);
    case 4:
      if constexpr (sizeof(VT) == 4) return adj_by_flags<VT, VALT, 4>(A, M, sh, spmm, wh, y2, sym, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint(const AdjDesc& A, int M, const Shape& sh, int vec_f64, int valt, bool spmm, bool w_hash,
                          bool y2, bool sym, hipStream_t s) {
  if (A.d <= 0) return hipSuccess;
  if (vec_f64) {
    if (valt == VAL_F64) return adj_by_vpl<double, VAL_F64>(A, M, sh, spmm, w_hash, y2, sym, s);
    if (valt == VAL_F32) return adj_by_vpl<double, VAL_F32>(A, M, sh, spmm, w_hash, y2, sym, s);
    if (valt == VAL_BF16) return adj_by_vpl<double, VAL_BF16>(A, M, sh, spmm, w_hash, y2, sym, s);
  } else {
    if (valt == VAL_F64) return adj_by_vpl<float, VAL_F64>(A, M, sh, spmm, w_hash, y2, sym, s);
    if (valt == VAL_F32) return adj_by_vpl<float, VAL_F32>(A, M, sh, spmm, w_hash, y2, sym, s);
    if (valt == VAL_BF16) return adj_by_vpl<float, VAL_BF16>(A, M, sh, spmm, w_hash, y2, sym, s);
  }
  return hipErrorInvalidValue;
}

template <typename VT, int VALT>
static hipError_t adj_stencil_by_vpl(const AdjDesc& A, const StencilDesc& S, int M, const Shape& sh, bool y2,
                                     bool sddmm, hipStream_t s) {
  const int tr = stencil_tile_rows(sh.lpr_log2);
  const int64_t ntiles = (A.d + tr - 1) / tr;
  const int64_t per = (ntiles + 7) / 8;
  const dim3 grid((unsigned)(per * 8));
  const size_t lds = 2 * (size_t)(tr + S.nofs) * (size_t)((1 << sh.lpr_log2) * sh.vpl) * sizeof(VT);
  if (tr > kStencilRows || lds > (size_t)kStencilLdsBytes || S.nofs > kHaloPasses * tr) return hipErrorInvalidValue;
  if (sddmm) {  // the closing SDDMM: FP32 vectors only (adjoint_stencil_sddmm_supported)
    if constexpr (sizeof(VT) == 4 && VALT != VAL_F64) {
#define LD_STEN_SD(V_, K_)                                                                                       \
  if (sh.vpl == V_ && S.K == K_) {                                                                               \
    hipLaunchKernelGGL((adjoint_stencil_kernel<VT, VALT, V_, false, K_, true>), grid, dim3(kBlock), lds, s, A, S, \
                       M, sh.lpr_log2, ntiles);                                                                 \
    return hipGetLastError();                                                                                   \
  }
      LD_STEN_SD(2, 5) LD_STEN_SD(2, 7) LD_STEN_SD(2, 8)
      LD_STEN_SD(4, 5) LD_STEN_SD(4, 7) LD_STEN_SD(4, 8)
#undef LD_STEN_SD
    }
    return hipErrorInvalidValue;
  }
  // K = 5 and 7 (2-D and 3-D grids) run exactly; other K up to kStencilK are planned as 8
#define LD_STEN(V_, Y_, K_)                                                                                      \
  if (sh.vpl == V_ && y2 == Y_ && S.K == K_) {                                                                   \
    hipLaunchKernelGGL((adjoint_stencil_kernel<VT, VALT, V_, Y_, K_>), grid, dim3(kBlock), lds, s, A, S, M,      \
                       sh.lpr_log2, ntiles);                                                                    \
    return hipGetLastError();                                                                                   \
  }
#define LD_STEN_K(V_, Y_) LD_STEN(V_, Y_, 5) LD_STEN(V_, Y_, 7) LD_STEN(V_, Y_, 8)
  LD_STEN_K(1, true)
  LD_STEN_K(1, false)
  LD_STEN_K(2, true)
  LD_STEN_K(2, false)
  LD_STEN_K(4, true)
  LD_STEN_K(4, false)
#undef LD_STEN_K
#undef LD_STEN
  return hipErrorInvalidValue;
}

hipError_t launch_adjoint_stencil(const AdjDesc& A, const StencilDesc& S, int M, const Shape& sh, int vec_f64,
                                  int valt, bool y2, bool sddmm, hipStream_t s) {
  if (A.d <= 0) return hipSuccess;
  if (sddmm && (y2 || !adjoint_stencil_sddmm_supported(vec_f64, valt, sh, S))) return hipErrorInvalidValue;
  if (vec_f64) {
    if (valt == VAL_F64) return adj_stencil_by_vpl<double, VAL_F64>(A, S, M, sh, y2, sddmm, s);
    if (valt == VAL_F32) return adj_stencil_by_vpl<double, VAL_F32>(A, S, M, sh, y2, sddmm, s);
    if (valt == VAL_BF16) return adj_stencil_by_vpl<double, VAL_BF16>(A, S, M, sh, y2, sddmm, s);
  } else {
    if (valt == VAL_F64) return adj_stencil_by_vpl<float, VAL_F64>(A, S, M, sh, y2, sddmm, s);
    if (valt == VAL_F32) return adj_stencil_by_vpl<float, VAL_F32>(A, S, M, sh, y2, sddmm, s);
    if (valt == VAL_BF16) return adj_stencil_by_vpl<float, VAL_BF16>(A, S, M, sh, y2, sddmm, s);
  }
  return hipErrorInvalidValue;
}

bool adjoint_stencil_sddmm_supported(int vec_f64, int valt, const Shape& sh, const StencilDesc& S) {
  return !vec_f64 && valt != VAL_F64 && (sh.vpl == 2 || sh.vpl == 4) && (S.K == 5 || S.K == 7 || S.K == 8);
}

// Operand sources and moment forms the staged step is built for: the product-identity forward (k = 0
// from the hash, k = 1 with the hash as W_{k-1}, then buffers), its recomputation without moments,
// the plain recurrence's probe moments, and the plain product with probe moments (Taylor series).
static bool stencil_combo(int g, int p, int mu) {
  if (g == SRC_HASH) return p == SRC_NONE && (mu == MU_PAIR || mu == MU_NONE || mu == MU_PROBE);
  if (g != SRC_BUF) return false;
  if (p == SRC_BUF || p == SRC_HASH) return mu == MU_PAIR || mu == MU_NONE || mu == MU_PROBE;
  return p == SRC_NONE && mu == MU_PROBE;
}

template <int VALT, int VPL>
static hipError_t step_stencil_by_flags(const StepLaunch& L, const StencilDesc& S, int gsrc, int psrc, int mu,
                                        size_t lds, dim3 grid, hipStream_t s) {
#define LD_SS(G_, P_, MU_, K_)                                                                                   \
  if (gsrc == G_ && psrc == P_ && mu == MU_ && S.K == K_) {                                                     \
    hipLaunchKernelGGL((step_stencil_kernel<VALT, VPL, G_, P_, MU_, K_>), grid, dim3(kBlock), lds, s, L, S);   \
    return hipGetLastError();                                                                                   \
  }
#define LD_SS_K(G_, P_, MU_) LD_SS(G_, P_, MU_, 5) LD_SS(G_, P_, MU_, 7) LD_SS(G_, P_, MU_, 8)
  LD_SS_K(SRC_BUF, SRC_BUF, MU_PAIR)
  LD_SS_K(SRC_BUF, SRC_HASH, MU_PAIR)
  LD_SS_K(SRC_HASH, SRC_NONE, MU_PAIR)
  LD_SS_K(SRC_BUF, SRC_BUF, MU_NONE)
  LD_SS_K(SRC_BUF, SRC_HASH, MU_NONE)
  LD_SS_K(SRC_HASH, SRC_NONE, MU_NONE)
  LD_SS_K(SRC_BUF, SRC_BUF, MU_PROBE)
  LD_SS_K(SRC_BUF, SRC_HASH, MU_PROBE)
  LD_SS_K(SRC_HASH, SRC_NONE, MU_PROBE)
  LD_SS_K(SRC_BUF, SRC_NONE, MU_PROBE)
#undef LD_SS_K
#undef LD_SS
  return hipErrorInvalidValue;
}

bool step_stencil_supported(const StepLaunch& L, int vec_f64, int valt, int gsrc, int dsrc, int psrc, int mu) {
  return !vec_f64 && valt != VAL_F64 && dsrc == SRC_SAME && stencil_combo(gsrc, psrc, mu) && L.descs == nullptr &&
         L.shape.probe_tiles == 1 && (L.shape.vpl == 2 || L.shape.vpl == 4) &&
         L.tile_rows % stencil_tile_rows(L.shape.lpr_log2) == 0 && stencil_tile_rows(L.shape.lpr_log2) <= kStencilRows;
}

hipError_t launch_step_stencil(const StepLaunch& L, const StencilDesc& S, int valt, int gsrc, int psrc, int mu,
                               hipStream_t s) {
  if (L.ntiles <= 0) return hipSuccess;
  const int tr = stencil_tile_rows(L.shape.lpr_log2);
  const size_t tp = (size_t)(1 << L.shape.lpr_log2) * L.shape.vpl;
  const size_t lds = std::max((size_t)(tr + S.nofs) * tp * sizeof(float),
                              (size_t)(mu == MU_PAIR ? 2 : mu == MU_PROBE ? 1 : 0) * kWaves * 256 * sizeof(double));
  if (lds > (size_t)kStencilLdsBytes || S.nofs > kHaloPasses * tr) return hipErrorInvalidValue;
  const int64_t per = (L.ntiles + 7) / 8;
  const dim3 grid((unsigned)(per * 8));
  if (valt == VAL_BF16)
    return L.shape.vpl == 4 ? step_stencil_by_flags<VAL_BF16, 4>(L, S, gsrc, psrc, mu, lds, grid, s)
                            : step_stencil_by_flags<VAL_BF16, 2>(L, S, gsrc, psrc, mu, lds, grid, s);
  if (valt == VAL_F32)
    return L.shape.vpl == 4 ? step_stencil_by_flags<VAL_F32, 4>(L, S, gsrc, psrc, mu, lds, grid, s)
                            : step_stencil_by_flags<VAL_F32, 2>(L, S, gsrc, psrc, mu, lds, grid, s);
  return hipErrorInvalidValue;
}

hipError_t launch_stencil_pack(const void* val, int valt, const int32_t* emap, const uint16_t* lcol, int64_t n,
                               void* ent, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = grid_for(n, 256);
  if (valt == VAL_F64)
    hipLaunchKernelGGL(stencil_pack_kernel<VAL_F64>, dim3(g), dim3(256), 0, s, val, emap, lcol, n, ent);
  else if (valt == VAL_F32)
    hipLaunchKernelGGL(stencil_pack_kernel<VAL_F32>, dim3(g), dim3(256), 0, s, val, emap, lcol, n, ent);
  else
    hipLaunchKernelGGL(stencil_pack_kernel<VAL_BF16>, dim3(g), dim3(256), 0, s, val, emap, lcol, n, ent);
  return hipGetLastError();
}

hipError_t launch_stencil_unpack(const void* hacc, int vec_f64, const int32_t* emap, int64_t n, void* acc,
                                 hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = grid_for(n, 256);
  if (vec_f64)
    hipLaunchKernelGGL(stencil_unpack_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)hacc, emap, n,
                       (double*)acc);
  else
    hipLaunchKernelGGL(stencil_unpack_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)hacc, emap, n,
                       (float*)acc);
  return hipGetLastError();
}

hipError_t launch_stencil_diag_sum(const void* hacc, int vec_f64, const int64_t* dslot, int64_t d, double* part,
                                   hipStream_t s) {
  if (d <= 0) return hipSuccess;
  if (vec_f64)
    hipLaunchKernelGGL(stencil_diag_sum_kernel<double>, dim3(256), dim3(256), 0, s, (const double*)hacc, dslot, d, part);
  else
    hipLaunchKernelGGL(stencil_diag_sum_kernel<float>, dim3(256), dim3(256), 0, s, (const float*)hacc, dslot, d, part);
  return hipGetLastError();
}

hipError_t launch_transpose_index(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t nnz, int64_t* perm,
                                  int* missing, hipStream_t s) {
  if (d <= 0 || nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_index_kernel, dim3(grid_for(nnz, 256, 1u << 20)), dim3(256), 0, s, row_ptr, col, d,
                     nnz, perm, missing);
  return hipGetLastError();
}

hipError_t launch_distance_hist(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t nnz,
                                unsigned long long* hist, hipStream_t s) {
  if (d <= 0) return hipSuccess;
  hipLaunchKernelGGL(distance_hist_kernel, dim3(grid_for(d, 256, 8192u)), dim3(256), 0, s, row_ptr, col, d, nnz, hist);
  return hipGetLastError();
}

hipError_t launch_plane_fit(const int64_t* row_ptr, const int32_t* col, int64_t d, int64_t band,
                            unsigned long long* out, hipStream_t s) {
  if (d <= 0) return hipSuccess;
  hipLaunchKernelGGL(plane_fit_kernel, dim3(grid_for(d, 256, 8192u)), dim3(256), 0, s, row_ptr, col, d, band, out);
  return hipGetLastError();
}

hipError_t launch_sym_scale(const void* a, int a_f64, const int64_t* perm, int64_t n, double scale, void* out,
                            int out_f64, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned g = grid_for(n, 256);
  if (a_f64 && out_f64)
    hipLaunchKernelGGL((sym_scale_kernel<double, double>), dim3(g), dim3(256), 0, s, (const double*)a, perm, n, scale,
                       (double*)out);
  else if (a_f64)
    hipLaunchKernelGGL((sym_scale_kernel<double, float>), dim3(g), dim3(256), 0, s, (const double*)a, perm, n, scale,
                       (float*)out);
  else if (out_f64)
    hipLaunchKernelGGL((sym_scale_kernel<float, double>), dim3(g), dim3(256), 0, s, (const float*)a, perm, n, scale,
                       (double*)out);
  else
    hipLaunchKernelGGL((sym_scale_kernel<float, float>), dim3(g), dim3(256), 0, s, (const float*)a, perm, n, scale,
                       (float*)out);
  return hipGetLastError();
}

size_t reduce_scratch_bytes(int nk, int M) { return (size_t)std::max(nk, 1) * kRedChunks * M * sizeof(double); }

hipError_t launch_reduce_moments(const double* part, int64_t ntiles, int M, int k_lo, int k_hi, int64_t kstride,
                                 double* mu, int ldmu, double* tmp, hipStream_t s) {
  if (k_hi < k_lo) return hipSuccess;
  const int nk = k_hi - k_lo + 1;
  dim3 grid((unsigned)nk, (unsigned)((M + 63) / 64), (unsigned)kRedChunks);
  hipLaunchKernelGGL(reduce_moments_stage1, grid, dim3(1024), 0, s, part, ntiles, M, kstride, tmp);
  hipLaunchKernelGGL(reduce_moments_stage2, dim3(grid_for((int64_t)nk * M, 256)), dim3(256), 0, s, tmp, M, k_lo, nk,
                     mu, ldmu);
  return hipGetLastError();
}

hipError_t launch_reduce_batched(const double* part, const int64_t* tile_range, const int* n, int count, int M,
                                 int kmax, int64_t kstride, double* mu, hipStream_t s) {
  if (count <= 0 || kmax < 1) return hipSuccess;
  dim3 grid((unsigned)count, (unsigned)kmax, (unsigned)((M + 63) / 64));
  hipLaunchKernelGGL(reduce_batched_kernel, grid, dim3(1024), 0, s, part, tile_range, n, M, kstride, mu, kmax);
  return hipGetLastError();
}

hipError_t launch_sum_doubles(const double* x, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_doubles_kernel, dim3(1), dim3(1024), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_gershgorin(const int64_t* row_ptr, const int32_t* col, const void* val, int valt, double shift,
                             int64_t d, double* lo_part, double* hi_part, int nblocks, hipStream_t s) {
  dim3 grid((unsigned)nblocks);
  if (valt == VAL_F64)
    hipLaunchKernelGGL(gershgorin_kernel<VAL_F64>, grid, dim3(256), 0, s, row_ptr, col, val, shift, d, lo_part, hi_part);
  else if (valt == VAL_F32)
    hipLaunchKernelGGL(gershgorin_kernel<VAL_F32>, grid, dim3(256), 0, s, row_ptr, col, val, shift, d, lo_part, hi_part);
  else
    hipLaunchKernelGGL(gershgorin_kernel<VAL_BF16>, grid, dim3(256), 0, s, row_ptr, col, val, shift, d, lo_part,
                       hi_part);
  return hipGetLastError();
}

constexpr int kDotBlocks = 512;

hipError_t launch_dot(const double* x, const double* y, int64_t n, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(dot_partials_kernel, dim3(kDotBlocks), dim3(256), 0, s, x, y, n, part);
  hipLaunchKernelGGL(sum_doubles_kernel, dim3(1), dim3(1024), 0, s, part, (int64_t)kDotBlocks, out);
  return hipGetLastError();
}

hipError_t launch_probes(uint64_t seed, int M, int64_t rows, int8_t* out, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(probes_kernel, dim3(grid_for(rows * (int64_t)M, 256)), dim3(256), 0, s, seed, M, rows, out);
  return hipGetLastError();
}

size_t transpose_scratch_bytes(int64_t d) {
  const int64_t n = d + 1;
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  return (size_t)(n + nt + 8) * sizeof(int64_t);
}

hipError_t launch_transpose(const int64_t* row_ptr, const int32_t* col, const void* val, int valt, int64_t d,
                            int64_t nnz, int64_t* row_ptr_t, int32_t* col_t, void* val_t, int64_t* cursor,
                            void* scan_tmp, size_t scan_tmp_bytes, hipStream_t s, int64_t* src_t) {
  const int64_t n = d + 1;
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  if (scan_tmp_bytes < transpose_scratch_bytes(d)) return hipErrorInvalidValue;
  int64_t* cnt = static_cast<int64_t*>(scan_tmp);
  int64_t* sums = cnt + n;
  hipError_t e = launch_fill_zero(cnt, (size_t)n * sizeof(int64_t), s);
  if (e != hipSuccess) return e;
  if (nnz > 0) hipLaunchKernelGGL(count_cols_kernel, dim3(grid_for(nnz, 256)), dim3(256), 0, s, col, nnz, cnt);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3((unsigned)nt), dim3(kScanBlock), 0, s, cnt, n, row_ptr_t, sums);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, s, sums, nt);
  hipLaunchKernelGGL(scan_add_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, row_ptr_t, n, sums);
  e = hipMemcpyAsync(cursor, row_ptr_t, (size_t)d * sizeof(int64_t), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return e;
  const unsigned g = grid_for(d, 256);
  if (valt == VAL_F64) {
    hipLaunchKernelGGL(scatter_t_kernel<VAL_F64>, dim3(g), dim3(256), 0, s, row_ptr, col, val, d, cursor, col_t, val_t,
                       src_t);
    hipLaunchKernelGGL(sort_rows_kernel<VAL_F64>, dim3(g), dim3(256), 0, s, row_ptr_t, d, col_t, val_t, src_t);
  } else if (valt == VAL_F32) {
    hipLaunchKernelGGL(scatter_t_kernel<VAL_F32>, dim3(g), dim3(256), 0, s, row_ptr, col, val, d, cursor, col_t, val_t,
                       src_t);
    hipLaunchKernelGGL(sort_rows_kernel<VAL_F32>, dim3(g), dim3(256), 0, s, row_ptr_t, d, col_t, val_t, src_t);
  } else {
    hipLaunchKernelGGL(scatter_t_kernel<VAL_BF16>, dim3(g), dim3(256), 0, s, row_ptr, col, val, d, cursor, col_t,
                       val_t, src_t);
    hipLaunchKernelGGL(sort_rows_kernel<VAL_BF16>, dim3(g), dim3(256), 0, s, row_ptr_t, d, col_t, val_t, src_t);
  }
  return hipGetLastError();
}

hipError_t launch_scale_grad(const void* Gacc, int acc_f64, int64_t nnz, double scale, void* out, int out_f64,
                             hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  const unsigned g = grid_for(nnz, 256);
  if (acc_f64 && out_f64)
    hipLaunchKernelGGL((scale_kernel<double, double>), dim3(g), dim3(256), 0, s, (const double*)Gacc, nnz, scale,
                       (double*)out);
  else if (acc_f64)
    hipLaunchKernelGGL((scale_kernel<double, float>), dim3(g), dim3(256), 0, s, (const double*)Gacc, nnz, scale,
                       (float*)out);
  else if (out_f64)
    hipLaunchKernelGGL((scale_kernel<float, double>), dim3(g), dim3(256), 0, s, (const float*)Gacc, nnz, scale,
                       (double*)out);
  else
    hipLaunchKernelGGL((scale_kernel<float, float>), dim3(g), dim3(256), 0, s, (const float*)Gacc, nnz, scale,
                       (float*)out);
  return hipGetLastError();
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 > 0)
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n16, 1024, 1u << 16)), dim3(256), 0, s,
                       static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  const int64_t tail = (int64_t)(bytes - (size_t)n16 * 16);
  if (tail > 0)
    hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(256), 0, s, static_cast<const uint8_t*>(src) + n16 * 16,
                       static_cast<uint8_t*>(dst) + n16 * 16, tail);
  return hipGetLastError();
}

template <typename VT, int N>
static void go_seed(void* out, const void* W, const void* Wm, const void* Wp, double cv, double cw, double cwm,
                    double cwp, uint64_t seed, int64_t d, int M, hipStream_t s) {
  const unsigned g = grid_for(d * (int64_t)(M / N), 256, 1u << 20);
  hipLaunchKernelGGL((seed_kernel<VT, N>), dim3(g), dim3(256), 0, s, static_cast<VT*>(out),
                     static_cast<const VT*>(W), static_cast<const VT*>(Wm), static_cast<const VT*>(Wp), cv, cw, cwm,
                     cwp, seed, d, M);
}

hipError_t launch_seed(void* out, int vec_f64, const void* W, const void* Wm, const void* Wp, double cv, double cw,
                       double cwm, double cwp, uint64_t seed, int64_t d, int M, hipStream_t s) {
  if (d <= 0) return hipSuccess;
  if (vec_f64) {
    if (M % 2 == 0)
      go_seed<double, 2>(out, W, Wm, Wp, cv, cw, cwm, cwp, seed, d, M, s);
    else
      go_seed<double, 1>(out, W, Wm, Wp, cv, cw, cwm, cwp, seed, d, M, s);
  } else {
    if (M % 4 == 0)
      go_seed<float, 4>(out, W, Wm, Wp, cv, cw, cwm, cwp, seed, d, M, s);
    else if (M % 2 == 0)
      go_seed<float, 2>(out, W, Wm, Wp, cv, cw, cwm, cwp, seed, d, M, s);
    else
      go_seed<float, 1>(out, W, Wm, Wp, cv, cw, cwm, cwp, seed, d, M, s);
  }
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 > 0)
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n16, 256, 1u << 20)), dim3(256), 0, s, static_cast<uint4*>(p), n16);
  const int64_t tail = (int64_t)(bytes - (size_t)n16 * 16);
  if (tail > 0)
    hipLaunchKernelGGL(zero_tail_kernel, dim3(1), dim3(256), 0, s, static_cast<uint8_t*>(p) + n16 * 16, tail);
  return hipGetLastError();
}

}  // namespace ld
